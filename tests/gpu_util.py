"""Helpers shared by the GPU tests: run the HIP path and map node-ordered
results to voxel order for comparison with the oracle."""
import numpy as np


def solver_for(mask, periodic, tau, force, pattern, ria, order="lex", block=0, **kw):
    from paper_1410_0412_amd import Lattice, Solver
    lat = Lattice(mask, periodic, order, block)
    return lat, Solver(lat, tau, force, pattern=pattern, ria=ria, **kw)


def node_fields(lat, rho_vox, u_vox):
    """Voxel-ordered seeded fields -> node-ordered arrays (N,), (3, N)."""
    nv = lat.node_voxel().astype(np.int64)
    return rho_vox.reshape(-1)[nv], u_vox.reshape(3, -1)[:, nv]


def oracle_at_nodes(lat, f_dense):
    """(19, N) PDFs of the dense oracle at the lattice's nodes."""
    nv = lat.node_voxel().astype(np.int64)
    return f_dense.reshape(19, -1)[:, nv]


def normwise_u_error(u_gpu, u_ref):
    """max_n |u_gpu(n) - u_ref(n)|_2 / max_n |u_ref(n)|_2."""
    d = np.sqrt(((u_gpu - u_ref) ** 2).sum(0)).max()
    return d / np.sqrt((u_ref ** 2).sum(0)).max()


#: (pattern, index source): adjacency list, the paper's runs, per-direction runs
VARIANTS = [("aa", False), ("aa", True), ("aa", "direction"),
            ("osnt", False), ("osnt", True), ("osnt", "direction")]
