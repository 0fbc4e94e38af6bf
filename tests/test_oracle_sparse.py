"""The oracle's sparse AA / OS-NT executors must equal the dense solver
bitwise at every step, for every enumeration (Sect. 4: the propagation
patterns and the enumeration change addressing only, never arithmetic)."""
import numpy as np
import pytest

from lbm_inputs import rsa_spheres, init_fields
from oracle import dense, sparse, tables

PERIODIC = (True, False, True)
TAU, F = 0.7, (1e-5, -2e-6, 3e-6)


@pytest.fixture(scope="module")
def case():
    mask = rsa_spheres((10, 9, 8), 2.0, 0.25, PERIODIC, seed=21)
    rho, u = init_fields(mask.shape, seed=22)
    solid = mask.astype(bool)
    traj = [dense.initial_state(solid, rho, u)]
    for _ in range(6):
        traj.append(dense.step(traj[-1], solid, PERIODIC, TAU, F))
    return mask, traj


def natural(f_dense, nodes, shape):
    flat = f_dense.reshape(19, -1)
    return flat[:, nodes.astype(np.int64)]


@pytest.mark.parametrize("order,block", [("lex", 0), ("lex", 3), ("morton", 0)])
def test_aa_equals_dense(case, order, block):
    mask, traj = case
    t = tables.build(mask, PERIODIC, order, block)
    nodes, adj = t["node_voxel"], t["adj"]
    ldf = len(nodes) + 5
    Fg = np.zeros((19, ldf))
    Fg[:, :len(nodes)] = natural(traj[0], nodes, mask.shape)
    for s in range(6):
        if s % 2 == 0:
            sparse.aa_even(Fg, len(nodes), TAU, F)
        else:
            sparse.aa_odd(Fg, adj, TAU, F)
        assert np.array_equal(sparse.aa_pdfs(Fg, adj, s + 1), natural(traj[s + 1], nodes, mask.shape))


@pytest.mark.parametrize("order,block", [("lex", 0), ("morton", 0)])
def test_osnt_equals_dense(case, order, block):
    mask, traj = case
    t = tables.build(mask, PERIODIC, order, block)
    nodes, adj = t["node_voxel"], t["adj"]
    G = sparse.osnt_from_pdfs(natural(traj[0], nodes, mask.shape), adj)
    assert np.array_equal(sparse.osnt_pdfs(G, adj), natural(traj[0], nodes, mask.shape))
    H = np.zeros_like(G)
    for s in range(6):
        sparse.osnt(G, H, adj, TAU, F)
        G, H = H, G
        assert np.array_equal(sparse.osnt_pdfs(G, adj), natural(traj[s + 1], nodes, mask.shape))
