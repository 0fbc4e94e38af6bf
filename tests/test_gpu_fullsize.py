"""Parity at the benchmark sizes, in the launch configuration the benchmark
times: sampled sites against the oracle's dependency-cone evaluation after a
few steps, and properties that hold at any size (bitwise identity of all four
propagation variants, mass conservation over many steps)."""
import numpy as np
import pytest

from lbm_inputs import init_fields, workload
from oracle import dense
from tests.gpu_util import solver_for, node_fields, VARIANTS

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pack():
    mask, p = workload("spherepack-512x128x128", seed=0)
    return mask, p


def test_spherepack_sampled_sites(pack):
    mask, p = pack
    steps = 3
    rho0, u0 = init_fields(mask.shape, seed=11)
    fl = np.argwhere(mask == 0)
    sites = fl[np.random.default_rng(12).choice(len(fl), 48, replace=False)]
    # add sites touching the walls and the periodic seam
    extra = fl[(fl[:, 0] == 0) | (fl[:, 1] == 0) | (fl[:, 2] == mask.shape[2] - 1)]
    sites = np.concatenate([sites, extra[np.random.default_rng(13).choice(len(extra), 16, replace=False)]])
    want = dense.cone_sites(mask.astype(bool), p["periodic"], p["tau"], p["force"], steps, rho0, u0, sites)
    vox = (sites[:, 0] * mask.shape[1] + sites[:, 1]) * mask.shape[2] + sites[:, 2]
    for pattern, ria in VARIANTS:
        print("case spherepack sampled", pattern, ria, flush=True)
        lat, s = solver_for(mask, p["periodic"], p["tau"], p["force"], pattern, ria, p["order"], p["block"])
        r, v = node_fields(lat, rho0, u0)
        s.init(torch.from_numpy(r).cuda(), torch.from_numpy(v).cuda())
        s.step(steps)
        f = s.export_pdfs().cpu().numpy()
        node_of = np.full(mask.size, -1, np.int64)
        node_of[lat.node_voxel().astype(np.int64)] = np.arange(lat.n_fluid)
        got = f[:, node_of[vox]].T
        assert np.array_equal(got, want), (pattern, ria)
        del s


def test_spherepack_variants_identical_and_conserve_mass(pack):
    mask, p = pack
    steps = 200
    results = []
    for pattern, ria in VARIANTS:
        print("case spherepack variants", pattern, ria, flush=True)
        lat, s = solver_for(mask, p["periodic"], p["tau"], p["force"], pattern, ria, p["order"], p["block"])
        s.init()
        _, _, t0 = s.moments()
        s.step(steps)
        rho, u, t1 = s.moments()
        m0, m1 = t0[0].item(), t1[0].item()
        assert abs(m1 - m0) / m0 < 1e-12
        # momentum grows by at most N*F per step (walls take some)
        assert 0 < t1[1].item() <= steps * lat.n_fluid * p["force"][0] * (1 + 1e-9)
        results.append(u.cpu().numpy())
        del s
    for r in results[1:]:
        assert np.array_equal(r, results[0])


@pytest.mark.parametrize("order,block,ria", [("lex", 0, True), ("lex", 8, "direction"), ("morton", 0, True),
                                             ("hilbert_ls", 8, True)])
def test_foam384_sampled_sites(order, block, ria):
    # the 384^3 foam of the enumeration sweep and the precision study
    mask, p = workload("foam-384", seed=0)
    steps = 2
    rho0, u0 = init_fields(mask.shape, seed=21)
    fl = np.flatnonzero(mask.reshape(-1) == 0)
    pick = fl[np.random.default_rng(22).choice(len(fl), 24, replace=False)]
    sites = np.stack(np.unravel_index(pick, mask.shape), 1)
    want = dense.cone_sites(mask.astype(bool), p["periodic"], p["tau"], p["force"], steps, rho0, u0, sites)
    print("case foam-384 sampled", order, block, ria, flush=True)
    lat, s = solver_for(mask, p["periodic"], p["tau"], p["force"], "aa", ria, order, block)
    r, v = node_fields(lat, rho0, u0)
    del rho0, u0
    s.init(torch.from_numpy(r).cuda(), torch.from_numpy(v).cuda())
    s.step(steps)
    f = s.export_pdfs()
    node_of = np.full(mask.size, -1, np.int64)
    node_of[lat.node_voxel().astype(np.int64)] = np.arange(lat.n_fluid)
    idx = torch.from_numpy(node_of[pick]).cuda()
    got = f[:, idx].T.cpu().numpy()
    assert np.array_equal(got, want)
