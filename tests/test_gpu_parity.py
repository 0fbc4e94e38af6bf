"""GPU parity: the HIP path against the FP64 oracle, through the C ABI.

FP64 kernels evaluate the collision in the oracle's order without
contraction, so results are expected to be bitwise identical; the stated
bound is the normwise relative velocity error 1e-12 after 100 steps.
"""
import numpy as np
import pytest

from lbm_inputs import rsa_spheres, init_fields, channel_mask, relaxed_spheres, workload
from oracle import dense
from tests.gpu_util import solver_for, node_fields, oracle_at_nodes, normwise_u_error, VARIANTS

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

PER = (True, False, False)


@pytest.fixture(scope="module")
def spheres32():
    mask, p = workload("spheres-32", seed=0)
    f = dense.run(mask.astype(bool), p["periodic"], p["tau"], p["force"], p["steps"])
    rho, u = dense.macroscopic(f)
    return mask, p, f, rho, u


@pytest.mark.parametrize("pattern,ria", VARIANTS)
def test_spheres32_100_steps(spheres32, pattern, ria):
    mask, p, f_ref, rho_ref, u_ref = spheres32
    print("case spheres-32", pattern, ria, flush=True)
    lat, s = solver_for(mask, p["periodic"], p["tau"], p["force"], pattern, ria)
    s.init()
    s.step(p["steps"])
    rho, u, tot = s.moments()
    nv = lat.node_voxel().astype(np.int64)
    ur = np.stack([u_ref[a].reshape(-1)[nv] for a in range(3)])
    err = normwise_u_error(u.cpu().numpy(), ur)
    assert err <= 1e-12, err
    # exact: same IEEE operations in the same order
    assert np.array_equal(u.cpu().numpy(), ur)
    assert np.array_equal(rho.cpu().numpy(), rho_ref.reshape(-1)[nv])
    assert np.array_equal(s.export_pdfs().cpu().numpy(), oracle_at_nodes(lat, f_ref))
    mass_ref = rho_ref.reshape(-1)[nv].sum()
    assert abs(tot[0].item() - mass_ref) / mass_ref < 1e-13


@pytest.mark.parametrize("pattern,ria", VARIANTS)
@pytest.mark.parametrize("order,block", [("lex", 0), ("lex", 4), ("morton", 0), ("hilbert", 0), ("hilbert_ls", 3)])
def test_every_step_random_state(pattern, ria, order, block):
    # non-trivial seeded initial state; all PDFs compared after every step, so
    # both AA parities and every slot of the layouts are exercised
    mask = rsa_spheres((20, 18, 22), 2.5, 0.25, PER, seed=5)
    rho0, u0 = init_fields(mask.shape, seed=6)
    tau, F = 0.65, (2e-5, -1e-5, 5e-6)
    print("case random-state", pattern, ria, order, block, flush=True)
    lat, s = solver_for(mask, PER, tau, F, pattern, ria, order, block)
    r, v = node_fields(lat, rho0, u0)
    s.init(torch.from_numpy(r).cuda(), torch.from_numpy(v).cuda())
    f = dense.initial_state(mask.astype(bool), rho0, u0)
    assert np.array_equal(s.export_pdfs().cpu().numpy(), oracle_at_nodes(lat, f))
    for t in range(1, 8):
        s.step(1)
        f = dense.step(f, mask.astype(bool), PER, tau, F)
        assert s.t == t
        assert np.array_equal(s.export_pdfs().cpu().numpy(), oracle_at_nodes(lat, f)), t


@pytest.mark.parametrize("pattern,ria", VARIANTS)
@pytest.mark.parametrize("prec,trt", [("f64", None), ("f64", 0.1875), ("f32", None), ("f32", 0.1875), ("f16", None)])
def test_wide_slots_every_step(pattern, ria, prec, trt):
    # the step kernels with 64-bit slot offsets (the form grids of more than
    # 2^31 - 1 elements take) against the 32-bit form after every step, bit
    # for bit, in every precision and with both collisions; FP64 against the
    # oracle too
    mask = rsa_spheres((20, 18, 22), 2.5, 0.25, PER, seed=5)
    rho0, u0 = init_fields(mask.shape, seed=6)
    tau, F = 0.65, (2e-5, -1e-5, 5e-6)
    print("case wide slots", pattern, ria, prec, trt, flush=True)
    lat, a = solver_for(mask, PER, tau, F, pattern, ria, precision=prec, trt_magic=trt, wide_slots=True)
    _, b = solver_for(mask, PER, tau, F, pattern, ria, precision=prec, trt_magic=trt)
    r, v = node_fields(lat, rho0, u0)
    r, v = torch.from_numpy(r).cuda(), torch.from_numpy(v).cuda()
    a.init(r, v)
    b.init(r, v)
    f = dense.initial_state(mask.astype(bool), rho0, u0)
    for t in range(1, 8):
        a.step(1)
        b.step(1)
        fa = a.export_pdfs()
        assert torch.equal(fa, b.export_pdfs()), t
        if prec == "f64":
            f = dense.step(f, mask.astype(bool), PER, tau, F, trt)
            assert np.array_equal(fa.cpu().numpy(), oracle_at_nodes(lat, f)), t


@pytest.mark.parametrize("ria", [False, True, "direction"])
@pytest.mark.parametrize("prec,trt,rows", [("f64", None, 8), ("f64", None, 16), ("f64", 0.1875, 8),
                                           ("f32", None, 8), ("f16", None, 16)])
def test_band_schedule_every_step(ria, prec, trt, rows):
    # the AA odd step launched in the band schedule's order gives the default
    # order's result bit for bit after every step; FP64 equals the oracle
    mask = rsa_spheres((20, 18, 22), 2.5, 0.25, PER, seed=5)
    rho0, u0 = init_fields(mask.shape, seed=6)
    tau, F = 0.65, (2e-5, -1e-5, 5e-6)
    print("case band schedule", ria, prec, trt, rows, flush=True)
    lat, a = solver_for(mask, PER, tau, F, "aa", ria, precision=prec, trt_magic=trt, odd_schedule="band",
                        band_rows=rows)
    _, b = solver_for(mask, PER, tau, F, "aa", ria, precision=prec, trt_magic=trt, odd_schedule=None)
    assert a.band_rows == rows and b.odd_sched is None
    r, v = node_fields(lat, rho0, u0)
    r, v = torch.from_numpy(r).cuda(), torch.from_numpy(v).cuda()
    a.init(r, v)
    b.init(r, v)
    f = dense.initial_state(mask.astype(bool), rho0, u0)
    for t in range(1, 8):
        a.step(1)
        b.step(1)
        fa = a.export_pdfs()
        assert torch.equal(fa, b.export_pdfs()), t
        if prec == "f64":
            f = dense.step(f, mask.astype(bool), PER, tau, F, trt)
            assert np.array_equal(fa.cpu().numpy(), oracle_at_nodes(lat, f)), t


def test_band_schedule_reset_and_auto():
    # NULL restores the default order; "auto" keeps it on small planes
    from paper_1410_0412_amd import _capi
    mask = rsa_spheres((20, 18, 22), 2.5, 0.25, PER, seed=5)
    lat, s = solver_for(mask, PER, 0.7, (1e-5, 0, 0), "aa", "direction", odd_schedule="band", band_rows=8)
    _, ref = solver_for(mask, PER, 0.7, (1e-5, 0, 0), "aa", "direction")
    assert ref.odd_sched is None and ref.band_rows is None
    s.init(); ref.init()
    s.step(3); ref.step(3)
    _capi.check(_capi.lib().lbm_solver_set_odd_schedule(s._h, None, 0, None))
    s.step(4); ref.step(4)
    assert torch.equal(s.export_pdfs(), ref.export_pdfs())


@pytest.mark.parametrize("pattern,ria", VARIANTS)
def test_import_export_roundtrip(pattern, ria):
    mask = rsa_spheres((16, 16, 16), 2.0, 0.2, PER, seed=7)
    rho0, u0 = init_fields(mask.shape, seed=8)
    lat, s = solver_for(mask, PER, 0.8, (1e-5, 0, 0), pattern, ria)
    f0 = oracle_at_nodes(lat, dense.initial_state(mask.astype(bool), rho0, u0))
    for t in (0, 1, 6, 7):
        s.import_pdfs(torch.from_numpy(f0).cuda(), t)
        assert s.t == t
        assert np.array_equal(s.export_pdfs().cpu().numpy(), f0)
    # continue from an odd time step and compare with the oracle
    s.import_pdfs(torch.from_numpy(f0).cuda(), 3)
    s.step(3)
    f = dense.initial_state(mask.astype(bool), rho0, u0)
    for _ in range(3):
        f = dense.step(f, mask.astype(bool), PER, 0.8, (1e-5, 0, 0))
    assert np.array_equal(s.export_pdfs().cpu().numpy(), oracle_at_nodes(lat, f))


@pytest.mark.parametrize("shape,periodic", [((1, 1, 1), (True, True, True)), ((3, 1, 1), (True, False, False)),
                                            ((5, 4, 3), (True, True, True)), ((7, 9, 11), (False, False, False)),
                                            ((64, 1, 1), (True, True, True)), ((65, 3, 2), (True, False, True))])
@pytest.mark.parametrize("pattern,ria", VARIANTS)
def test_small_and_ragged(shape, periodic, pattern, ria):
    rng = np.random.default_rng(sum(shape))
    mask = (rng.random(shape) < 0.2).astype(np.uint8)
    mask.reshape(-1)[0] = 0
    rho0, u0 = init_fields(shape, seed=9)
    lat, s = solver_for(mask, periodic, 0.9, (1e-5, 2e-5, -1e-5), pattern, ria)
    r, v = node_fields(lat, rho0, u0)
    s.init(torch.from_numpy(r).cuda(), torch.from_numpy(v).cuda())
    s.step(5)
    f = dense.run(mask.astype(bool), periodic, 0.9, (1e-5, 2e-5, -1e-5), 5, rho0, u0)
    assert np.array_equal(s.export_pdfs().cpu().numpy(), oracle_at_nodes(lat, f))


@pytest.mark.parametrize("pattern,ria", VARIANTS)
def test_empty_lattice(pattern, ria):
    from paper_1410_0412_amd import Lattice, Solver
    lat = Lattice(np.ones((4, 4, 4), np.uint8))
    sched = ("auto", "band") if pattern == "aa" else ("auto",)
    for odd_schedule in sched:
        s = Solver(lat, 0.8, (1e-6, 0, 0), pattern=pattern, ria=ria, odd_schedule=odd_schedule)
        assert s.odd_sched is None
        s.init()
        s.step(3)
        rho, u, tot = s.moments()
        assert rho.numel() == 0 and s.t == 3 and float(tot.abs().sum()) == 0.0


def test_rest_state_and_no_remap():
    mask = rsa_spheres((24, 24, 24), 3.0, 0.2, PER, seed=10)
    for remap in (True, False):
        lat, s = solver_for(mask, PER, 0.8, (0, 0, 0), "aa", True, xcd_remap=remap)
        s.init()
        s.step(20)
        f = s.export_pdfs().cpu().numpy()
        w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
        assert np.max(np.abs(f - w[:, None])) < 1e-15


def test_errors_from_host():
    from paper_1410_0412_amd import Lattice, Solver, LbmError
    lat = Lattice(np.zeros((4, 4, 4), np.uint8), (True, True, True))
    with pytest.raises(LbmError):
        Solver(lat, 0.5)
    with pytest.raises(LbmError):
        Solver(lat, float("nan"))


@pytest.mark.parametrize("pattern,ria", VARIANTS)
@pytest.mark.parametrize("magic", [3 / 16, 0.05])
def test_trt_every_step(pattern, ria, magic):
    mask = rsa_spheres((18, 16, 20), 2.5, 0.25, PER, seed=15)
    rho0, u0 = init_fields(mask.shape, seed=16)
    tau, F = 0.75, (1e-5, 2e-6, -3e-6)
    lat, s = solver_for(mask, PER, tau, F, pattern, ria, trt_magic=magic)
    r, v = node_fields(lat, rho0, u0)
    s.init(torch.from_numpy(r).cuda(), torch.from_numpy(v).cuda())
    f = dense.initial_state(mask.astype(bool), rho0, u0)
    for t in range(1, 6):
        s.step(1)
        f = dense.step(f, mask.astype(bool), PER, tau, F, magic)
        assert np.array_equal(s.export_pdfs().cpu().numpy(), oracle_at_nodes(lat, f)), t


def test_trt_spheres32_100_steps(spheres32):
    mask, p, _, _, _ = spheres32
    f = dense.run(mask.astype(bool), p["periodic"], p["tau"], p["force"], p["steps"], magic=3 / 16)
    for pattern, ria in VARIANTS:
        lat, s = solver_for(mask, p["periodic"], p["tau"], p["force"], pattern, ria, trt_magic=3 / 16)
        s.init()
        s.step(p["steps"])
        assert np.array_equal(s.export_pdfs().cpu().numpy(), oracle_at_nodes(lat, f))


def test_totals_are_reproducible():
    # the FP64 totals use a fixed reduction order over nodes, so equal states
    # give bitwise equal totals whatever the pattern, index source or parity
    import math
    mask = rsa_spheres((40, 36, 30), 3.0, 0.25, PER, seed=7)
    rho0, u0 = init_fields(mask.shape, seed=8)
    tau, F = 0.7, (1e-5, 0.0, 0.0)
    f_ref = dense.run(mask.astype(bool), PER, tau, F, 3, rho0, u0)
    seen = None
    for pattern, ria in VARIANTS:
        lat, s = solver_for(mask, PER, tau, F, pattern, ria)
        r, v = node_fields(lat, rho0, u0)
        s.init(torch.from_numpy(r).cuda(), torch.from_numpy(v).cuda())
        s.step(3)
        tots = [s.moments()[2].cpu().numpy() for _ in range(3)]
        assert all(np.array_equal(t, tots[0]) for t in tots), (pattern, ria)
        # the totals alone, without the per-node fields
        assert np.array_equal(s.totals().cpu().numpy(), tots[0]), (pattern, ria)
        if seen is None:
            seen = tots[0]
        assert np.array_equal(tots[0], seen), (pattern, ria)
    # against exactly rounded sums of the oracle's f(3)
    f = oracle_at_nodes(lat, f_ref)
    mass = math.fsum(f.reshape(-1))
    assert abs(seen[0] - mass) <= 1e-14 * mass
    from oracle.d3q19 import C
    for a in range(3):
        j = math.fsum((C[:, a][:, None] * f).reshape(-1))
        assert abs(seen[1 + a] - j) <= 1e-14 * mass, a


def test_work_runs_on_the_current_stream():
    # the binding queues every call on torch's current stream; a solver
    # driven on a side stream gives the default-stream result bitwise
    mask = rsa_spheres((20, 18, 22), 2.5, 0.2, PER, seed=3)
    lat, a = solver_for(mask, PER, 0.8, (1e-5, 0.0, 0.0), "aa", "direction")
    _, b = solver_for(mask, PER, 0.8, (1e-5, 0.0, 0.0), "aa", "direction")
    a.init()
    a.step(9)
    fa = a.export_pdfs()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b.init()
        b.step(9)
        fb = b.export_pdfs()
        _, _, tb = b.moments()
    torch.cuda.current_stream().wait_stream(side)
    assert torch.equal(fa, fb)
    assert torch.equal(a.moments()[2], tb)
