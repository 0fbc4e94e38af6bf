"""Deviation storage (FP32 and FP16 PDFs, FP32 arithmetic, FP64 moments and
reductions) against the FP64 oracle, error stated per field.

Tolerances (derived in the design notes from the unit roundoff of the storage
format and the step count): FP32 normwise velocity error <= 1e-5, density
<= 1e-7 absolute, mass <= 1e-9 relative; FP16 (relative precision 2^-11)
normwise velocity error <= 5e-3, density <= 5e-5, mass <= 1e-6.
"""
import numpy as np
import pytest

from lbm_inputs import rsa_spheres, init_fields, workload
from oracle import dense
from tests.gpu_util import solver_for, node_fields, normwise_u_error, VARIANTS

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

PER = (True, False, False)
TOL = {"f32": dict(u=1e-5, rho=1e-7, mass=1e-9), "f16": dict(u=5e-3, rho=5e-5, mass=1e-6)}


def field_errors(lat, s, f_ref):
    rho, u, tot = s.moments()
    nv = lat.node_voxel().astype(np.int64)
    r_ref, u_ref = dense.macroscopic(f_ref)
    rr = r_ref.reshape(-1)[nv]
    ur = np.stack([u_ref[a].reshape(-1)[nv] for a in range(3)])
    ug = u.cpu().numpy()
    scale = np.sqrt((ur ** 2).sum(0)).max()
    e = dict(
        u=normwise_u_error(ug, ur),
        rho=float(np.max(np.abs(rho.cpu().numpy() - rr))),
        mass=abs(tot[0].item() - rr.sum()) / rr.sum(),
    )
    # per component: max |u_a - u_a,ref| over nodes, relative to max |u_ref|
    for a, name in enumerate(("ux", "uy", "uz")):
        e[name] = float(np.max(np.abs(ug[a] - ur[a])) / scale)
    return e


@pytest.fixture(scope="module")
def spheres32():
    mask, p = workload("spheres-32", seed=0)
    f = dense.run(mask.astype(bool), p["periodic"], p["tau"], p["force"], p["steps"])
    return mask, p, f


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_spheres32_forced_flow(spheres32, prec):
    mask, p, f_ref = spheres32
    lat, s = solver_for(mask, p["periodic"], p["tau"], p["force"], "aa", True, precision=prec)
    s.init()
    s.step(p["steps"])
    e = field_errors(lat, s, f_ref)
    print("spheres-32 %s errors %r" % (prec, e), flush=True)
    for k, tol in TOL[prec].items():
        assert e[k] <= tol, (k, e[k])
    for k in ("ux", "uy", "uz"):  # bounded by the normwise error
        assert e[k] <= e["u"] * (1 + 1e-12), (k, e[k])


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_random_state(prec):
    mask = rsa_spheres((20, 18, 22), 2.5, 0.25, PER, seed=5)
    rho0, u0 = init_fields(mask.shape, seed=6)
    tau, F = 0.65, (2e-5, -1e-5, 5e-6)
    lat, s = solver_for(mask, PER, tau, F, "aa", True, precision=prec)
    r, v = node_fields(lat, rho0, u0)
    s.init(torch.from_numpy(r).cuda(), torch.from_numpy(v).cuda())
    s.step(40)
    f = dense.run(mask.astype(bool), PER, tau, F, 40, rho0, u0)
    e = field_errors(lat, s, f)
    print("random-state %s errors %r" % (prec, e), flush=True)
    for k, tol in TOL[prec].items():
        assert e[k] <= tol, (k, e[k])


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_variants_bitwise_identical(prec):
    # the arithmetic per node does not depend on addressing or pattern
    mask = rsa_spheres((24, 20, 18), 2.5, 0.25, PER, seed=7)
    rho0, u0 = init_fields(mask.shape, seed=8)
    outs = []
    for pattern, ria in VARIANTS:
        lat, s = solver_for(mask, PER, 0.7, (1e-5, 0, 0), pattern, ria, precision=prec)
        r, v = node_fields(lat, rho0, u0)
        s.init(torch.from_numpy(r).cuda(), torch.from_numpy(v).cuda())
        s.step(11)
        outs.append(s.export_pdfs().cpu().numpy())
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_import_export_roundtrip(prec):
    mask = rsa_spheres((12, 12, 12), 2.0, 0.2, PER, seed=9)
    rho0, u0 = init_fields(mask.shape, seed=10)
    lat, s = solver_for(mask, PER, 0.8, (0, 0, 0), "aa", True, precision=prec)
    r, v = node_fields(lat, rho0, u0)
    s.init(torch.from_numpy(r).cuda(), torch.from_numpy(v).cuda())
    f0 = s.export_pdfs()
    for t in (0, 1, 4, 5):
        s.import_pdfs(f0, t)
        assert np.array_equal(s.export_pdfs().cpu().numpy(), f0.cpu().numpy())


def test_rest_state_exact():
    # deviations of the rest state are exactly zero in every format
    mask = rsa_spheres((16, 16, 16), 2.5, 0.2, PER, seed=11)
    for prec in ("f32", "f16"):
        lat, s = solver_for(mask, PER, 0.8, (0, 0, 0), "aa", True, precision=prec)
        s.init()
        s.step(10)
        rho, u, tot = s.moments()
        assert float(u.abs().max()) == 0.0 and float((rho - 1).abs().max()) == 0.0


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_trt_random_state(prec):
    mask = rsa_spheres((20, 18, 22), 2.5, 0.25, PER, seed=5)
    rho0, u0 = init_fields(mask.shape, seed=6)
    tau, F, magic = 0.65, (2e-5, -1e-5, 5e-6), 3 / 16
    lat, s = solver_for(mask, PER, tau, F, "aa", True, precision=prec, trt_magic=magic)
    r, v = node_fields(lat, rho0, u0)
    s.init(torch.from_numpy(r).cuda(), torch.from_numpy(v).cuda())
    s.step(40)
    f = dense.run(mask.astype(bool), PER, tau, F, 40, rho0, u0, magic=magic)
    e = field_errors(lat, s, f)
    print("trt random-state %s errors %r" % (prec, e), flush=True)
    for k, tol in TOL[prec].items():
        assert e[k] <= tol, (k, e[k])


def test_f16_import_rounds_once():
    # FP16 storage holds x = (f - w_q rho0) * 2^s / w_q rounded once to the
    # nearest half (ties to even), as numpy converts float64 to float16. The
    # inputs sit next to half-way points between two halves, where rounding
    # first to float and then to half would land on the wrong side for many
    # of them (about 40 % of these).
    from paper_1410_0412_amd import Lattice, Solver
    mask = rsa_spheres((16, 16, 16), 2.5, 0.2, PER, seed=3)
    lat = Lattice(mask, PER, "lex", 0)
    N = lat.n_fluid
    s = Solver(lat, 0.8, (0.0, 0.0, 0.0), precision="f16", f16_scale_log2=10)
    w = np.array([1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12)
    hs = np.array([2.0 ** 10 * (3 if q == 0 else (18 if q < 7 else 36)) for q in range(19)])
    rng = np.random.default_rng(5)
    h = rng.uniform(-2000, 2000, (19, N)).astype(np.float16).astype(np.float64)
    ulp = np.spacing(np.abs(h).astype(np.float16)).astype(np.float64)
    x = (np.abs(h) + ulp / 2) * np.sign(h) * (1 + rng.integers(-3, 4, (19, N)) * 2.0 ** -35)
    f = x / hs[:, None] + w[:, None] * 1.0
    # the kernel's own double operations, in its order
    want = ((f - w[:, None] * 1.0) * hs[:, None]).astype(np.float16)
    twice = ((f - w[:, None] * 1.0) * hs[:, None]).astype(np.float32).astype(np.float16)
    assert (want.view(np.uint16) != twice.view(np.uint16)).mean() > 0.2  # the case is sensitive
    s.import_pdfs(torch.from_numpy(f).cuda(), t=0)
    grid = s.pdf[0].cpu().numpy()
    n = np.arange(N)
    slots = (19 * (n // 64))[None, :] * 64 + np.arange(19)[:, None] * 64 + (n % 64)[None, :]
    got = grid[slots]
    assert np.array_equal(got.view(np.uint16), want.view(np.uint16))
