"""Parity at the benchmark sizes, in the launch configuration the benchmark
times: sampled sites against the oracle's dependency-cone evaluation after a
few steps, properties that hold at any size (bitwise identity of all
propagation variants, mass conservation over many steps), deviation storage
against the FP64 path, the largest lattice the 32-bit slot offsets allow,
and the 512^3 foam, whose grids need 64-bit offsets."""
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


@pytest.fixture(scope="module")
def foam():
    # the 384^3 foam of the benchmark's default line, the enumeration sweep
    # and the precision study
    return workload("foam-384", seed=0)


@pytest.mark.parametrize("order,block,ria", [("lex", 0, "direction"), ("lex", 0, True), ("lex", 8, "direction"),
                                             ("morton", 0, True), ("hilbert_ls", 8, True)])
def test_foam384_sampled_sites(foam, order, block, ria):
    # ("lex", 0, "direction") is the benchmark's main line: LS without
    # blocking, per-direction runs (the automatic choice on this lattice)
    mask, p = foam
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


@pytest.mark.parametrize("pattern,steps", [("aa", 20), ("aa", 21), ("osnt", 20)])
def test_foam384_twenty_steps_sampled_sites(foam, pattern, steps):
    # the main line's lattice and index (LS without blocking, per-direction
    # runs) after 20 and 21 steps (AA exports its natural layout after an
    # even count, its odd-step slots after an odd one): 6 sites against the
    # oracle's dependency cone (a 43^3 or 45^3 crop each), bitwise
    mask, p = foam
    rho0, u0 = init_fields(mask.shape, seed=25)
    fl = np.flatnonzero(mask.reshape(-1) == 0)
    pick = fl[np.random.default_rng(26).choice(len(fl), 6, replace=False)]
    sites = np.stack(np.unravel_index(pick, mask.shape), 1)
    want = dense.cone_sites(mask.astype(bool), p["periodic"], p["tau"], p["force"], steps, rho0, u0, sites)
    print("case foam-384", steps, "steps", pattern, flush=True)
    lat, s = solver_for(mask, p["periodic"], p["tau"], p["force"], pattern, "direction", p["order"], p["block"])
    r, v = node_fields(lat, rho0, u0)
    del rho0, u0
    s.init(torch.from_numpy(r).cuda(), torch.from_numpy(v).cuda())
    s.step(steps)
    f = s.export_pdfs()
    node_of = np.full(mask.size, -1, np.int64)
    node_of[lat.node_voxel().astype(np.int64)] = np.arange(lat.n_fluid)
    got = f[:, torch.from_numpy(node_of[pick]).cuda()].T.cpu().numpy()
    assert np.array_equal(got, want)


def test_foam384_variants_identical_and_conserve_mass(foam):
    # the benchmark's lattice: all six variants (two patterns x three index
    # sources) give bitwise the same state after 60 steps from a random
    # state, and conserve mass to 1e-12
    mask, p = foam
    steps = 60
    rho0, u0 = init_fields(mask.shape, seed=27)
    from paper_1410_0412_amd import Lattice, Solver
    lat = Lattice(mask, p["periodic"], p["order"], p["block"])
    r, v = node_fields(lat, rho0, u0)
    del rho0, u0
    first = None
    for pattern, ria in VARIANTS:
        s = Solver(lat, p["tau"], p["force"], pattern=pattern, ria=ria)
        print("case foam-384 variants", pattern, s.index, flush=True)
        s.init(torch.from_numpy(r).cuda(), torch.from_numpy(v).cuda())
        _, _, t0 = s.moments()
        s.step(steps)
        _, u, t1 = s.moments()
        m0, m1 = t0[0].item(), t1[0].item()
        assert abs(m1 - m0) / m0 < 1e-12, (pattern, ria)
        if first is None:
            first = u
        else:
            assert torch.equal(u, first), (pattern, ria)
        del s, u
        torch.cuda.empty_cache()


@pytest.mark.parametrize("prec,tol_u,tol_rho", [("f32", 1e-5, 1e-7), ("f16", 5e-3, 5e-5)])
def test_foam384_deviation_storage_against_fp64(foam, prec, tol_u, tol_rho):
    # the benchmark's FP32 and FP16 lines (LS without blocking, automatic
    # index choice) against the FP64 line on the same random state, 20
    # steps; bounds as for the sphere pack
    mask, p = foam
    steps = 20
    rho0, u0 = init_fields(mask.shape, seed=23)
    from paper_1410_0412_amd import Lattice, Solver
    lat = Lattice(mask, p["periodic"], p["order"], p["block"])
    r, v = node_fields(lat, rho0, u0)
    del rho0, u0
    out = {}
    for pr in ("f64", prec):
        s = Solver(lat, p["tau"], p["force"], pattern="aa", ria="auto", precision=pr)
        print("case foam-384 deviation storage", pr, "index", s.index, flush=True)
        s.init(torch.from_numpy(r).cuda(), torch.from_numpy(v).cuda())
        s.step(steps)
        rho, u, tot = s.moments()
        out[pr] = (rho, u, tot[0].item())
        del s
        torch.cuda.empty_cache()
    (r64, u64, m64), (rl, ul, ml) = out["f64"], out[prec]
    du = (torch.sqrt(((ul - u64) ** 2).sum(0)).max() / torch.sqrt((u64 ** 2).sum(0)).max()).item()
    drho = (rl - r64).abs().max().item()
    print("%s on the foam: normwise u %.3e, max rho %.3e, mass %.3e" % (prec, du, drho, abs(ml - m64) / m64),
          flush=True)
    assert du <= tol_u and drho <= tol_rho and abs(ml - m64) / m64 <= 1e-6


def test_channel_sampled_sites_and_variants():
    # the paper's empty 500x100x100 channel (Sect. 5.1), LS with B = 1: long
    # runs in every direction, the case RIA was designed for
    mask, p = workload("channel-500x100x100")
    steps = 3
    rho0, u0 = init_fields(mask.shape, seed=41)
    fl = np.argwhere(mask == 0)
    rng = np.random.default_rng(42)
    wall = fl[(fl[:, 1] == 1) | (fl[:, 1] == 98) | (fl[:, 2] == 1) | (fl[:, 2] == 98)]
    seam = fl[(fl[:, 0] == 0) | (fl[:, 0] == mask.shape[0] - 1)]
    sites = np.concatenate([fl[rng.choice(len(fl), 24, replace=False)],
                            wall[rng.choice(len(wall), 8, replace=False)],
                            seam[rng.choice(len(seam), 4, replace=False)]])
    want = dense.cone_sites(mask.astype(bool), p["periodic"], p["tau"], p["force"], steps, rho0, u0, sites)
    vox = (sites[:, 0] * mask.shape[1] + sites[:, 1]) * mask.shape[2] + sites[:, 2]
    first = None
    for pattern, ria in VARIANTS:
        print("case channel sampled", pattern, ria, flush=True)
        lat, s = solver_for(mask, p["periodic"], p["tau"], p["force"], pattern, ria, p["order"], p["block"])
        assert lat.n_fluid == 500 * 98 * 98
        r, v = node_fields(lat, rho0, u0)
        s.init(torch.from_numpy(r).cuda(), torch.from_numpy(v).cuda())
        s.step(steps)
        f = s.export_pdfs()
        node_of = np.full(mask.size, -1, np.int64)
        node_of[lat.node_voxel().astype(np.int64)] = np.arange(lat.n_fluid)
        got = f[:, torch.from_numpy(node_of[vox]).cuda()].T.cpu().numpy()
        assert np.array_equal(got, want), (pattern, ria)
        # 16 more steps: t = 19 is odd, so AA exports through its odd-step slots
        s.step(16)
        g = s.export_pdfs()
        if first is None:
            first = g
        else:
            assert torch.equal(g, first), (pattern, ria)
        del s, f, g


@pytest.mark.parametrize("prec,tol_u,tol_rho", [("f32", 1e-5, 1e-7), ("f16", 5e-3, 5e-5)])
def test_spherepack_deviation_storage_against_fp64(pack, prec, tol_u, tol_rho):
    # deviation storage at the benchmark size against the FP64 path (which is
    # bitwise the oracle), random state, 20 steps; bounds as for the small cases
    mask, p = pack
    steps = 20
    rho0, u0 = init_fields(mask.shape, seed=31)
    out = {}
    for pr in ("f64", prec):
        print("case spherepack deviation storage", pr, flush=True)
        lat, s = solver_for(mask, p["periodic"], p["tau"], p["force"], "aa", "auto", p["order"], p["block"],
                            precision=pr)
        r, v = node_fields(lat, rho0, u0)
        s.init(torch.from_numpy(r).cuda(), torch.from_numpy(v).cuda())
        s.step(steps)
        rho, u, tot = s.moments()
        out[pr] = (rho.cpu().numpy(), u.cpu().numpy(), tot[0].item())
        del s
    (r64, u64, m64), (rl, ul, ml) = out["f64"], out[prec]
    du = np.sqrt(((ul - u64) ** 2).sum(0)).max() / np.sqrt((u64 ** 2).sum(0)).max()
    drho = np.abs(rl - r64).max()
    print("%s: normwise u %.3e, max rho %.3e, mass %.3e" % (prec, du, drho, abs(ml - m64) / m64), flush=True)
    assert du <= tol_u and drho <= tol_rho and abs(ml - m64) / m64 <= 1e-6


@pytest.fixture(scope="module")
def maxcase():
    # the largest lattice the 32-bit slot offsets allow: a fully fluid
    # periodic 480 x 480 x 490 box, N = 112,896,000 nodes, 19 * ldf just
    # below 2^31 - 1
    shape = (480, 480, 490)
    per = (True, True, True)
    tau, force, steps = 0.7, (1e-6, 0.0, 0.0), 3
    mask = np.zeros(shape, np.uint8)
    print("case maximum size: building the lattice", flush=True)
    from paper_1410_0412_amd import Lattice
    lat = Lattice(mask, per, "lex", 0)
    N = lat.n_fluid
    assert N == 480 * 480 * 490 and 19 * ((N + 63) // 64 * 64) <= 2 ** 31 - 1
    rho0, u0 = init_fields(shape, seed=41)
    r, v = node_fields(lat, rho0, u0)
    rng = np.random.default_rng(42)
    sites = np.stack([rng.integers(0, n, 30) for n in shape], 1)
    sites = np.concatenate([sites, [[479, 479, 489], [0, 0, 0]]])
    want = dense.cone_sites(mask.astype(bool), per, tau, force, steps, rho0, u0, sites)
    del rho0, u0
    node = (sites[:, 0] * shape[1] + sites[:, 1]) * shape[2] + sites[:, 2]
    return lat, per, tau, force, steps, r, v, node, want


@pytest.mark.parametrize("pattern,ria", [("aa", "auto"), ("osnt", "auto"), ("aa", False), ("osnt", "direction")])
def test_maximum_size_lattice(maxcase, pattern, ria):
    # sampled sites (including the last node) after 3 steps against the
    # oracle's dependency cone, bitwise
    from paper_1410_0412_amd import Solver
    lat, per, tau, force, steps, r, v, node, want = maxcase
    s = Solver(lat, tau, force, pattern=pattern, ria=ria)
    s.init(torch.from_numpy(r).cuda(), torch.from_numpy(v).cuda())
    print("case maximum size:", pattern, "index", s.index, flush=True)
    s.step(steps)
    f = s.export_pdfs()
    got = f[:, torch.from_numpy(node).cuda()].T.cpu().numpy()
    del s, f
    torch.cuda.empty_cache()
    assert np.array_equal(got, want)


@pytest.mark.parametrize("pattern", ["aa", "osnt"])
def test_spherepack_trt_sampled_sites(pack, pattern):
    # the paper's TRT collision (magic 3/16) at the benchmark size, bitwise
    mask, p = pack
    steps, magic = 3, 3.0 / 16.0
    rho0, u0 = init_fields(mask.shape, seed=51)
    fl = np.argwhere(mask == 0)
    sites = fl[np.random.default_rng(52).choice(len(fl), 32, replace=False)]
    want = dense.cone_sites(mask.astype(bool), p["periodic"], p["tau"], p["force"], steps, rho0, u0, sites,
                            magic=magic)
    print("case spherepack TRT sampled", pattern, flush=True)
    lat, s = solver_for(mask, p["periodic"], p["tau"], p["force"], pattern, "auto", p["order"], p["block"],
                        trt_magic=magic)
    r, v = node_fields(lat, rho0, u0)
    s.init(torch.from_numpy(r).cuda(), torch.from_numpy(v).cuda())
    s.step(steps)
    f = s.export_pdfs().cpu().numpy()
    node_of = np.full(mask.size, -1, np.int64)
    node_of[lat.node_voxel().astype(np.int64)] = np.arange(lat.n_fluid)
    vox = (sites[:, 0] * mask.shape[1] + sites[:, 1]) * mask.shape[2] + sites[:, 2]
    assert np.array_equal(f[:, node_of[vox]].T, want)


@pytest.fixture(scope="module")
def foam512():
    # the foam recipe at 512^3: N = 114,085,068 nodes, so a grid holds more
    # than 2^31 - 1 elements and the step kernels take 64-bit slot offsets
    print("case 64-bit slots: generating the 512^3 foam", flush=True)
    mask, p = workload("foam-512", seed=0)
    from paper_1410_0412_amd import Lattice
    lat = Lattice(mask, p["periodic"], p["order"], p["block"])
    N = lat.n_fluid
    top = (2 ** 31 - 1) // 19  # nodes from about here on own slots beyond 2^31 - 1
    assert 19 * ((N + 63) // 64 * 64) > 2 ** 31 - 1 and N > top
    steps = 3
    rho0, u0 = init_fields(mask.shape, seed=61)
    r, v = node_fields(lat, rho0, u0)
    nv = lat.node_voxel().astype(np.int64)  # increasing in lexicographic order
    rng = np.random.default_rng(62)
    shape = np.array(mask.shape)

    def fluid_sites(lo, hi, count):
        pts = np.stack([rng.integers(lo[a], hi[a], 4 * count) for a in range(3)], 1)
        pts = pts[mask[pts[:, 0], pts[:, 1], pts[:, 2]] == 0]
        return pts[:count]

    # anywhere; the last planes (nodes whose own slots lie beyond 2^31 - 1);
    # the first plane (periodic neighbours of the last); the last node
    last = np.array(np.unravel_index(nv[-1], mask.shape))
    sites = np.concatenate([fluid_sites([0, 0, 0], shape, 24),
                            fluid_sites([507, 0, 0], shape, 24),
                            fluid_sites([0, 0, 0], [1, 512, 512], 8), last[None]])
    vox = (sites[:, 0] * shape[1] + sites[:, 1]) * shape[2] + sites[:, 2]
    node = np.searchsorted(nv, vox)
    assert np.array_equal(nv[node], vox)
    assert (node >= top).sum() >= 20 and node.max() == N - 1
    want = dense.cone_sites(mask.astype(bool), p["periodic"], p["tau"], p["force"], steps, rho0, u0, sites)
    del rho0, u0, nv
    return lat, p, steps, r, v, node, want


W_Q = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def test_foam384_band_schedule_bitwise(foam):
    # the default line's lattice with the odd step in the band order (32
    # rows), 20 steps: bitwise the default order's state
    from paper_1410_0412_amd import Lattice, Solver
    mask, p = foam
    lat = Lattice(mask, p["periodic"], p["order"], p["block"])
    out = []
    for sched in (None, "band"):
        print("case foam-384 odd schedule", sched, flush=True)
        s = Solver(lat, p["tau"], p["force"], pattern="aa", ria="direction", odd_schedule=sched)
        s.init()
        s.step(20)
        out.append(s.export_pdfs())
        del s
    assert torch.equal(out[0], out[1])
    del out
    torch.cuda.empty_cache()


@pytest.mark.parametrize("pattern,ria,prec,pbb", [
    ("aa", "auto", "f64", False), ("osnt", "auto", "f64", False), ("aa", False, "f64", False),
    ("aa", True, "f64", False), ("osnt", True, "f64", False), ("aa", "auto", "f64", True),
    ("aa", "auto", "f32", False), ("osnt", "auto", "f32", False), ("aa", "auto", "f16", False),
    ("aa", "band", "f64", False)])
def test_foam512_wide_slots_sampled_sites(foam512, pattern, ria, prec, pbb):
    # sampled sites after 3 steps against the oracle's dependency cone:
    # bitwise in FP64 (with partial bounce-back at ns = 0 too), within the
    # rounding of the storage format in FP32 and FP16 (max |df_q| / w_q;
    # a value from a wrong slot is off by about 3 |c_q . du| ~ 4e-2)
    from paper_1410_0412_amd import Solver
    lat, p, steps, r, v, node, want = foam512
    band = ria == "band"  # per-direction runs with the odd step in the band order
    s = Solver(lat, p["tau"], p["force"], pattern=pattern, ria="auto" if band else ria, precision=prec, pbb=pbb,
               odd_schedule="band" if band else "auto")
    print("case 64-bit slots:", pattern, "index", s.index, prec, "pbb" if pbb else "", flush=True)
    s.init(torch.from_numpy(r).cuda(), torch.from_numpy(v).cuda())
    s.step(steps)
    f = s.export_pdfs()
    got = f[:, torch.from_numpy(node).cuda()].T.cpu().numpy()
    del s, f
    torch.cuda.empty_cache()
    if prec == "f64":
        assert np.array_equal(got, want)
    else:
        err = float(np.max(np.abs(got - want) / W_Q))
        print("max |df_q| / w_q = %.3e" % err, flush=True)
        assert err <= {"f32": 1e-6, "f16": 5e-4}[prec]
