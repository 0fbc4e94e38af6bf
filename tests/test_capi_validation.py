"""Argument validation of the solver C ABI, on the CPU: lbm_solver_create
checks its parameters before it touches the device, so invalid calls can be
exercised with placeholder pointers that are never dereferenced."""
import ctypes
import os

import pytest

capi = pytest.importorskip("paper_1410_0412_amd._capi")
L = capi.lib()

DUMMY = 0x1000  # never dereferenced: every case below fails validation or creates no work


def params(**kw):
    p = capi.Params()
    p.tau, p.rho0 = 0.8, 1.0
    p.pattern, p.ria, p.precision, p.flags = 0, 0, 0, 0
    p.n_fluid, p.n_runs, p.ldf, p.lda, p.ldr = 100, 10, 128, 128, 64
    p.f16_scale_log2, p.collision, p.trt_magic = 10, 0, 0.0
    for k, v in kw.items():
        if k == "force":
            for a in range(3):
                p.force[a] = v[a]
        else:
            setattr(p, k, v)
    return p


def buffers(**kw):
    b = capi.Buffers()
    b.pdf[0] = DUMMY
    b.pdf[1] = DUMMY
    b.adj = b.run_delta = b.head_bits = b.run_base = DUMMY
    b.solid_frac = None
    for k, v in kw.items():
        setattr(b, k, v)
    return b


def create(p, b, ws_bytes=None):
    need = ctypes.c_int64()
    assert L.lbm_solver_workspace_bytes(ctypes.byref(p), ctypes.byref(need)) == 0
    h = ctypes.c_void_p()
    rc = L.lbm_solver_create(ctypes.byref(p), ctypes.byref(b), ctypes.c_void_p(DUMMY),
                             need.value if ws_bytes is None else ws_bytes, None, ctypes.byref(h))
    if rc == 0:
        L.lbm_solver_free(h)
    return rc


def test_valid_parameters_create():
    assert create(params(), buffers()) == 0
    assert create(params(ria=1), buffers()) == 0
    assert create(params(ria=2, n_runs=18 * 3), buffers()) == 0
    assert create(params(pattern=1, precision=2, collision=1, trt_magic=0.1875), buffers()) == 0
    # both flags; 64-bit slots asked for on a small grid
    assert create(params(flags=capi.FLAG_NO_XCD_REMAP | capi.FLAG_WIDE_SLOTS), buffers()) == 0
    # grids beyond 2^31 - 1 elements (64-bit slot offsets) and the largest node count
    assert create(params(n_fluid=150_000_000, ldf=150_000_000, lda=150_000_000), buffers()) == 0
    big = 2 ** 31 - 65
    assert create(params(n_fluid=big, ldf=2 ** 31 - 64, lda=2 ** 31 - 64, pattern=1), buffers()) == 0


@pytest.mark.parametrize("kw,code", [
    (dict(tau=0.5), capi.LBM_EINVAL),
    (dict(tau=float("nan")), capi.LBM_EINVAL),
    (dict(force=(float("inf"), 0, 0)), capi.LBM_EINVAL),
    (dict(rho0=0.0), capi.LBM_EINVAL),
    (dict(pattern=2), capi.LBM_EINVAL),
    (dict(ria=3), capi.LBM_EINVAL),
    (dict(ria=2, n_runs=17), capi.LBM_EINVAL),   # every direction has at least one run
    (dict(ria=2, n_runs=2 ** 31), capi.LBM_ERANGE),
    (dict(precision=3), capi.LBM_EINVAL),
    (dict(flags=4), capi.LBM_EINVAL),
    (dict(collision=1, trt_magic=0.0), capi.LBM_EINVAL),
    (dict(collision=2), capi.LBM_EINVAL),
    (dict(f16_scale_log2=30), capi.LBM_EINVAL),
    (dict(ldf=100), capi.LBM_EINVAL),            # not a multiple of 64
    (dict(ldf=64), capi.LBM_EINVAL),             # < N
    (dict(lda=50), capi.LBM_EINVAL),
    (dict(n_fluid=2 ** 31), capi.LBM_ERANGE),
    (dict(n_fluid=2 ** 31 - 64, ldf=2 ** 31, lda=2 ** 31), capi.LBM_ERANGE),  # node index beyond int32
    (dict(ldf=2 ** 31 + 64), capi.LBM_ERANGE),
    (dict(lda=2 ** 31 + 64), capi.LBM_ERANGE),
    (dict(ria=1, ldr=2 ** 31 + 64), capi.LBM_ERANGE),
    (dict(ria=1, ldr=5), capi.LBM_EINVAL),
    (dict(ria=1, n_runs=0), capi.LBM_EINVAL),
])
def test_invalid_parameters(kw, code):
    assert create(params(**kw), buffers()) == code
    assert L.lbm_last_error()


def test_missing_buffers_and_workspace():
    assert create(params(), buffers(adj=None)) == capi.LBM_EINVAL
    assert create(params(ria=1), buffers(run_delta=None)) == capi.LBM_EINVAL
    for k in ("run_delta", "head_bits", "run_base"):
        assert create(params(ria=2, n_runs=18), buffers(**{k: None})) == capi.LBM_EINVAL
    assert create(params(pattern=1), buffers(pdf=(ctypes.c_void_p * 2)(DUMMY, None))) == capi.LBM_EINVAL
    assert create(params(), buffers(), ws_bytes=8) == capi.LBM_EINVAL


def test_partial_bounce_back_restrictions():
    assert create(params(), buffers(solid_frac=DUMMY)) == 0
    assert create(params(pattern=1), buffers(solid_frac=DUMMY)) == capi.LBM_EINVAL
    assert create(params(precision=1), buffers(solid_frac=DUMMY)) == capi.LBM_EINVAL
    assert create(params(collision=1, trt_magic=0.2), buffers(solid_frac=DUMMY)) == capi.LBM_EINVAL


def test_bench_stream_validation():
    vp = ctypes.c_void_p
    assert L.lbm_bench_stream(9, vp(DUMMY), vp(DUMMY), 10, 10, None) == capi.LBM_EINVAL
    assert L.lbm_bench_stream(0, vp(DUMMY), vp(DUMMY), -1, 0, None) == capi.LBM_EINVAL
    assert L.lbm_bench_stream(1, vp(DUMMY), vp(DUMMY), 10, 5, None) == capi.LBM_EINVAL
    assert L.lbm_bench_stream(0, vp(DUMMY + 8), vp(DUMMY), 10, 0, None) == capi.LBM_EINVAL
    assert L.lbm_bench_stream(5, vp(DUMMY), vp(DUMMY), 100, 64, None) == capi.LBM_EINVAL
    assert L.lbm_bench_stream(6, vp(DUMMY), vp(DUMMY), 100, 100, None) == capi.LBM_EINVAL
    assert L.lbm_bench_stream(0, vp(DUMMY), vp(DUMMY), 0, 0, None) == 0  # nothing to do


def test_null_handles():
    t = ctypes.c_int64()
    assert L.lbm_solver_step(None, 1) == capi.LBM_EINVAL
    assert L.lbm_solver_time(None, ctypes.byref(t)) == capi.LBM_EINVAL
    assert L.lbm_solver_moments(None, None, None, None) == capi.LBM_EINVAL
    assert L.lbm_lattice_sizes(None, None, None, None) == capi.LBM_EINVAL


def test_driver_rejects_bad_arguments(tmp_path):
    # lbm_run checks its arguments and the mask file before any HIP call
    import subprocess

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    driver = os.path.join(root, "paper_1410_0412_amd", "lbm_run")
    assert os.path.exists(driver), "lbm_run is not built (run the package's build.py)"
    mask = tmp_path / "mask.u8"
    mask.write_bytes(b"\0" * 10)
    out = str(tmp_path / "f.bin")

    def run(*args):
        return subprocess.run([driver] + [str(a) for a in args], capture_output=True, text=True, timeout=60)

    r = run()
    assert r.returncode == 1 and "usage" in r.stderr
    good = [mask, 2, 2, 2, 1, "lex", 0, "aa", "runs", "f64", 0.8, 0, 0, 0, 1, out]
    r = run(*good)  # 10 bytes for a 2x2x2 box
    assert r.returncode == 1 and "mask size" in r.stderr
    for pos, bad, msg in ((5, "zigzag", "unknown order"), (7, "push", "unknown pattern"),
                          (8, "list", "unknown index source"), (9, "f8", "unknown precision"),
                          (1, 0, "bad extents")):
        args = list(good)
        args[pos] = bad
        r = run(*args)
        assert r.returncode == 1 and msg in r.stderr, (bad, r.stderr)


def required(p):
    grid, ws = ctypes.c_int64(), ctypes.c_int64()
    rc = L.lbm_required_bytes(ctypes.byref(p), ctypes.byref(grid), ctypes.byref(ws))
    return rc, grid.value, ws.value


@pytest.mark.parametrize("prec,size", [(0, 8), (1, 4), (2, 2)])
def test_required_bytes_per_grid(prec, size):
    # one grid holds 19 PDFs per node slot (Sect. 4) in the storage type
    need = ctypes.c_int64()
    assert L.lbm_solver_workspace_bytes(ctypes.byref(params()), ctypes.byref(need)) == 0
    assert required(params(precision=prec, n_fluid=100, ldf=128)) == (0, 19 * 128 * size, need.value)
    # ldf = 0: the smallest valid stride, N rounded up to 64
    assert required(params(precision=prec, n_fluid=100, ldf=0)) == (0, 19 * 128 * size, need.value)
    assert required(params(precision=prec, n_fluid=128, ldf=0))[1] == 19 * 128 * size
    assert required(params(precision=prec, n_fluid=0, ldf=0))[1] == 19 * 64 * size
    # the largest stride the 32-bit slot offsets allow, the next one (64-bit
    # offsets), and the largest node count
    top = (2 ** 31 - 1) // 19 // 64 * 64
    assert required(params(precision=prec, n_fluid=top, ldf=top))[1] == 19 * top * size
    assert required(params(precision=prec, n_fluid=top + 1, ldf=0))[1] == 19 * (top + 64) * size
    big = 2 ** 31 - 65
    assert required(params(precision=prec, n_fluid=big, ldf=0)) == (0, 19 * (2 ** 31 - 64) * size, need.value)


@pytest.mark.parametrize("kw,code", [
    (dict(precision=3), capi.LBM_EINVAL),
    (dict(n_fluid=-1, ldf=0), capi.LBM_EINVAL),
    (dict(n_fluid=100, ldf=96), capi.LBM_EINVAL),
    (dict(n_fluid=100, ldf=130), capi.LBM_EINVAL),
    (dict(n_fluid=2 ** 31, ldf=0), capi.LBM_ERANGE),
    (dict(n_fluid=2 ** 31 - 64, ldf=0), capi.LBM_ERANGE),
    (dict(n_fluid=100, ldf=2 ** 31 + 64), capi.LBM_ERANGE),
])
def test_required_bytes_rejects(kw, code):
    assert required(params(**kw))[0] == code
    assert L.lbm_last_error()


def test_required_bytes_null_pointers():
    out = ctypes.c_int64()
    assert L.lbm_required_bytes(None, ctypes.byref(out), ctypes.byref(out)) == capi.LBM_EINVAL
    assert L.lbm_required_bytes(ctypes.byref(params()), None, ctypes.byref(out)) == capi.LBM_EINVAL
    assert L.lbm_required_bytes(ctypes.byref(params()), ctypes.byref(out), None) == capi.LBM_EINVAL


def test_adjoint_argument_checks():
    # the binding refuses tensors the adjoint kernels would read or write out
    # of bounds, before any call reaches the device
    torch = pytest.importorskip("torch")
    from paper_1410_0412_amd.solver import check_device_tensor

    cpu = torch.device("cpu")
    ok = torch.zeros(19 * 128, dtype=torch.float64)
    check_device_tensor(torch, ok, "lam", torch.float64, 19 * 128, cpu)
    bad = [ok.float(),                                  # FP32
           ok[: 19 * 128 - 1],                          # one element short
           torch.zeros(2 * 19 * 128, dtype=torch.float64)[::2],  # strided view
           None]
    for t in bad:
        with pytest.raises(ValueError):
            check_device_tensor(torch, t, "lam", torch.float64, 19 * 128, cpu)
    with pytest.raises(ValueError):  # wrong device
        check_device_tensor(torch, ok, "lam", torch.float64, 19 * 128, torch.device("cuda", 0))
