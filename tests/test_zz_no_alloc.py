"""lbm_solver_moments_static (partial sums in the library's static device
scratch array, no allocation) against lbm_solver_moments (the solver's
workspace), through the C ABI: bitwise equal fields and totals, on two calls
in a row, the second on a smaller lattice whose reduction reads fewer
partial sums than the first left in the array."""
import ctypes

import numpy as np
import pytest

from lbm_inputs import rsa_spheres, init_fields

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def call_static(s):
    from paper_1410_0412_amd import _capi
    L = _capi.lib()
    N = s.n_fluid
    rho = torch.full((N,), float("nan"), dtype=torch.float64, device=s.device)
    u = torch.full((3, N), float("nan"), dtype=torch.float64, device=s.device)
    tot = torch.full((4,), float("nan"), dtype=torch.float64, device=s.device)
    _capi.check(L.lbm_solver_set_stream(s._h, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    _capi.check(L.lbm_solver_moments_static(s._h, ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                            ctypes.c_void_p(tot.data_ptr())))
    return rho, u, tot


def make(shape, seed, pattern, prec):
    from paper_1410_0412_amd import Lattice, Solver
    per = (True, False, False)
    mask = rsa_spheres(shape, 2.5, 0.15, per, seed=seed)
    lat = Lattice(mask, per, "lex", 0)
    s = Solver(lat, 0.8, (1e-5, 0.0, 0.0), pattern=pattern, precision=prec)
    rho0, u0 = init_fields(mask.shape, seed=seed + 1)
    nv = lat.node_voxel().astype(np.int64)
    s.init(torch.from_numpy(rho0.reshape(-1)[nv]).cuda(), torch.from_numpy(u0.reshape(3, -1)[:, nv]).cuda())
    s.step(3)  # odd t: the AA state sits in the odd-step slots
    return s


@pytest.mark.parametrize("pattern,prec", [("aa", "f64"), ("aa", "f32"), ("aa", "f16"), ("osnt", "f64")])
def test_moments_static_matches_workspace_moments(pattern, prec):
    # 96 x 64 x 64 (about 330k nodes: the full 1024 partial sums), then
    # 16 x 16 x 16 (about 3k nodes: 12 partial sums)
    for shape, seed in (((96, 64, 64), 3), ((16, 16, 16), 5)):
        s = make(shape, seed, pattern, prec)
        print("case moments_static", pattern, prec, shape, "N", s.n_fluid, flush=True)
        want = s.moments()
        got = call_static(s)
        for a, b in zip(got, want):
            assert torch.equal(a, b)
        assert torch.isfinite(got[2]).all()
        del s


def test_moments_static_binding():
    # the Python binding's call of the same entry point
    s = make((16, 16, 16), 9, "aa", "f32")
    want = s.moments()
    got = s.moments_static()
    for a, b in zip(got, want):
        assert torch.equal(a, b)


def test_moments_static_reports_nonfinite_totals():
    from paper_1410_0412_amd import LbmError
    from paper_1410_0412_amd._capi import LBM_ERANGE
    s = make((16, 16, 16), 7, "aa", "f64")
    f = s.export_pdfs()
    f[3, 11] = float("nan")
    s.import_pdfs(f, t=3)
    with pytest.raises(LbmError) as e:
        call_static(s)
    assert e.value.code == LBM_ERANGE
