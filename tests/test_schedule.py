"""The band schedule of the AA odd step (host side): its layout, its errors,
the host checks of lbm_solver_set_odd_schedule, and the automatic choice.
Runs on the CPU (no device call is reached)."""
import ctypes
from types import SimpleNamespace

import numpy as np
import pytest

import paper_1410_0412_amd._capi as capi
from paper_1410_0412_amd import Lattice, choose_odd_schedule
from paper_1410_0412_amd.solver import BAND_PLANE_BYTES, BAND_ROWS
from lbm_inputs import rsa_spheres
from tests.test_capi_validation import params, buffers

L = capi.lib()
PER = (True, False, False)


@pytest.fixture(scope="module")
def lat():
    mask = rsa_spheres((40, 48, 44), 3.0, 0.25, PER, seed=3)
    return mask, Lattice(mask, PER, "lex", 0)


@pytest.mark.parametrize("rows", [8, 16, 24, 48, 64])
def test_band_schedule_layout(lat, rows):
    mask, lt = lat
    S = lt.band_schedule(rows)
    G = (lt.n_fluid + 255) // 256
    assert S.dtype == np.int32 and len(S) % 8 == 0
    # every 256-node block once, -1 elsewhere
    assert np.array_equal(np.sort(S[S >= 0]), np.arange(G))
    assert np.all(S >= -1)
    ny, nz = mask.shape[1], mask.shape[2]
    first = lt.node_voxel().astype(np.int64)[np.arange(G) * 256]
    x, y = first // (ny * nz), (first // nz) % ny
    for k in range(8):
        col = S[k::8]
        blocks = col[col >= 0]
        # XCD k holds the blocks whose first node lies in its rows of a band
        assert np.all(((y[blocks] % rows) * 8) // rows == k)
        # band by band, plane by plane, then node order
        key = (y[blocks] // rows) * mask.shape[0] + x[blocks]
        assert np.all(np.diff(key) >= 0)
        same = np.diff(key) == 0
        assert np.all(np.diff(blocks)[same] > 0)
        # empty slots only after an XCD's last block
        assert np.all(col[len(blocks):] == -1)


def test_band_schedule_errors(lat):
    mask, lt = lat
    n = ctypes.c_int64()
    for rows in (0, -8, 12, 4):
        assert L.lbm_lattice_band_schedule(lt._h, rows, None, ctypes.byref(n)) == capi.LBM_EINVAL
    assert L.lbm_lattice_band_schedule(lt._h, 16, None, None) == capi.LBM_EINVAL
    assert L.lbm_lattice_band_schedule(None, 16, None, ctypes.byref(n)) == capi.LBM_EINVAL
    assert L.lbm_lattice_band_schedule(lt._h, 16, None, ctypes.byref(n)) == 0
    short = np.empty(n.value, np.int32)
    m = ctypes.c_int64(n.value - 8)
    assert L.lbm_lattice_band_schedule(lt._h, 16, short.ctypes.data_as(ctypes.c_void_p), ctypes.byref(m)) == capi.LBM_EINVAL
    # other enumerations have no x-planes in node order
    for order, block in (("morton", 0), ("lex", 4), ("hilbert", 0)):
        other = Lattice(mask, PER, order, block)
        assert not other.plain_lex
        assert L.lbm_lattice_band_schedule(other._h, 16, None, ctypes.byref(n)) == capi.LBM_EINVAL
        assert "LS order" in L.lbm_last_error().decode()
    assert Lattice(mask, PER, "lex", 1).plain_lex and Lattice(mask, PER, "lex", 48).plain_lex


def test_band_schedule_empty_lattice():
    lt = Lattice(np.ones((8, 8, 8), np.uint8), PER, "lex", 0)
    assert lt.n_fluid == 0 and len(lt.band_schedule(8)) == 0


def _solver(pattern=0, n_fluid=1000):
    h = ctypes.c_void_p()
    p = params(pattern=pattern, n_fluid=n_fluid, ldf=1024, lda=1024)
    need = ctypes.c_int64()
    L.lbm_solver_workspace_bytes(ctypes.byref(p), ctypes.byref(need))
    assert L.lbm_solver_create(ctypes.byref(p), ctypes.byref(buffers()), ctypes.c_void_p(0x1000), need.value, None,
                               ctypes.byref(h)) == 0
    return h


@pytest.mark.parametrize("sched,why", [
    ([0, 1, 2, 3, -1, -1, -1, -1, -1], "len not a multiple of 8"),
    ([0, 1, 2, -1, -1, -1, -1, -1], "block 3 missing"),
    ([0, 1, 2, 3, 3, -1, -1, -1], "block 3 twice"),
    ([0, 1, 2, 4, -1, -1, -1, -1], "block 4 beyond the 4 blocks"),
    ([0, 1, 2, 3, -2, -1, -1, -1], "negative entry other than -1"),
])
def test_set_odd_schedule_rejects(sched, why):
    # 1000 nodes: 4 blocks of 256; every check runs on the host before any copy
    h = _solver()
    a = np.array(sched, np.int32)
    rc = L.lbm_solver_set_odd_schedule(h, a.ctypes.data_as(ctypes.c_void_p), len(a), ctypes.c_void_p(0x1000))
    assert rc == capi.LBM_EINVAL, why
    assert L.lbm_last_error()
    L.lbm_solver_free(h)


def test_set_odd_schedule_argument_checks():
    h = _solver()
    a = np.array([0, 1, 2, 3, -1, -1, -1, -1], np.int32)
    ptr = a.ctypes.data_as(ctypes.c_void_p)
    assert L.lbm_solver_set_odd_schedule(h, ptr, len(a), None) == capi.LBM_EINVAL
    assert L.lbm_solver_set_odd_schedule(h, ptr, 0, ctypes.c_void_p(0x1000)) == capi.LBM_EINVAL
    assert L.lbm_solver_set_odd_schedule(None, ptr, len(a), ctypes.c_void_p(0x1000)) == capi.LBM_EINVAL
    # NULL restores the default order and touches no device
    assert L.lbm_solver_set_odd_schedule(h, None, 0, None) == 0
    L.lbm_solver_free(h)
    h = _solver(pattern=1)  # OS-NT
    assert L.lbm_solver_set_odd_schedule(h, ptr, len(a), ctypes.c_void_p(0x1000)) == capi.LBM_ESTATE
    L.lbm_solver_free(h)


def _fake(n, plane_nodes_frac=0.85, plain=True, ib=5.8):
    return SimpleNamespace(plain_lex=plain, n_fluid=int(n ** 3 * plane_nodes_frac), shape=(n, n, n),
                           index_bytes=lambda: {"direction": ib, "runs": 9.8, "adjacency": 72.0})


def test_choose_odd_schedule_rule():
    # one x-plane's odd-step traffic against the threshold: the foam recipe
    # at 384^3 and 512^3 keeps the default order, 768^3 and 1024^3 take bands
    assert BAND_ROWS % 8 == 0
    for n, prec, want in ((384, "f64", None), (512, "f64", None), (512, "f32", None), (768, "f32", BAND_ROWS),
                          (768, "f64", BAND_ROWS), (1024, "f32", BAND_ROWS), (1024, "f64", BAND_ROWS),
                          (768, "f16", None)):
        assert choose_odd_schedule(_fake(n), "aa", prec) == want, (n, prec)
    assert choose_odd_schedule(_fake(1024), "osnt", "f64") is None
    assert choose_odd_schedule(_fake(1024, plain=False), "aa", "f64") is None
    # the threshold itself
    n = 1000
    per_node = 38 * 8 + 5.8
    nodes = BAND_PLANE_BYTES / per_node * n
    assert choose_odd_schedule(_fake(n, nodes * 0.999 / n ** 3), "aa", "f64") is None
    assert choose_odd_schedule(_fake(n, nodes * 1.001 / n ** 3), "aa", "f64") == BAND_ROWS
