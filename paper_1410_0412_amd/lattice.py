"""Host lattice: enumeration, adjacency list and RIA tables (C++ builder).

Thin wrapper over ``lbm_lattice_*``: the tables are built by the library and
copied into numpy arrays on request.
"""

from __future__ import annotations

import ctypes

import numpy as np

from . import _capi


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


class Lattice:
    """Sparse D3Q19 lattice of a voxel mask.

    mask      uint8 (nx, ny, nz), C order, nonzero = solid.
    periodic  three booleans; outside of a non-periodic axis counts as solid.
    order     "lex" (lexicographic, x slowest), "morton", "hilbert", or
              "hilbert_ls" (Hilbert partitions re-enumerated by LS).
    block     LS blocking factor B (0 or 1: none); for "hilbert_ls" the
              number of partitions.
    """

    def __init__(self, mask, periodic=(True, False, False), order="lex", block=0):
        L = _capi.lib()
        m = np.ascontiguousarray(np.asarray(mask), dtype=np.uint8)
        if m.ndim != 3:
            raise ValueError("mask must be 3-D")
        self.shape = tuple(int(s) for s in m.shape)
        self.periodic = tuple(bool(p) for p in periodic)
        self.order = order
        self.block = int(block)
        pmask = sum(1 << a for a in range(3) if self.periodic[a])
        h = ctypes.c_void_p()
        _capi.check(L.lbm_lattice_build(_ptr(m), *self.shape, pmask, _capi.ORDERS[order],
                                        self.block, ctypes.byref(h)))
        self._h = h
        self._free = L.lbm_lattice_free  # bound now: module globals may be gone at exit
        n, r, w = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _capi.check(L.lbm_lattice_sizes(h, ctypes.byref(n), ctypes.byref(r), ctypes.byref(w)))
        self.n_fluid, self.n_runs, self.n_waves = n.value, r.value, w.value

    @classmethod
    def from_mask(cls, mask, periodic=(True, False, False), order="lex", block=0):
        """The lattice of ``mask``; the same as the constructor."""
        return cls(mask, periodic, order, block)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._free(h)
            self._h = None

    def node_voxel(self):
        out = np.empty(self.n_fluid, dtype=np.int32)
        _capi.check(_capi.lib().lbm_lattice_copy_nodes(self._h, _ptr(out)))
        return out

    def adjacency(self, ld=None):
        """int32 (18, ld): entry of direction q at row q-1."""
        ld = self.n_fluid if ld is None else int(ld)
        out = np.empty((18, ld), dtype=np.int32)
        _capi.check(_capi.lib().lbm_lattice_copy_adjacency(self._h, _ptr(out), ld))
        return out

    def run_start(self):
        out = np.empty(self.n_runs + 1, dtype=np.int32)
        _capi.check(_capi.lib().lbm_lattice_copy_runs(self._h, _ptr(out)))
        return out

    def wave_tables(self, ldr=None):
        """(run_delta int32 (18, ldr), head_bits uint64 (W,), run_base int32 (W,))."""
        ldr = self.n_runs if ldr is None else int(ldr)
        delta = np.empty((18, ldr), dtype=np.int32)
        bits = np.empty(self.n_waves, dtype=np.uint64)
        base = np.empty(self.n_waves, dtype=np.int32)
        _capi.check(_capi.lib().lbm_lattice_copy_wave_tables(self._h, _ptr(delta), ldr, _ptr(bits),
                                                             _ptr(base)))
        return delta, bits, base

    @property
    def runs_per_node(self):
        return self.n_runs / max(self.n_fluid, 1)

    @property
    def n_direction_runs(self):
        """RD: total number of per-direction runs (all 18 directions)."""
        if getattr(self, "_rd", None) is None:
            rd = ctypes.c_int64()
            _capi.check(_capi.lib().lbm_lattice_direction_runs(self._h, ctypes.byref(rd)))
            self._rd = rd.value
        return self._rd

    @property
    def plain_lex(self):
        """LS order without blocking (x slowest, z fastest)."""
        return self.order == "lex" and (self.block <= 1 or self.block >= max(self.shape))

    def band_schedule(self, band_rows=32):
        """Workgroup order of the AA odd step that sweeps y-bands of
        ``band_rows`` rows plane by plane, XCD k taking rows k/8 of every
        band (lbm_lattice_band_schedule); int32, -1 for empty slots."""
        L = _capi.lib()
        n = ctypes.c_int64()
        _capi.check(L.lbm_lattice_band_schedule(self._h, int(band_rows), None, ctypes.byref(n)))
        out = np.empty(n.value, dtype=np.int32)
        _capi.check(L.lbm_lattice_band_schedule(self._h, int(band_rows), _ptr(out), ctypes.byref(n)))
        return out[: n.value]

    def direction_tables(self):
        """(dir_delta int32 (RD,), dir_bits uint64 (W, 18), dir_base int32 (W, 18))."""
        delta = np.empty(self.n_direction_runs, dtype=np.int32)
        bits = np.empty((self.n_waves, 18), dtype=np.uint64)
        base = np.empty((self.n_waves, 18), dtype=np.int32)
        _capi.check(_capi.lib().lbm_lattice_copy_direction_tables(self._h, _ptr(delta), _ptr(bits),
                                                                  _ptr(base)))
        return delta, bits, base

    def index_bytes(self):
        """Index bytes per node of one indirect step, per index source: the
        adjacency list (72), the paper's runs (72 per run + 12 per 64-node
        wave) and per-direction runs (4 per run + 12 per wave and direction)."""
        N = max(self.n_fluid, 1)
        return {"adjacency": 72.0,
                "runs": (72.0 * self.n_runs + 12.0 * self.n_waves) / N,
                "direction": (4.0 * self.n_direction_runs + 216.0 * self.n_waves) / N}
