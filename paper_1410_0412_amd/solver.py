"""Device solver: PDF grids and lattice tables in torch device memory, every
step run by the HIP kernels of ``liblbm_sparse.so`` (``lbm_solver_*``).

torch provides device memory and the current HIP stream only; no arithmetic
of the method runs in Python.
"""

from __future__ import annotations

import ctypes

import numpy as np

from . import _capi


def _round_up(x, m):
    return (int(x) + m - 1) // m * m


def _vp(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


_GRID_ALIGN = 2 << 20  # bytes


def grid_stride(n):
    """Node slots of a PDF grid: n rounded up to whole 64-node tiles."""
    return _round_up(max(n, 1), 64)


def aligned_empty(torch, numel, dtype, device, align=_GRID_ALIGN):
    """A 1-D tensor of ``numel`` elements whose first element is ``align``-aligned."""
    esize = torch.empty((), dtype=dtype).element_size()
    extra = align // esize
    base = torch.empty(numel + extra, dtype=dtype, device=device)
    off = (-base.data_ptr() % align) // esize
    return base[off:off + numel]


def required_bytes(params):
    """(PDF bytes per grid, workspace bytes) of a solver with these
    parameters, as the library sizes them (``lbm_required_bytes``)."""
    grid, ws = ctypes.c_int64(), ctypes.c_int64()
    _capi.check(_capi.lib().lbm_required_bytes(ctypes.byref(params), ctypes.byref(grid), ctypes.byref(ws)))
    return grid.value, ws.value


def check_device_tensor(torch, t, name, dtype, numel, device):
    """ValueError unless ``t`` is a contiguous ``dtype`` tensor of at least
    ``numel`` elements on ``device``: a kernel reads or writes that many."""
    if not isinstance(t, torch.Tensor):
        raise ValueError("%s must be a torch tensor" % name)
    if t.dtype != dtype or t.device != device or not t.is_contiguous() or t.numel() < numel:
        raise ValueError("%s must be a contiguous %s tensor of at least %d elements on %s (got %s, %d elements "
                         "on %s%s)" % (name, str(dtype).replace("torch.", ""), numel, device,
                                       str(t.dtype).replace("torch.", ""), t.numel(), t.device,
                                       "" if t.is_contiguous() else ", not contiguous"))


def choose_index(lattice, pattern="aa", precision="f64", margin=0.0, ratio=0.7):
    """Index source for ``ria="auto"``: per-direction runs when they need at
    most ``ratio`` times the index bytes of the paper's runs (and save more
    than ``margin`` of the loop balance, the bytes per FLUP with the paper's
    runs); else the paper's runs. The AA pattern pays the index in every
    second step, OS-NT in every step. The ratio bound keeps the paper's runs
    where runs are short in every direction (space-filling curves): there
    per-direction deltas are read without sharing between lanes and save too
    few bytes to pay for the extra table reads."""
    try:
        b = lattice.index_bytes()
    except _capi.LbmError:  # per-direction run count exceeds the int32 table index
        return "runs"
    s = {"f64": 8, "f32": 4, "f16": 2}[precision]
    share = 0.5 if pattern == "aa" else 1.0
    balance = 38.0 * s + share * b["runs"]
    saves = share * (b["runs"] - b["direction"]) > margin * balance
    return "direction" if saves and b["direction"] <= ratio * b["runs"] else "runs"


#: odd-step traffic of one x-plane beyond which the band schedule pays
#: (measured on the foam recipe: neutral at 69 MB, 6-18 % faster odd steps
#: from 79 MB up; slower below, where the default order keeps x-neighbours
#: cached)
BAND_PLANE_BYTES = 72e6
#: rows per band of the automatic band schedule
BAND_ROWS = 32


def choose_odd_schedule(lattice, pattern="aa", precision="f64", index_bytes=None):
    """Workgroup order of the AA odd step for ``odd_schedule="auto"``: the
    band schedule (:meth:`Lattice.band_schedule` with ``BAND_ROWS`` rows)
    when the lattice is in LS order without blocking and one x-plane's
    odd-step traffic, fluid nodes per plane times the bytes a node moves in
    the odd step, exceeds ``BAND_PLANE_BYTES``; else None (the default
    chunked order). The band keeps a block's x-neighbours, one plane away, on
    its XCD within a short time; on small planes the default order already
    finds them in cache."""
    if pattern != "aa" or not lattice.plain_lex or lattice.n_fluid == 0:
        return None
    s = {"f64": 8, "f32": 4, "f16": 2}[precision]
    ib = lattice.index_bytes()["direction"] if index_bytes is None else index_bytes
    plane = lattice.n_fluid / lattice.shape[0] * (38.0 * s + ib)
    return BAND_ROWS if plane > BAND_PLANE_BYTES else None


def _index_source(ria, lattice, pattern, precision):
    if ria is True or ria == "runs":
        return "runs"
    if ria is False or ria == "adjacency":
        return "adjacency"
    if ria == "direction":
        return "direction"
    if ria == "auto":
        return choose_index(lattice, pattern, precision)
    raise ValueError("ria must be True, False, 'runs', 'adjacency', 'direction' or 'auto'")


class Solver:
    """D3Q19 BGK solver on a :class:`Lattice`.

    pattern    "aa" (one grid) or "osnt" (two grids, pull).
    ria        Neighbour index source. "auto" (default): the choice of
               :func:`choose_index`; True or "runs": the paper's RIA runs
               (Sect. 4.1) as per-wavefront tables; False or "adjacency": the
               adjacency list; "direction": per-direction runs.
    precision  "f64" (FP64 storage and arithmetic), "f32" or "f16"
               (storage of deviations from the rest state, FP32 arithmetic).
    f16_scale_log2  FP16 storage holds d_q * 2^s / w_q (default s = 10).
    trt_magic  None: BGK collision; a number Lambda > 0: TRT collision (the
               paper's operator) with that magic parameter.
    pbb        True: allocate a per-node partial-bounce-back solid fraction
               (``solid_frac``, zero-initialised; AA, FP64, BGK only).
    xcd_remap  step kernels: each XCD takes chunks of consecutive tiles in
               turn (False: plain tile order).
    wide_slots step kernels: 64-bit slot offsets even where 32-bit ones
               suffice (grids of at most 2^31 - 1 elements); the same
               result bit for bit.
    odd_schedule  workgroup order of the AA odd step: "auto" (default):
               :func:`choose_odd_schedule`; "band": the band schedule with
               ``band_rows`` rows (AA pattern and LS order without
               blocking only; nothing to order on an empty lattice);
               None: the default chunked order. The result is the same
               bit for bit.
    """

    def __init__(self, lattice, tau, force=(0.0, 0.0, 0.0), pattern="aa", ria="auto",
                 precision="f64", rho0=1.0, device=None, xcd_remap=True, f16_scale_log2=10,
                 trt_magic=None, pbb=False, wide_slots=False, odd_schedule="auto", band_rows=BAND_ROWS):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("Solver needs a GPU (HIP device); none is visible")
        self.torch = torch
        self.device = torch.device(device if device is not None else "cuda")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.lattice = lattice
        self.pattern = pattern
        self.index = _index_source(ria, lattice, pattern, precision)
        self.ria = self.index != "adjacency"
        self.precision = precision
        N, R = lattice.n_fluid, lattice.n_runs
        self.n_fluid = N
        dtype = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16}[precision]
        self.ldf = grid_stride(N)
        ngrids = 2 if pattern == "osnt" else 1
        dev = self.device
        with torch.cuda.device(dev):
            sizing = _capi.Params()
            sizing.precision = _capi.PRECISIONS[precision]
            sizing.n_fluid, sizing.ldf = N, self.ldf
            grid_bytes, ws_bytes = required_bytes(sizing)
            numel = grid_bytes // torch.empty((), dtype=dtype).element_size()
            self.pdf = [aligned_empty(torch, numel, dtype, dev) for _ in range(ngrids)]
            self.adj = self.run_delta = self.head_bits = self.run_base = None
            self.solid_frac = torch.zeros(max(N, 1), dtype=torch.float64, device=dev) if pbb else None
            lda = ldr = 0
            if self.index == "runs":
                ldr = _round_up(max(R, 1), 64)
                delta, bits, base = lattice.wave_tables(ldr)
                self.run_delta = torch.from_numpy(delta).to(dev)
                self.head_bits = torch.from_numpy(bits.view(np.int64)).to(dev)
                self.run_base = torch.from_numpy(base).to(dev)
            elif self.index == "direction":
                R = lattice.n_direction_runs
                delta, bits, base = lattice.direction_tables()
                self.run_delta = torch.from_numpy(delta).to(dev)
                self.head_bits = torch.from_numpy(bits.reshape(-1).view(np.int64)).to(dev)
                self.run_base = torch.from_numpy(base.reshape(-1)).to(dev)
            else:
                lda = _round_up(max(N, 1), 64)
                self.adj = torch.from_numpy(lattice.adjacency(lda)).to(dev)
            p = _capi.Params()
            p.tau = float(tau)
            for a in range(3):
                p.force[a] = float(force[a])
            p.rho0 = float(rho0)
            p.pattern = _capi.PATTERNS[pattern]
            p.ria = _capi.INDEX[self.index]
            p.precision = _capi.PRECISIONS[precision]
            p.flags = (0 if xcd_remap else _capi.FLAG_NO_XCD_REMAP) | (_capi.FLAG_WIDE_SLOTS if wide_slots else 0)
            p.n_fluid, p.n_runs, p.ldf, p.lda, p.ldr = N, R, self.ldf, lda, ldr
            p.f16_scale_log2 = int(f16_scale_log2)
            p.collision = 0 if trt_magic is None else 1
            p.trt_magic = 0.0 if trt_magic is None else float(trt_magic)
            self._params = p
            b = _capi.Buffers()
            b.pdf[0] = self.pdf[0].data_ptr()
            b.pdf[1] = self.pdf[1].data_ptr() if ngrids == 2 else None
            b.adj = self.adj.data_ptr() if self.adj is not None else None
            b.run_delta = self.run_delta.data_ptr() if self.ria else None
            b.head_bits = self.head_bits.data_ptr() if self.ria else None
            b.run_base = self.run_base.data_ptr() if self.ria else None
            b.solid_frac = self.solid_frac.data_ptr() if pbb else None
            self._buffers = b
            L = _capi.lib()
            self.workspace = torch.empty(max(ws_bytes, 8), dtype=torch.uint8, device=dev)
            h = ctypes.c_void_p()
            _capi.check(L.lbm_solver_create(ctypes.byref(p), ctypes.byref(b),
                                            _vp(self.workspace), self.workspace.numel(),
                                            ctypes.c_void_p(self._stream()), ctypes.byref(h)))
            self._h = h
            self._free = L.lbm_solver_free  # bound now: module globals may be gone at exit
            if odd_schedule == "auto":
                ib = lattice.index_bytes()[self.index] if self.index != "adjacency" else 72.0
                rows = choose_odd_schedule(lattice, pattern, precision, ib)
            elif odd_schedule == "band":
                # an empty lattice has no odd-step blocks to order
                rows = int(band_rows) if lattice.n_fluid else None
            elif odd_schedule is None:
                rows = None
            else:
                raise ValueError('odd_schedule must be "auto", "band" or None')
            self.band_rows = rows
            self.odd_sched = None
            if rows:
                sched = lattice.band_schedule(rows)
                self.odd_sched = torch.empty(len(sched), dtype=torch.int32, device=dev)
                sched = np.ascontiguousarray(sched, dtype=np.int32)
                _capi.check(L.lbm_solver_set_odd_schedule(h, sched.ctypes.data_as(ctypes.c_void_p), len(sched),
                                                          _vp(self.odd_sched)))

    # ------------------------------------------------------------------
    def _stream(self):
        return self.torch.cuda.current_stream(self.device).cuda_stream

    def _call(self, fn, *args):
        L = _capi.lib()
        with self.torch.cuda.device(self.device):
            _capi.check(L.lbm_solver_set_stream(self._h, ctypes.c_void_p(self._stream())))
            _capi.check(fn(self._h, *args))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._free(h)
            self._h = None

    # ------------------------------------------------------------------
    def _dev(self, t, shape):
        if t is None:
            return None
        t = self.torch.as_tensor(t, dtype=self.torch.float64, device=self.device).contiguous()
        if tuple(t.shape) != shape:
            raise ValueError("expected shape %r, got %r" % (shape, tuple(t.shape)))
        return t

    def init(self, rho=None, u=None):
        """f(0) = feq(rho, u); rho (N,), u (3, N) in node order (None: rest state)."""
        N = self.n_fluid
        r = self._dev(rho, (N,))
        v = self._dev(u, (3, N))
        self._call(_capi.lib().lbm_solver_init_equilibrium, _vp(r), _vp(v))
        self._keep = (r, v)  # alive until the queued kernel has run

    def step(self, n=1):
        self._call(_capi.lib().lbm_solver_step, int(n))

    @property
    def t(self):
        out = ctypes.c_int64()
        _capi.check(_capi.lib().lbm_solver_time(self._h, ctypes.byref(out)))
        return out.value

    def moments(self):
        """(rho (N,), u (3, N), totals (4,) = mass, jx, jy, jz) of f(t), float64."""
        torch = self.torch
        N = self.n_fluid
        rho = torch.empty(N, dtype=torch.float64, device=self.device)
        u = torch.empty((3, N), dtype=torch.float64, device=self.device)
        tot = torch.empty(4, dtype=torch.float64, device=self.device)
        self._call(_capi.lib().lbm_solver_moments, _vp(rho), _vp(u), _vp(tot))
        return rho, u, tot

    def totals(self):
        """(4,) float64 on the device: mass, jx, jy, jz of f(t), summed in
        the fixed order of :meth:`moments` (the same values bit for bit),
        without writing the per-node fields."""
        tot = self.torch.empty(4, dtype=self.torch.float64, device=self.device)
        self._call(_capi.lib().lbm_solver_moments, None, None, _vp(tot))
        return tot

    def moments_static(self):
        """As :meth:`moments`, through ``lbm_solver_moments_static``: the
        reduction's partial sums go to the library's static device scratch
        array instead of the solver's workspace (for callers that cannot
        allocate; calls that overlap on one device race)."""
        torch = self.torch
        N = self.n_fluid
        rho = torch.empty(N, dtype=torch.float64, device=self.device)
        u = torch.empty((3, N), dtype=torch.float64, device=self.device)
        tot = torch.empty(4, dtype=torch.float64, device=self.device)
        self._call(_capi.lib().lbm_solver_moments_static, _vp(rho), _vp(u), _vp(tot))
        return rho, u, tot

    def export_pdfs(self):
        """f(t) in natural order, float64 (19, N)."""
        f = self.torch.empty((19, self.n_fluid), dtype=self.torch.float64, device=self.device)
        self._call(_capi.lib().lbm_solver_export_pdfs, _vp(f))
        return f

    def set_time(self, t):
        """Declare that ``pdf[0]`` holds the AA state of time ``t``."""
        self._call(_capi.lib().lbm_solver_set_time, int(t))

    def set_solid_fraction(self, ns):
        """Copy per-node solid fractions (N,) into the partial-bounce-back buffer."""
        if self.solid_frac is None:
            raise RuntimeError("solver was created without pbb=True")
        self.solid_frac[: self.n_fluid].copy_(self._dev(ns, (self.n_fluid,)))

    def weighted_momentum(self, weight, axis=0):
        """sum_n weight[n] j_axis(n, t) of f(t), FP64 (0-dim tensor)."""
        w = self._dev(weight, (self.n_fluid,))
        out = self.torch.empty((), dtype=self.torch.float64, device=self.device)
        self._call(_capi.lib().lbm_solver_weighted_momentum, _vp(w), int(axis), _vp(out))
        return out

    def adjoint_seed(self, weight, axis, t, lam):
        """lam (a float64 grid like ``pdf[0]``) = dJ/df(t) of J = sum_n
        weight[n] j_axis(n, t)."""
        check_device_tensor(self.torch, lam, "lam", self.torch.float64, 19 * self.ldf, self.device)
        w = self._dev(weight, (self.n_fluid,))
        self._call(_capi.lib().lbm_adjoint_seed_momentum, _vp(w), int(axis), int(t), _vp(lam))
        self._keep = (w,)

    def step_save(self, save):
        """One AA step that also writes the PDFs f(t) it reads into ``save``
        (a float64 grid like ``pdf[0]``): the forward state
        :meth:`adjoint_step` needs for step t. AA, FP64 and BGK only."""
        check_device_tensor(self.torch, save, "save", self.torch.float64, 19 * self.ldf, self.device)
        self._call(_capi.lib().lbm_solver_step_save, _vp(save))

    def adjoint_step(self, fwd, t, lam, grad):
        """Backward through the step t -> t+1: ``fwd`` holds f(t) (a grid
        like ``pdf[0]``), ``lam`` dJ/df(t+1) on entry and dJ/df(t) on exit,
        ``grad`` (N float64, or None) accumulates dJ/dns."""
        torch = self.torch
        check_device_tensor(torch, fwd, "fwd", torch.float64, 19 * self.ldf, self.device)
        check_device_tensor(torch, lam, "lam", torch.float64, 19 * self.ldf, self.device)
        if grad is not None:
            check_device_tensor(torch, grad, "grad", torch.float64, self.n_fluid, self.device)
        self._call(_capi.lib().lbm_adjoint_step, _vp(fwd), int(t), _vp(lam), _vp(grad))

    def import_pdfs(self, f, t=0):
        g = self._dev(f, (19, self.n_fluid))
        self._call(_capi.lib().lbm_solver_import_pdfs, _vp(g), int(t))
        self._keep = (g,)


def bench_stream(kind, src, dst, n, ld=0):
    """Queue one bandwidth micro-benchmark kernel on torch's current stream."""
    import torch

    _capi.check(_capi.lib().lbm_bench_stream(int(kind), _vp(src), _vp(dst), int(n), int(ld),
                                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
