"""Gradient oracle for partial bounce-back (test infrastructure only).

A plain dense FP64 PyTorch (CPU) copy of the forward solver of
``oracle.dense`` (BGK, simple forcing, halfway bounce-back) with partial
bounce-back: each fluid site has a solid fraction ns in [0, 1], and its
post-collision PDFs are post_q = (1 - ns) f*_q + ns f_qbar. The objective is
the momentum along one axis summed with per-site weights after T steps,
J = sum_x w(x) j_a(x, T) (an outlet mass flux when w marks an outlet plane).
dJ/dns comes from torch autograd, i.e. from the chain rule applied by a
library primitive to this forward definition.

Partial bounce-back and the objective are not part of the paper; they define
the differentiation extension of the sparse-lattice solver.
"""

from __future__ import annotations

import numpy as np
import torch

from .d3q19 import C, W, OPP, Q
from . import dense


def _fold(terms):
    acc = None
    for t in terms:
        acc = t if acc is None else acc + t
    return acc


def _signed(c, v):
    return v if c > 0 else -v


def _cdot(q, v):
    terms = [_signed(C[q, a], v[a]) for a in range(3) if C[q, a] != 0]
    return 0.0 if not terms else _fold(terms)


def collide_pbb(f, tau, force, ns):
    """Torch version of ``dense.collide`` with partial bounce-back (same order)."""
    omega = 1.0 / tau
    rho = _fold(f[q] for q in range(Q))
    j = [_fold(_signed(C[q, a], f[q]) for q in range(Q) if C[q, a] != 0) for a in range(3)]
    u = [j[a] / rho for a in range(3)]
    usq = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]
    S = dense.force_source(force)
    star = []
    for q in range(Q):
        cu = _cdot(q, u)
        feq = (W[q] * rho) * (((1.0 + 3.0 * cu) + (4.5 * cu) * cu) - 1.5 * usq)
        star.append((f[q] - omega * (f[q] - feq)) + S[q])
    return [((1.0 - ns) * star[q]) + (ns * f[OPP[q]]) for q in range(Q)]


def stream(fstar, solid, periodic):
    out = []
    for q in range(Q):
        pulled = fstar[q]
        for a in range(3):
            if C[q, a] != 0:
                pulled = torch.roll(pulled, int(C[q, a]), dims=a)
        up = torch.from_numpy(dense.upstream_solid(solid, periodic, q))
        out.append(torch.where(up, fstar[OPP[q]], pulled))
    return out


def objective(ns_field, solid, periodic, tau, force, steps, weight, axis=0):
    """J(ns) with f(0) the rest state; ns_field and weight are (nx, ny, nz)."""
    solid = np.asarray(solid, dtype=bool)
    f = [torch.full(solid.shape, W[q], dtype=torch.float64) for q in range(Q)]
    for _ in range(steps):
        f = stream(collide_pbb(f, tau, force, ns_field), solid, periodic)
    j = _fold(_signed(C[q, axis], f[q]) for q in range(Q) if C[q, axis] != 0)
    return (torch.as_tensor(weight, dtype=torch.float64) * j).sum()


def gradient(ns, solid, periodic, tau, force, steps, weight, axis=0):
    """(J, dJ/dns) as numpy arrays over the voxel box (zero on solid voxels)."""
    t = torch.tensor(np.asarray(ns, dtype=np.float64), requires_grad=True)
    J = objective(t, solid, periodic, tau, force, steps, weight, axis)
    J.backward()
    g = t.grad.numpy().copy()
    g[np.asarray(solid, dtype=bool)] = 0.0
    return float(J.detach()), g
