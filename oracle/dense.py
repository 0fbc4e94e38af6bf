"""Full-array FP64 D3Q19 BGK solver (oracle; test infrastructure only).

The sparse-lattice propagation steps of the paper (OS-NT and the AA pattern,
with or without reduced indirect addressing, under any enumeration) change
only where PDFs are stored and in which order nodes are visited; they reach
exactly the result of a plain full-array stream-and-collide solver of the
lattice Boltzmann equation, Sect. 2, eq. (1). This module is that solver,
written on dense arrays ``f[q, x, y, z]`` with one full copy per step.

The paper names the collision operator (TRT) but gives no formulas, no
equilibrium, no wall rule and no forcing. The readings used here:

* BGK collision with relaxation time tau (omega = 1/tau), or the paper's TRT
  operator with magic parameter Lambda;
* second-order equilibrium with c_s^2 = 1/3:
  feq_q = w_q rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u);
* constant body-force density F added after relaxation as
  S_q = 3 w_q (c_q . F), with u = j / rho (no half-force shift);
* halfway bounce-back at solid voxels; on a non-periodic axis the outside
  of the box counts as solid.

Every sum and product is evaluated in one fixed order (left folds in
ascending q, axis order x, y, z, zero-coefficient terms skipped) so that the
result is a single well-defined IEEE double value per site.
"""

from __future__ import annotations

import numpy as np

from .d3q19 import C, W, OPP, Q


def _fold(terms):
    acc = None
    for t in terms:
        acc = t if acc is None else acc + t
    return acc


def _signed(c, v):
    return v if c > 0 else -v


def density_and_momentum(f):
    """rho = sum_q f_q and j = sum_q c_q f_q (moments of the PDFs, Sect. 2).

    Left folds in ascending q; for j, terms with c_qa = 0 are skipped.
    """
    rho = _fold(f[q] for q in range(Q))
    j = [_fold(_signed(C[q, a], f[q]) for q in range(Q) if C[q, a] != 0)
         for a in range(3)]
    return rho, j


def macroscopic(f):
    """Density and velocity u = j / rho of the PDFs ``f`` (arrays)."""
    rho, j = density_and_momentum(f)
    return rho, [j[a] / rho for a in range(3)]


def _cdot(q, v):
    """c_q . v folded over x, y, z with zero-coefficient terms skipped."""
    terms = [_signed(C[q, a], v[a]) for a in range(3) if C[q, a] != 0]
    return 0.0 if not terms else _fold(terms)


def equilibrium(rho, u):
    """Second-order equilibrium feq_q(rho, u), returned as a (19, ...) array."""
    rho = np.asarray(rho, dtype=np.float64)
    u = [np.asarray(u[a], dtype=np.float64) for a in range(3)]
    usq = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]
    out = np.empty((Q,) + rho.shape, dtype=np.float64)
    for q in range(Q):
        cu = _cdot(q, u)
        out[q] = (W[q] * rho) * (((1.0 + 3.0 * cu) + (4.5 * cu) * cu) - 1.5 * usq)
    return out


def force_source(force):
    """S_q = 3 w_q (c_q . F) for a constant force density F (19 floats)."""
    force = [float(x) for x in force]
    return [(3.0 * W[q]) * _cdot(q, force) for q in range(Q)]


def trt_omega_minus(tau, magic):
    """Relaxation rate of the antisymmetric part for a TRT magic parameter
    Lambda = (1/omega_plus - 1/2)(1/omega_minus - 1/2)."""
    return 1.0 / (magic / (tau - 0.5) + 0.5)


def collide(f, tau, force, magic=None, ns=None):
    """Collision with body force, returns the post-collision PDFs.

    ``ns`` (array of per-site solid fractions in [0, 1], BGK only) applies
    partial bounce-back: post_q = (1 - ns) f*_q + ns f_qbar.

    BGK (``magic`` None): f*_q = (f_q - omega (f_q - feq_q)) + S_q.
    TRT (Sect. 2; two relaxation times, ``magic`` = Lambda): with
    f+- = (f_q +- f_qbar)/2 and feq+- the symmetric and antisymmetric
    equilibrium parts, f*_q = ((f_q - w+ (f+ - feq+)) - w- (f- - feq-)) + S_q,
    w+ = 1/tau, w- from Lambda.
    """
    omega = 1.0 / tau
    rho, u = macroscopic(f)
    usq = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]
    S = force_source(force)
    out = np.empty_like(f)
    if magic is None:
        for q in range(Q):
            cu = _cdot(q, u)
            feq = (W[q] * rho) * (((1.0 + 3.0 * cu) + (4.5 * cu) * cu) - 1.5 * usq)
            out[q] = (f[q] - omega * (f[q] - feq)) + S[q]
        if ns is not None:
            out = np.stack([((1.0 - ns) * out[q]) + (ns * f[OPP[q]]) for q in range(Q)])
        return out
    if ns is not None:
        raise ValueError("partial bounce-back is defined for BGK only")
    omega_m = trt_omega_minus(tau, magic)
    for q in range(Q):
        qb = OPP[q]
        cu = _cdot(q, u)
        wr = W[q] * rho
        ep = wr * ((1.0 + (4.5 * cu) * cu) - 1.5 * usq)
        em = wr * (3.0 * cu)
        fp = (f[q] + f[qb]) * 0.5
        fm = (f[q] - f[qb]) * 0.5
        out[q] = ((f[q] - omega * (fp - ep)) - omega_m * (fm - em)) + S[q]
    return out


def upstream_solid(solid, periodic, q):
    """Mask of sites x whose upstream site x - c_q is solid or outside the box."""
    up = np.asarray(solid, dtype=bool)
    for a in range(3):
        s = int(C[q, a])
        if s == 0:
            continue
        up = np.roll(up, s, axis=a)
        if not periodic[a]:
            idx = [slice(None)] * 3
            idx[a] = 0 if s > 0 else -1
            up[tuple(idx)] = True
    return up


def stream(fstar, solid, periodic):
    """Propagation of eq. (1) with halfway bounce-back.

    f_q(x, t+1) = f*_q(x - c_q) if x - c_q is a fluid site of the lattice,
    else f*_qbar(x), where qbar is the direction opposite to q. Solid sites
    are reset to the rest weights (their values are never read).
    """
    solid = np.asarray(solid, dtype=bool)
    out = np.empty_like(fstar)
    for q in range(Q):
        pulled = fstar[q]
        for a in range(3):
            if C[q, a] != 0:
                pulled = np.roll(pulled, int(C[q, a]), axis=a)
        out[q] = np.where(upstream_solid(solid, periodic, q), fstar[OPP[q]], pulled)
    for q in range(Q):
        out[q][solid] = W[q]
    return out


def step(f, solid, periodic, tau, force, magic=None, ns=None):
    """One time step of eq. (1): collide, then propagate."""
    with np.errstate(all="ignore"):
        return stream(collide(f, tau, force, magic, ns), solid, periodic)


def initial_state(solid, rho=None, u=None):
    """f(0) = feq(rho, u); rest state (rho=1, u=0) where fields are omitted."""
    solid = np.asarray(solid, dtype=bool)
    if rho is None:
        rho = np.ones(solid.shape)
    if u is None:
        u = np.zeros((3,) + solid.shape)
    f = equilibrium(rho, u)
    for q in range(Q):
        f[q][solid] = W[q]
    return f


def run(solid, periodic, tau, force, steps, rho=None, u=None, f0=None, magic=None, ns=None):
    """Advance f(0) by ``steps`` time steps; returns f(steps) as (19, nx, ny, nz)."""
    f = initial_state(solid, rho, u) if f0 is None else np.array(f0, dtype=np.float64)
    for _ in range(steps):
        f = step(f, solid, periodic, tau, force, magic, ns)
    return f


def cone_sites(solid, periodic, tau, force, steps, rho, u, sites, magic=None):
    """PDFs f(steps) at selected fluid sites of a lattice too large to run whole.

    After k steps a site depends only on sites within k lattice units
    (Chebyshev distance) of it, so each requested site is computed on a crop
    of half-width k + 1 around it, in which everything outside the crop is
    treated as solid. Returns an array of shape (len(sites), 19).
    """
    solid = np.asarray(solid, dtype=bool)
    shape = solid.shape
    h = int(steps) + 1
    out = np.empty((len(sites), Q), dtype=np.float64)
    for i, s in enumerate(sites):
        idx, outside = [], []
        for a in range(3):
            v = int(s[a]) + np.arange(-h, h + 1)
            if periodic[a]:
                o = np.zeros(v.shape, bool)
                v = np.mod(v, shape[a])
            else:
                o = (v < 0) | (v >= shape[a])
                v = np.clip(v, 0, shape[a] - 1)
            idx.append(v)
            outside.append(o)
        ix = np.ix_(*idx)
        crop = solid[ix] | (outside[0][:, None, None] | outside[1][None, :, None]
                            | outside[2][None, None, :])
        if crop[h, h, h]:
            raise ValueError("cone_sites: site %r is solid" % (tuple(s),))
        f = initial_state(crop, rho[ix], [u[a][ix] for a in range(3)])
        for _ in range(int(steps)):
            f = step(f, crop, (False, False, False), tau, force, magic)
        out[i] = f[:, h, h, h]
    return out
