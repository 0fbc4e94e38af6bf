"""Sparse-lattice propagation steps on the oracle's tables (test infrastructure).

Executes the two propagation patterns of Sect. 4 with plain numpy gathers and
scatters over all fluid nodes at once, using ``oracle.tables`` and the dense
oracle's collision. The tests require these to equal the dense solver
bitwise, which ties the adjacency direction and the slot algebra below to the
physics pinned for the dense solver.

PDF storage is ``F[q, n]`` (one stream per direction, Sect. 4.3).

OS-NT (Sect. 4, pull scheme): grid G holds post-collision values f*_q(n) of
the previous step. Node n pulls f_q from slot (q, adj_q(n)) of its upstream
neighbour, or from its own slot (qbar, n) when that neighbour is solid
(bounce-back), collides and writes f*_q to (q, n) of the other grid.

AA pattern (Sect. 4): one grid. Even steps (t = 0, 2, ...) read (q, n) and
write f*_q to (qbar, n). Odd steps read f_q from
L_q(n) = (qbar, adj_q(n)), or (q, n) for a solid upstream site, and write
f*_q to L_qbar(n), the slot the node read f_qbar from; L is a bijection on
slots, so the update is in place. After an even number of steps the grid
holds f(t) in natural order.
"""

from __future__ import annotations

import numpy as np

from .d3q19 import OPP, Q
from . import dense


def _slots(adj, q, n_idx, ldf, aa):
    """Flat slot index of f_q for node n (AA: L_q(n); OS-NT: pull slot)."""
    if q == 0:
        return n_idx.astype(np.int64)
    a = adj[q - 1].astype(np.int64)
    fluid = a >= 0
    if aa:
        return np.where(fluid, OPP[q] * ldf + a, q * ldf + n_idx)
    return np.where(fluid, q * ldf + a, OPP[q] * ldf + n_idx)


def aa_even(F, n, tau, force):
    fs = dense.collide(F[:, :n].copy(), tau, force)
    for q in range(Q):
        F[OPP[q], :n] = fs[q]


def aa_odd(F, adj, tau, force):
    ldf = F.shape[1]
    n_idx = np.arange(adj.shape[1], dtype=np.int64)
    flat = F.reshape(-1)
    slots = [_slots(adj, q, n_idx, ldf, True) for q in range(Q)]
    f = np.stack([flat[slots[q]] for q in range(Q)])
    fs = dense.collide(f, tau, force)
    for q in range(Q):
        flat[slots[OPP[q]]] = fs[q]


def osnt(G, H, adj, tau, force):
    ldf = G.shape[1]
    n = adj.shape[1]
    n_idx = np.arange(n, dtype=np.int64)
    flat = G.reshape(-1)
    f = np.stack([flat[_slots(adj, q, n_idx, ldf, False)] for q in range(Q)])
    H[:, :n] = dense.collide(f, tau, force)


def aa_pdfs(F, adj, t):
    """f(t) in natural order from the AA grid at time t."""
    if t % 2 == 0:
        return F[:, :adj.shape[1]].copy()
    ldf = F.shape[1]
    n_idx = np.arange(adj.shape[1], dtype=np.int64)
    flat = F.reshape(-1)
    return np.stack([flat[_slots(adj, q, n_idx, ldf, True)] for q in range(Q)])


def osnt_pdfs(G, adj):
    """f(t) in natural order from an OS-NT grid holding f*(t-1)."""
    ldf = G.shape[1]
    n_idx = np.arange(adj.shape[1], dtype=np.int64)
    flat = G.reshape(-1)
    return np.stack([flat[_slots(adj, q, n_idx, ldf, False)] for q in range(Q)])


def osnt_from_pdfs(f, adj, ldf=None):
    """Grid G with G pulled through the stream equal to f (inverse stream)."""
    n = adj.shape[1]
    ldf = n if ldf is None else ldf
    G = np.zeros((Q, ldf))
    flat = G.reshape(-1)
    n_idx = np.arange(n, dtype=np.int64)
    for q in range(Q):
        flat[_slots(adj, q, n_idx, ldf, False)] = f[q]
    return G
