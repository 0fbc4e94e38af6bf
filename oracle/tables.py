"""Sparse-lattice integer tables (oracle; test infrastructure only).

Sect. 1 and Sect. 4: only fluid nodes are stored, as a 1-D vector whose order
is fixed by an enumeration function; neighbours are reached through an
adjacency list of 18 four-byte indices per node (the rest direction needs no
entry). Sect. 4.1: reduced indirect addressing (RIA) skips the index load of
a node whose access pattern equals that of the previous node shifted by one;
the lengths of such runs are stored run-length coded. Sect. 5.6 and Sect. 6:
enumeration by lexicographic sorting (LS) with a blocking factor B, or by a
space-filling curve.

Readings where the paper is silent:

* LS axis order: x slowest, z fastest (C order of the voxel box).
* Blocking factor B: the box is tiled by B x B x B blocks visited in LS order;
  inside a block voxels are visited in LS order. B = 0 means no blocking.
* Space-filling curve: Morton order (bit interleaving, x the most significant
  bit of each triple); the paper uses a Hilbert curve.
* Adjacency entry for direction q (q = 1..18) of node n: the node at the
  upstream site x_n - c_q (periodic wrap on periodic axes), or -1 when that
  site is solid or outside the box (pull scheme, Sect. 4).
* Run rule: node n > 0 continues the run of node n - 1 iff for every q the
  entry of n is the entry of n - 1 plus one, or both entries are -1.
* Per-direction runs (a GPU encoding of the same idea, not in the paper):
  the run rule applied to one direction q at a time. A node starts a run of
  the paper's rule iff it starts a run of at least one direction.
"""

from __future__ import annotations

import numpy as np

from .d3q19 import C

WAVE = 64
NO_NEIGHBOUR = -1
DELTA_SOLID = np.iinfo(np.int32).min


def fluid_voxels(mask):
    """Linear voxel ids (x*ny + y)*nz + z of the fluid voxels, ascending."""
    return np.flatnonzero(np.asarray(mask).ravel() == 0).astype(np.int64)


def _coords(vid, shape):
    nx, ny, nz = shape
    return vid // (ny * nz), (vid // nz) % ny, vid % nz


def lex_keys(vid, shape, block):
    """Sort keys of LS with blocking factor ``block`` (0: no blocking)."""
    nx, ny, nz = shape
    B = int(block)
    if B <= 0 or B >= max(shape):
        return vid.copy()
    x, y, z = _coords(vid, shape)
    nby = -(-ny // B)
    nbz = -(-nz // B)
    blk = ((x // B) * nby + (y // B)) * nbz + (z // B)
    inner = ((x % B) * B + (y % B)) * B + (z % B)
    return blk * (B * B * B) + inner


def morton_keys(vid, shape):
    """Morton keys: bits of x, y, z interleaved, x most significant per triple."""
    x, y, z = _coords(vid, shape)
    key = np.zeros(vid.shape, dtype=np.int64)
    for b in range(21):
        key |= ((x >> b) & 1) << (3 * b + 2)
        key |= ((y >> b) & 1) << (3 * b + 1)
        key |= ((z >> b) & 1) << (3 * b)
    return key


def hilbert_keys(vid, shape):
    """3-D Hilbert curve index of each voxel (Sect. 5.6 uses a Hilbert curve).

    Skilling's transpose method on the bounding 2^b cube: undo the excess
    rotations and reflections from the top bit down, Gray-encode, then read
    the bits of (x, y, z) interleaved, x most significant per triple.
    """
    b = max(1, int(np.ceil(np.log2(max(max(shape), 2)))))
    x, y, z = _coords(vid, shape)
    X = [x.copy(), y.copy(), z.copy()]
    Qb = 1 << (b - 1)
    while Qb > 1:
        P = Qb - 1
        for i in range(3):
            hit = (X[i] & Qb) != 0
            inv = X[0] ^ P
            t = (X[0] ^ X[i]) & P
            X0_new = np.where(hit, inv, X[0] ^ t)
            if i > 0:
                X[i] = np.where(hit, X[i], X[i] ^ t)
            X[0] = X0_new
        Qb >>= 1
    for i in range(1, 3):
        X[i] = X[i] ^ X[i - 1]
    t = np.zeros_like(X[0])
    Qb = 1 << (b - 1)
    while Qb > 1:
        t = np.where((X[2] & Qb) != 0, t ^ (Qb - 1), t)
        Qb >>= 1
    X = [X[i] ^ t for i in range(3)]
    key = np.zeros(vid.shape, dtype=np.int64)
    for bit in range(b - 1, -1, -1):
        for i in range(3):
            key = (key << 1) | ((X[i] >> bit) & 1)
    return key


def enumerate_nodes(mask, order="lex", block=0):
    """Fluid-node enumeration: node n sits at voxel ``node_voxel[n]`` (int32).

    order: "lex" (LS with blocking factor ``block``), "morton", "hilbert", or
    "hilbert_ls": the two-stage renumbering of Sect. 6.1 -- the Hilbert order
    is cut into ``block`` contiguous chunks of ceil(N / block) nodes (the
    partitions), and every chunk is re-enumerated by plain LS.
    """
    mask = np.asarray(mask)
    vid = fluid_voxels(mask)
    if order == "lex":
        key = lex_keys(vid, mask.shape, block)
    elif order == "morton":
        key = morton_keys(vid, mask.shape)
    elif order in ("hilbert", "hilbert_ls"):
        key = hilbert_keys(vid, mask.shape)
    else:
        raise ValueError(order)
    perm = np.argsort(key, kind="stable")
    nodes = vid[perm]
    if order == "hilbert_ls":
        parts = max(int(block), 1)
        chunk = -(-len(nodes) // parts) if len(nodes) else 1
        part = np.arange(len(nodes)) // chunk
        nodes = nodes[np.lexsort((nodes, part))]
    return nodes.astype(np.int32)


def adjacency(mask, periodic, node_voxel):
    """Adjacency list adj[q-1, n] (q = 1..18), int32, -1 for solid/outside."""
    mask = np.asarray(mask)
    shape = mask.shape
    nvox = mask.size
    node_of = np.full(nvox, NO_NEIGHBOUR, dtype=np.int64)
    node_of[node_voxel.astype(np.int64)] = np.arange(len(node_voxel))
    x, y, z = _coords(node_voxel.astype(np.int64), shape)
    adj = np.empty((18, len(node_voxel)), dtype=np.int32)
    for q in range(1, 19):
        up = [x - C[q, 0], y - C[q, 1], z - C[q, 2]]
        valid = np.ones(len(node_voxel), dtype=bool)
        for a in range(3):
            if periodic[a]:
                up[a] = np.mod(up[a], shape[a])
            else:
                valid &= (up[a] >= 0) & (up[a] < shape[a])
                up[a] = np.clip(up[a], 0, shape[a] - 1)
        v = (up[0] * shape[1] + up[1]) * shape[2] + up[2]
        nb = node_of[v]
        nb[~valid] = NO_NEIGHBOUR
        adj[q - 1] = nb
    return adj


def run_heads(adj):
    """Boolean vector: node n starts a run of "shifted by one" access patterns."""
    n = adj.shape[1]
    head = np.ones(n, dtype=bool)
    if n > 1:
        prev, cur = adj[:, :-1].astype(np.int64), adj[:, 1:].astype(np.int64)
        same = ((prev >= 0) & (cur == prev + 1)) | ((prev < 0) & (cur < 0))
        head[1:] = ~np.all(same, axis=0)
    return head


def run_starts(adj):
    """run_start[R+1]: first node of each run, then N (int32)."""
    head = run_heads(adj)
    return np.concatenate([np.flatnonzero(head), [adj.shape[1]]]).astype(np.int32)


def wave_tables(adj, run_start, wave=WAVE):
    """Per-wavefront RIA encoding.

    run_delta[q-1, r] = adj[q-1, head_r] - head_r (DELTA_SOLID for -1):
    inside run r the entry of node n is n + run_delta[q-1, r].
    head_bits[w] has bit l set iff node wave*w + l starts a run.
    run_base[w] = (number of run heads below node wave*w) - 1, so node
    wave*w + l lies in run run_base[w] + popcount(head_bits[w] & bits 0..l).
    """
    n = adj.shape[1]
    heads = run_start[:-1].astype(np.int64)
    a = adj[:, heads].astype(np.int64)
    delta = np.where(a >= 0, a - heads[None, :], DELTA_SOLID).astype(np.int32)
    nw = -(-n // wave)
    head = np.zeros(nw * wave, dtype=bool)
    head[heads] = True
    hb = head.reshape(nw, wave)
    bits = np.zeros(nw, dtype=np.uint64)
    for l in range(wave):
        bits |= hb[:, l].astype(np.uint64) << np.uint64(l)
    per_wave = hb.sum(axis=1)
    base = (np.cumsum(per_wave) - per_wave - 1).astype(np.int32)
    return delta, bits, base


def direction_heads(adj):
    """Boolean (18, N): node n starts a run of direction q (the run rule of
    Sect. 4.1 applied to the entries of direction q alone)."""
    q, n = adj.shape
    head = np.ones((q, n), dtype=bool)
    if n > 1:
        prev, cur = adj[:, :-1].astype(np.int64), adj[:, 1:].astype(np.int64)
        same = ((prev >= 0) & (cur == prev + 1)) | ((prev < 0) & (cur < 0))
        head[:, 1:] = ~same
    return head


def direction_tables(adj, wave=WAVE):
    """Per-direction, per-wavefront RIA encoding.

    The runs of direction q (q = 1..18) are numbered consecutively after those
    of directions 1..q-1. dir_delta[r] = adj[q-1, head_r] - head_r (DELTA_SOLID
    for -1) for run r, whose first node is head_r. For wave w and direction q
    (row w, column q-1 of the (W, 18) tables):
      dir_bits  has bit l set iff node wave*w + l starts a run of direction q;
      dir_base  = (index of the first run of direction q) + (number of
                  direction-q run heads below node wave*w) - 1.
    Node wave*w + l then lies in run dir_base + popcount(dir_bits & bits 0..l)
    of its direction, and its entry is the node index plus that run's delta.
    """
    nq, n = adj.shape
    head = direction_heads(adj)
    nw = -(-n // wave)
    deltas, bits, base = [], np.zeros((nw, nq), dtype=np.uint64), np.zeros((nw, nq), dtype=np.int64)
    first = 0
    for q in range(nq):
        h = np.flatnonzero(head[q])
        a = adj[q, h].astype(np.int64)
        deltas.append(np.where(a >= 0, a - h, DELTA_SOLID))
        hw = np.zeros(nw * wave, dtype=bool)
        hw[h] = True
        hw = hw.reshape(nw, wave)
        for l in range(wave):
            bits[:, q] |= hw[:, l].astype(np.uint64) << np.uint64(l)
        per_wave = hw.sum(axis=1)
        base[:, q] = first + np.cumsum(per_wave) - per_wave - 1
        first += len(h)
    delta = np.concatenate(deltas).astype(np.int32) if nq else np.zeros(0, np.int32)
    return delta, bits, base.astype(np.int32)


def simd_fraction(run_start, vector=4):
    """Share of nodes updatable in SIMD chunks of ``vector`` inside runs (Sect. 4.2)."""
    lengths = np.diff(run_start.astype(np.int64))
    return float(np.sum((lengths // vector) * vector)) / float(run_start[-1])


def build(mask, periodic, order="lex", block=0):
    """All tables for one lattice: dict with node_voxel, adj, run_start and wave tables."""
    nodes = enumerate_nodes(mask, order, block)
    adj = adjacency(mask, periodic, nodes)
    rs = run_starts(adj)
    delta, bits, base = wave_tables(adj, rs)
    return dict(node_voxel=nodes, adj=adj, run_start=rs, run_delta=delta,
                head_bits=bits, run_base=base)
