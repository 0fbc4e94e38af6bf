"""Pins for the oracle's sparse-lattice tables: the paper's worked channel
example (Sect. 5.1, Table 2), its printed model numbers (Sect. 4, Tables 3
and 4), and brute-force definitions on tiny random masks."""
import json
import os
from itertools import product

import numpy as np
import pytest

from lbm_inputs import channel_mask
from oracle import tables, model
from oracle.d3q19 import C

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


# ---------------------------------------------------------------- model ----

def test_model_constants_and_bounds():
    m = GOLD["model"]
    assert model.D_PDF == m["D_pdf_B"] and model.D_IDX == m["D_idx_B"] and model.D_BLOCK == m["D_block_B"]
    assert model.b_osnt() == m["B_osnt"] and model.b_aa() == m["B_aa"]
    assert [model.b_osnt_r(0, 1), model.b_osnt_r(1, 1)] == m["B_osnt_r_bounds"]
    assert [model.b_aa_r(0, 1), model.b_aa_r(1, 1)] == m["B_aa_r_bounds"]


def test_roofline_recipe_reproduces_table4():
    # Table 4 = Table 3 bandwidth / Table 2 loop balance, CNT-19A for OS-NT
    # and U-19A for AA. Table 2 prints loop balances rounded to integers, so
    # each printed prediction must lie in bw / [B_l + 1/2, B_l - 1/2] up to
    # its own rounding to 0.1.
    bench = {"OS-NT": "CNT-19A", "OS-NT-R": "CNT-19A", "AA": "U-19A", "AA-R": "U-19A"}
    for geo in ("channel", "fixed_bed"):
        for f in ("1.2GHz", "2.6GHz"):
            for k, b in bench.items():
                bw = GOLD["table3_bandwidth_GBs"][f][b]
                bl = GOLD["table2_loop_balance"][geo][k]
                lo = model.roofline_mflups(bw, bl + 0.5) - 0.05
                hi = model.roofline_mflups(bw, bl - 0.5) + 0.05
                assert lo <= GOLD["table4_roofline_MFLUPs"][geo][f][k] <= hi, (geo, f, k)


def test_large_scale_sizes_imply_18_index_entries():
    # Sect. 6: the PDFs need 4.8 TiB and the adjacency list 2.3 TiB (both
    # rounded to 0.1). Their ratio fixes the index bytes per node relative to
    # the 19 * 8 B of PDFs: 18 four-byte entries fit, 19 do not.
    ls = GOLD["large_scale"]
    lo = (ls["adjacency_TiB"] - 0.05) / (ls["pdf_TiB"] + 0.05)
    hi = (ls["adjacency_TiB"] + 0.05) / (ls["pdf_TiB"] - 0.05)
    assert lo <= model.D_IDX / (19 * 8) <= hi
    assert not lo <= (19 * 4) / (19 * 8) <= hi
    n = ls["pdf_TiB"] * 2.0 ** 40 / (19 * 8)
    assert abs(n - ls["fluid_nodes"]) / ls["fluid_nodes"] < 0.05


# -------------------------------------------------------- channel example --

@pytest.fixture(scope="module")
def channel_tables():
    mask = channel_mask(*GOLD["channel"]["shape"])
    nodes = tables.enumerate_nodes(mask, "lex", 1)
    adj = tables.adjacency(mask, (True, False, False), nodes)
    return mask, nodes, adj, tables.run_starts(adj)


def test_channel_matches_table2(channel_tables):
    mask, nodes, adj, rs = channel_tables
    n, r = len(nodes), len(rs) - 1
    assert abs(n - GOLD["channel"]["fluid_nodes_approx"]) / n < 0.01
    t2 = GOLD["table2_loop_balance"]["channel"]
    assert model.b_osnt() == t2["OS-NT"] and model.b_aa() == t2["AA"]
    assert round(model.b_osnt_r(r, n)) == t2["OS-NT-R"]
    assert round(model.b_aa_r(r, n)) == t2["AA-R"]
    assert round(100 * tables.simd_fraction(rs, 4)) == GOLD["channel"]["simd_percent"]


def test_channel_direction_runs_by_hand(channel_tables):
    # 500 x 100 x 100 channel, fluid y, z in 1..98, periodic x, LS (z
    # fastest), pull entries at x - c_q. Counted by hand per direction:
    # * c_z != 0, c_y = 0: the wall side of each z-line reads -1, so every
    #   line has 2 heads (where the entries turn -1 and where they turn
    #   fluid): 2 * 98 * 500.
    # * c_z = 0, c_y != 0: the y-line next to the wall reads -1 in every
    #   plane: 2 heads per plane.
    # * only c_x: one offset per plane pair, broken once by the wrap: 2.
    # * c_y and c_z both nonzero: per plane, the all-wall y-line adds one
    #   head and each other y-line two, except where the all-wall line
    #   continues a -1 run left by the previous line: 194 per plane; for
    #   (0,+1,-1) and (0,-1,+1) the all-wall line follows a -1 entry of the
    #   previous plane, so only node 0 adds a head there: 97,000 + 1.
    _, _, adj, _ = channel_tables
    heads = tables.direction_heads(adj).sum(axis=1)
    for q in range(1, 19):
        cx, cy, cz = C[q]
        if cz and not cy:
            want = 98_000
        elif cy and not cz:
            want = 1_000
        elif not cy and not cz:
            want = 2
        else:
            want = 97_001 if cy != cz else 97_000
        assert heads[q - 1] == want, (q, heads[q - 1], want)


def test_channel_blocking_100_equals_1():
    # Sect. 5.6: on the 100-wide channel, B = 1 and B = 100 give the same order
    mask = channel_mask(40, 100, 100)
    a = tables.enumerate_nodes(mask, "lex", 1)
    b = tables.enumerate_nodes(mask, "lex", 100)
    assert np.array_equal(a, b)
    c = tables.enumerate_nodes(mask, "lex", 10)
    assert not np.array_equal(a, c)


def test_channel_other_fastest_axis_contradicts_table2():
    # evidence for the LS axis reading: with x (periodic, 500 long) fastest,
    # the OS-NT-R loop balance would round to 304 or 305, not 306
    mask = np.ascontiguousarray(channel_mask(500, 100, 100).transpose(2, 1, 0))
    nodes = tables.enumerate_nodes(mask, "lex", 1)
    adj = tables.adjacency(mask, (False, False, True), nodes)
    r = len(tables.run_starts(adj)) - 1
    assert round(model.b_osnt_r(r, len(nodes))) != GOLD["table2_loop_balance"]["channel"]["OS-NT-R"]


# ---------------------------------------------------------- brute force ----

def tiny_masks():
    rng = np.random.default_rng(11)
    out = []
    for shape in [(3, 3, 3), (4, 3, 5), (5, 6, 4), (7, 5, 6)]:
        for frac in (0.0, 0.3, 0.6):
            out.append((rng.random(shape) < frac).astype(np.uint8))
    return out


def brute_nodes(mask, order, block):
    nx, ny, nz = mask.shape
    cells = [(x, y, z) for x in range(nx) for y in range(ny) for z in range(nz) if mask[x, y, z] == 0]
    if order == "morton":
        def key(c):
            k = 0
            for b in range(8):
                for a, sh in ((0, 2), (1, 1), (2, 0)):
                    k |= ((c[a] >> b) & 1) << (3 * b + sh)
            return k
    elif block == 0:
        key = lambda c: c
    else:
        B = block
        key = lambda c: ((c[0] // B, c[1] // B, c[2] // B), (c[0] % B, c[1] % B, c[2] % B))
    cells.sort(key=key)
    return [(x * ny + y) * nz + z for x, y, z in cells]


@pytest.mark.parametrize("order,block", [("lex", 0), ("lex", 1), ("lex", 2), ("lex", 3), ("morton", 0)])
def test_enumeration_brute_force(order, block):
    for mask in tiny_masks():
        assert tables.enumerate_nodes(mask, order, block).tolist() == brute_nodes(mask, order, block)


@pytest.mark.parametrize("periodic", list(product((False, True), repeat=3)))
def test_adjacency_brute_force(periodic):
    for mask in tiny_masks():
        nodes = tables.enumerate_nodes(mask, "lex", 2)
        adj = tables.adjacency(mask, periodic, nodes)
        nx, ny, nz = mask.shape
        where = {int(v): i for i, v in enumerate(nodes)}
        assert adj.shape == (18, len(nodes)) and adj.dtype == np.int32
        for i, v in enumerate(nodes):
            x = [int(v) // (ny * nz), (int(v) // nz) % ny, int(v) % nz]
            for q in range(1, 19):
                up = [x[a] - int(C[q, a]) for a in range(3)]
                ok = True
                for a in range(3):
                    if periodic[a]:
                        up[a] %= mask.shape[a]
                    elif not 0 <= up[a] < mask.shape[a]:
                        ok = False
                want = -1
                if ok and mask[up[0], up[1], up[2]] == 0:
                    want = where[(up[0] * ny + up[1]) * nz + up[2]]
                assert adj[q - 1, i] == want


def brute_heads(adj):
    n = adj.shape[1]
    heads = []
    for i in range(n):
        if i == 0:
            heads.append(0)
            continue
        cont = all((adj[q, i - 1] >= 0 and adj[q, i] == adj[q, i - 1] + 1) or
                   (adj[q, i - 1] < 0 and adj[q, i] < 0) for q in range(18))
        if not cont:
            heads.append(i)
    return heads + [n]


@pytest.mark.parametrize("order,block", [("lex", 0), ("lex", 2), ("morton", 0)])
def test_runs_and_wave_tables_brute_force(order, block):
    for mask in tiny_masks() + [channel_mask(6, 9, 70)]:
        if mask.min() == 1:
            continue
        periodic = (True, False, True)
        nodes = tables.enumerate_nodes(mask, order, block)
        adj = tables.adjacency(mask, periodic, nodes)
        rs = tables.run_starts(adj)
        assert rs.tolist() == brute_heads(adj)
        delta, bits, base = tables.wave_tables(adj, rs, wave=8)
        # decode every node from the wave tables alone
        for i in range(adj.shape[1]):
            w, l = divmod(i, 8)
            b = int(bits[w])
            r = int(base[w]) + bin(b & ((2 << l) - 1)).count("1")
            assert rs[r] <= i < rs[r + 1]
            for q in range(18):
                d = int(delta[q, r])
                assert (adj[q, i] == -1) if d == tables.DELTA_SOLID else (adj[q, i] == i + d)


@pytest.mark.parametrize("order,block", [("lex", 0), ("lex", 2), ("morton", 0)])
def test_direction_tables_brute_force(order, block):
    # per-direction runs: the run rule for one direction at a time; decoding
    # every entry from the tables alone must give the adjacency list back
    for mask in tiny_masks() + [channel_mask(6, 9, 70)]:
        if mask.min() == 1:
            continue
        nodes = tables.enumerate_nodes(mask, order, block)
        adj = tables.adjacency(mask, (True, False, True), nodes)
        n = adj.shape[1]
        heads = tables.direction_heads(adj)
        for q in range(18):
            want = [0] + [i for i in range(1, n)
                          if not ((adj[q, i - 1] >= 0 and adj[q, i] == adj[q, i - 1] + 1) or
                                  (adj[q, i - 1] < 0 and adj[q, i] < 0))]
            assert np.flatnonzero(heads[q]).tolist() == want
        # the paper's run heads are the nodes where at least one direction breaks
        assert np.flatnonzero(heads.any(axis=0)).tolist() == brute_heads(adj)[:-1]
        delta, bits, base = tables.direction_tables(adj, wave=8)
        assert len(delta) == heads.sum()
        for i in range(n):
            w, l = divmod(i, 8)
            for q in range(18):
                r = int(base[w, q]) + bin(int(bits[w, q]) & ((2 << l) - 1)).count("1")
                assert heads[:q].sum() <= r < heads[:q + 1].sum()
                d = int(delta[r])
                assert (adj[q, i] == -1) if d == tables.DELTA_SOLID else (adj[q, i] == i + d)


def test_direction_runs_of_open_periodic_box():
    # 4^3 fully fluid, all axes periodic, x slowest: the upstream entry of
    # direction q wraps once per line along every axis c_q moves on. Per
    # direction that breaks runs twice per z-line (c_z != 0: 2 * 16), twice
    # per x-plane (c_z = 0, c_y != 0: 2 * 4) or twice in the box (only c_x).
    t = tables.build(np.zeros((4, 4, 4), np.uint8), (True, True, True))
    heads = tables.direction_heads(t["adj"])
    for q in range(1, 19):
        want = 32 if C[q][2] else (8 if C[q][1] else 2)
        assert heads[q - 1].sum() == want, q


def test_morton_has_no_runs_in_open_box():
    # every step of a Morton curve changes more than one coordinate bit, so
    # no node continues a run on an all-fluid periodic box
    mask = np.zeros((8, 8, 8), np.uint8)
    t = tables.build(mask, (True, True, True), "morton")
    assert len(t["run_start"]) - 1 == 8 * 8 * 8


# --------------------------------------------------------------- Hilbert ----

@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_hilbert_curve_is_a_face_connected_bijection(k):
    # the defining property of a Hilbert curve on a 2^k cube: it visits every
    # cell once and consecutive cells share a face
    n = 1 << k
    mask = np.zeros((n, n, n), np.uint8)
    nodes = tables.enumerate_nodes(mask, "hilbert").astype(np.int64)
    assert sorted(nodes.tolist()) == list(range(n ** 3))
    xyz = np.stack([nodes // (n * n), (nodes // n) % n, nodes % n], 1)
    assert tuple(xyz[0]) == (0, 0, 0)
    steps = np.abs(np.diff(xyz, axis=0)).sum(1)
    assert np.all(steps == 1)
    # the curve of a 2^k cube ends on a corner adjacent to its start corner
    assert np.count_nonzero(xyz[-1]) == 1 and xyz[-1].max() == n - 1


def test_hilbert_sub_box_keeps_curve_order():
    # a box inside the bounding cube takes the cube's curve order
    n = 8
    full = tables.enumerate_nodes(np.zeros((n, n, n), np.uint8), "hilbert").astype(np.int64)
    mask = np.ones((n, n, n), np.uint8)
    mask[:5, :6, :7] = 0
    sub = tables.enumerate_nodes(mask[:5, :6, :7], "hilbert").astype(np.int64)
    xyz_sub = np.stack([sub // 42, (sub // 7) % 6, sub % 7], 1)
    xyz_full = [tuple(v) for v in np.stack([full // 64, (full // 8) % 8, full % 8], 1)
                if v[0] < 5 and v[1] < 6 and v[2] < 7]
    assert [tuple(v) for v in xyz_sub] == xyz_full


def test_hilbert_ls_partitions():
    mask = (np.random.default_rng(5).random((9, 7, 8)) < 0.3).astype(np.uint8)
    h = tables.enumerate_nodes(mask, "hilbert")
    for parts in (1, 3, 4):
        r = tables.enumerate_nodes(mask, "hilbert_ls", parts)
        chunk = -(-len(h) // parts)
        for p in range(parts):
            a, b = p * chunk, min(len(h), (p + 1) * chunk)
            # same set of voxels per partition, LS order inside
            assert sorted(r[a:b].tolist()) == sorted(h[a:b].tolist())
            assert np.all(np.diff(r[a:b]) > 0)
