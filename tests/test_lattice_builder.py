"""The C++ lattice builder (product path) must reproduce the oracle's integer
tables bit for bit: enumeration, adjacency, runs, wave tables and the
per-direction run tables. Runs on the CPU (the builder is host code of the
library)."""
import ctypes
import os
import re
from itertools import product

import numpy as np
import pytest

from lbm_inputs import channel_mask, rsa_spheres, foam, relaxed_spheres
from oracle import tables

lattice_mod = pytest.importorskip("paper_1410_0412_amd.lattice")
from paper_1410_0412_amd import Lattice, LbmError, _capi  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def compare(mask, periodic, order, block):
    L = Lattice(mask, periodic, order, block)
    ref = tables.build(mask, periodic, order, block)
    assert L.n_fluid == len(ref["node_voxel"])
    assert np.array_equal(L.node_voxel(), ref["node_voxel"])
    assert np.array_equal(L.adjacency(), ref["adj"])
    assert np.array_equal(L.run_start(), ref["run_start"])
    d, b, base = L.wave_tables()
    assert np.array_equal(d, ref["run_delta"])
    assert np.array_equal(b, ref["head_bits"])
    assert np.array_equal(base, ref["run_base"])
    dd, db, dbase = L.direction_tables()
    rd, rb, rbase = tables.direction_tables(ref["adj"])
    assert L.n_direction_runs == len(rd)
    assert np.array_equal(dd, rd)
    assert np.array_equal(db, rb)
    assert np.array_equal(dbase, rbase)
    return L


def test_header_symbols_exported():
    hdr = open(os.path.join(ROOT, "include", "lbm_sparse.h")).read()
    declared = set(re.findall(r"^\s*(?:const char\*|int|void|int64_t)\s+(lbm_\w+)\s*\(", hdr, re.M))
    assert declared == set(_capi.EXPORTED)
    lib = ctypes.CDLL(_capi.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name


def test_header_is_c99_and_links(tmp_path):
    # the header is plain C: a C99 program that takes the address of every
    # declared entry point compiles with -pedantic and links against the
    # library (no device is touched: nothing is called)
    import shutil
    import subprocess
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "abi.c"
    body = "\n".join("    (void)&%s;" % name for name in sorted(_capi.EXPORTED))
    src.write_text('#include "lbm_sparse.h"\nint main(void) {\n%s\n    return 0;\n}\n' % body)
    lib_dir = os.path.dirname(_capi.LIB_PATH)
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I",
                        os.path.join(ROOT, "include"), str(src), "-L", lib_dir, "-llbm_sparse",
                        "-Wl,-rpath," + lib_dir, "-o", str(tmp_path / "abi")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


@pytest.mark.parametrize("order,block", [("lex", 0), ("lex", 1), ("lex", 2), ("lex", 3), ("lex", 5), ("morton", 0),
                                         ("hilbert", 0), ("hilbert_ls", 1), ("hilbert_ls", 3)])
def test_tiny_masks_all_periodicities(order, block):
    rng = np.random.default_rng(3)
    for shape in [(1, 1, 1), (3, 3, 3), (4, 3, 5), (7, 5, 6), (2, 9, 3)]:
        for frac in (0.0, 0.35, 0.7, 1.0):
            mask = (rng.random(shape) < frac).astype(np.uint8)
            for periodic in product((False, True), repeat=3):
                compare(mask, periodic, order, block)


@pytest.mark.parametrize("order,block", [("lex", 0), ("lex", 8), ("lex", 7), ("morton", 0), ("hilbert", 0),
                                         ("hilbert_ls", 8)])
def test_sphere_masks(order, block):
    mask = rsa_spheres((32, 32, 32), 3.0, 0.2, (True, False, False), seed=0)
    compare(mask, (True, False, False), order, block)
    mask = rsa_spheres((20, 33, 17), 2.5, 0.3, (True, True, False), seed=1)
    compare(mask, (True, True, False), order, block)


def test_foam_crop():
    mask = foam((48, 40, 36), 3.0, 0.85, seed=2)
    for order, block in [("lex", 0), ("lex", 8), ("morton", 0), ("hilbert", 0), ("hilbert_ls", 5)]:
        compare(mask, (True, False, False), order, block)


def test_channel_counts():
    L = Lattice(channel_mask(500, 100, 100), (True, False, False), "lex", 1)
    assert L.n_fluid == 4_802_000 and L.n_runs == 147_000


def test_channel_small_bit_exact():
    compare(channel_mask(20, 100, 100), (True, False, False), "lex", 1)


def test_padding_columns():
    mask = rsa_spheres((10, 10, 10), 2.0, 0.2, (True, False, False), seed=4)
    L = Lattice(mask, (True, False, False))
    a = L.adjacency(L.n_fluid + 13)
    assert np.all(a[:, L.n_fluid:] == -1)
    d, _, _ = L.wave_tables(L.n_runs + 5)
    assert np.all(d[:, L.n_runs:] == np.iinfo(np.int32).min)


def test_empty_and_full():
    L = Lattice(np.ones((3, 4, 5), np.uint8))
    assert (L.n_fluid, L.n_runs, L.n_waves) == (0, 0, 0)
    L = Lattice(np.zeros((3, 4, 5), np.uint8), (True, True, True))
    assert L.n_fluid == 60


def test_from_mask_is_the_constructor():
    mask = rsa_spheres((20, 18, 16), 3.0, 0.3, (True, False, False), seed=5)
    a = Lattice.from_mask(mask, (True, False, False), "lex", 4)
    b = Lattice(mask, (True, False, False), "lex", 4)
    assert (a.n_fluid, a.n_runs, a.n_waves) == (b.n_fluid, b.n_runs, b.n_waves)
    assert np.array_equal(a.node_voxel(), b.node_voxel())
    assert np.array_equal(a.adjacency(), b.adjacency())


def test_errors():
    with pytest.raises(LbmError) as e:
        Lattice(np.zeros((2, 2, 2), np.uint8), order="lex", block=-1)
    assert e.value.code == _capi.LBM_EINVAL
    with pytest.raises(LbmError):
        Lattice(np.zeros((0, 2, 2), np.uint8))
    L = Lattice(np.zeros((2, 2, 2), np.uint8))
    with pytest.raises(LbmError):
        L.adjacency(3)
