"""Host logic of the benchmark: the algorithmic bytes the roofline divides by,
the digest that ties counter results to the kernel sources, and the scaling
and grouping of rocprofv3 counter rows."""
import csv
import json

import pytest

import bench
from lbm_inputs import rsa_spheres


def test_kernel_bytes_match_the_table_sizes():
    # one launch moves the 19 PDFs in and out (38 s B per node) plus the index
    # tables: 72 B per node (adjacency), 72 B per run + 12 B per tile (the
    # paper's runs), 4 B per direction run + 216 B per tile (per-direction)
    from paper_1410_0412_amd import Lattice
    mask = rsa_spheres((20, 18, 22), 2.5, 0.2, (True, False, False), seed=5)
    lat = Lattice(mask, (True, False, False), "lex", 0)
    N, R, W, RD = lat.n_fluid, lat.n_runs, lat.n_waves, lat.n_direction_runs
    ib = lat.index_bytes()
    assert W == (N + 63) // 64
    want = {"adjacency": 72 * N, "runs": 72 * R + 12 * W, "direction": 4 * RD + 216 * W}
    for index, extra in want.items():
        for s in (8, 4, 2):
            assert bench.kernel_bytes("even", N, ib[index], s) == 38 * s * N
            for kind in ("odd", "osnt"):
                assert bench.kernel_bytes(kind, N, ib[index], s) == pytest.approx(38 * s * N + extra, rel=1e-12)
    with pytest.raises(KeyError):
        bench.kernel_bytes("copy", N, 0.0)


def test_source_digest_ignores_comments_and_layout():
    base = {"solver.hip": 'int f(int x) {\n  return x + 1;  // one\n}\nconst char* s = "// not a comment";\n'}
    digest = lambda files: bench.source_digest(read=lambda name: files.get(name, ""))
    d0 = digest(base)
    same = {"solver.hip": '/* header */\nint  f(int x)   {\n\n    return x + 1;\n}\nconst char* s = "// not a comment";'}
    assert digest(same) == d0
    assert digest({"solver.hip": base["solver.hip"].replace("x + 1", "x + 2")}) != d0
    assert digest({"solver.hip": base["solver.hip"].replace('"// not a comment"', '"//"')}) != d0


def test_source_digest_covers_the_device_sources():
    from paper_1410_0412_amd.build import DEVICE_SOURCES, HEADERS
    seen = []
    bench.source_digest(read=lambda name: seen.append(name) or "")
    assert sorted(seen) == sorted(DEVICE_SOURCES)
    assert "solver.hip" in seen and set(HEADERS) <= set(seen) and "lattice.cpp" not in seen


def test_kernel_key():
    assert bench.kernel_key("void lbm::aa_odd<double, lbm::IndexRIADir, false>(double*, int, lbm::IndexRIADir, "
                            "lbm::Collision, int)") == "aa_odd<double, IndexRIADir, false>"
    # the slot-type argument of the time-step kernels is left out
    for slot in ("int", "long"):
        assert bench.kernel_key("void lbm::aa_odd<double, lbm::IndexRIADir, false, %s>(double*, int, "
                                "lbm::IndexRIADir, lbm::Collision, int)" % slot) == "aa_odd<double, IndexRIADir, false>"
        assert bench.kernel_key("void lbm::aa_even<float, true, %s>(float*, int, lbm::Collision, int)"
                                % slot) == "aa_even<float, true>"
    assert bench.kernel_key("(anonymous namespace)::bench_copy(double const*, double*, long)") == "bench_copy"


def _write_csv(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for d, k, v in rows:
            w.writerow({"Dispatch_Id": d, "Kernel_Name": k, "Counter_Name": counter, "Counter_Value": v})


def test_traffic_from_scales_by_the_copy_kernel_and_splits_clusters(tmp_path):
    # spheres-32 has 26,185 fluid nodes: ld = 26,240, and the copy kernel
    # moves 19 * 8 * ld bytes in and as many out
    n = 26185
    ld = (n + 63) // 64 * 64
    copy_bytes = 19 * 8 * ld
    odd = "void lbm::aa_odd<double, lbm::IndexRIA, false>(double*, int, lbm::IndexRIA, lbm::Collision, int)"
    copy = "(anonymous namespace)::bench_copy(double const*, double*, long)"
    fetch = [(1, odd, 100.0), (2, odd, 110.0), (3, odd, 120.0), (40, odd, 300.0), (41, odd, 310.0),
             (60, copy, copy_bytes / 2 / 1024)]  # the counter reads half the copy's reads
    write = [(1, odd, 50.0), (2, odd, 50.0), (3, odd, 50.0), (40, odd, 70.0), (41, odd, 70.0),
             (60, copy, copy_bytes / 1024)]
    fc, wc, out = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "traffic.json"
    _write_csv(fc, "FETCH_SIZE", fetch)
    _write_csv(wc, "WRITE_SIZE", write)
    doc = bench.traffic_from(str(fc), str(wc), "spheres-32", "test", out_path=str(out))
    assert json.load(open(out)) == doc
    assert doc["scale"]["fetch"] == pytest.approx(2.0) and doc["scale"]["write"] == pytest.approx(1.0)
    k = doc["kernels"]["aa_odd<double, IndexRIA, false>"]
    assert k["dispatches"] == 3
    assert k["fetch_bytes"] == int(110.0 * 1024 * 2) and k["write_bytes"] == int(50.0 * 1024)
    assert k["hbm_bytes_per_launch"] == int(110.0 * 1024 * 2 + 50.0 * 1024)
    (later,) = k["later_clusters"]
    assert later["dispatches"] == 2 and later["fetch_bytes"] == int(305.0 * 1024 * 2)
    assert "bench_copy" not in doc["kernels"]
    assert doc["source_digest"] == bench.source_digest()


def test_traffic_request_check(tmp_path):
    # read requests of 128 B (the copy's bytes over its request count),
    # writes of 64 B and 32 B
    n = 26185
    ld = (n + 63) // 64 * 64
    copy_bytes = 19 * 8 * ld
    odd = "void lbm::aa_odd<double, lbm::IndexRIADir, false>(double*, int, lbm::IndexRIADir, lbm::Collision, int)"
    copy = "(anonymous namespace)::bench_copy(double const*, double*, long)"
    fc, wc = tmp_path / "f.csv", tmp_path / "w.csv"
    _write_csv(fc, "FETCH_SIZE", [(1, odd, 100.0), (60, copy, copy_bytes / 2 / 1024)])
    _write_csv(wc, "WRITE_SIZE", [(1, odd, 50.0), (60, copy, copy_bytes / 1024)])
    rc, wq = tmp_path / "r.csv", tmp_path / "q.csv"
    with open(rc, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for d, k, req, r32 in ((1, odd, 1000, 10), (60, copy, copy_bytes // 128, 0)):
            for c, v in (("TCC_EA0_RDREQ_sum", req), ("TCC_EA0_RDREQ_32B_sum", r32), ("TCC_BUBBLE_sum", 0)):
                w.writerow({"Dispatch_Id": d, "Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})
    with open(wq, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for d, k, req, r64 in ((1, odd, 800, 700), (60, copy, copy_bytes // 64, copy_bytes // 64)):
            for c, v in (("TCC_EA0_WRREQ_sum", req), ("TCC_EA0_WRREQ_64B_sum", r64)):
                w.writerow({"Dispatch_Id": d, "Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})
    doc = bench.traffic_from(str(fc), str(wc), "spheres-32", "test", out_path=str(tmp_path / "t.json"),
                             rdreq_csv=str(rc), wrreq_csv=str(wq))
    assert doc["request_check"]["read_request_bytes"] == pytest.approx(128.0)
    r = doc["kernels"]["aa_odd<double, IndexRIADir, false>"]["requests"]
    assert r["read_bytes"] == 990 * 128 + 10 * 32
    assert r["write_bytes"] == 700 * 64 + 100 * 32


def test_order_traffic_maps_clusters_to_orders(tmp_path):
    # two orders; per order the sweep runs the paper's runs in FP64 and FP32,
    # then per-direction runs in FP64 and FP32; each variant's launches form
    # one cluster of dispatch ids
    N = 1000
    sweep = {"config": {"workload": "test"}, "orders": {}}
    for o, ib in (("lex:0", {"runs": 10.0, "direction": 6.0}), ("morton", {"runs": 72.0, "direction": 60.0})):
        sweep["orders"][o] = {"fluid_nodes": N, "runs_per_node": 0.1, "index_bytes_per_node": ib}
        for k in ("f64", "f32", "f64_direction", "f32_direction"):
            sweep["orders"][o][k] = {"mflups": 1.0, "odd_us": 2.0, "even_us": 1.0}
    sj = tmp_path / "sweep.json"
    sj.write_text(json.dumps(sweep))
    ev = {8: "void lbm::aa_even<double, false>(double*, int, lbm::Collision, int)",
          4: "void lbm::aa_even<float, false>(float*, int, lbm::Collision, int)"}
    od = {(8, "runs"): "void lbm::aa_odd<double, lbm::IndexRIA, false>(double*)",
          (8, "direction"): "void lbm::aa_odd<double, lbm::IndexRIADir, false>(double*)",
          (4, "runs"): "void lbm::aa_odd<float, lbm::IndexRIA, false>(float*)",
          (4, "direction"): "void lbm::aa_odd<float, lbm::IndexRIADir, false>(float*)"}
    rows = {"FETCH_SIZE": [], "WRITE_SIZE": [], "TCP_TCC_READ_REQ_sum": [], "TCP_TCC_WRITE_REQ_sum": []}
    d = 1
    for i, o in enumerate(sweep["orders"]):
        for ria in ("runs", "direction"):
            for s in (8, 4):
                alg_e = 38 * s * N
                alg_o = alg_e + sweep["orders"][o]["index_bytes_per_node"][ria] * N
                f = 1.0 + 0.1 * (i + 1)  # the odd step's excess grows with the order index
                for k in range(3):
                    for name, ab, x in ((ev[s], alg_e, 1.0), (od[(s, ria)], alg_o, f)):
                        rows["FETCH_SIZE"].append((d, name, ab / 2 * x / 2 / 1024))
                        rows["WRITE_SIZE"].append((d, name, ab / 2 * x / 1024))
                        rows["TCP_TCC_READ_REQ_sum"].append((d, name, ab / 2 * x * 1.5 / 128))
                        rows["TCP_TCC_WRITE_REQ_sum"].append((d, name, ab / 2 * x * 1.5 / 64))
                        d += 1
                d += 10
    paths = {}
    for c, r in rows.items():
        paths[c] = tmp_path / (c + ".csv")
        _write_csv(paths[c], c, r)
    tcp = tmp_path / "tcp.csv"
    with open(tcp, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for c in ("TCP_TCC_READ_REQ_sum", "TCP_TCC_WRITE_REQ_sum"):
            for dd, k, v in rows[c]:
                w.writerow({"Dispatch_Id": dd, "Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})
    out = bench.order_traffic(str(sj), str(paths["FETCH_SIZE"]), str(paths["WRITE_SIZE"]), str(tcp))
    assert out["l1_to_l2_request_bytes"]["read"] == pytest.approx(128 / 1.5, abs=0.01)
    for i, o in enumerate(("lex:0", "morton")):
        for key in ("f64_runs", "f64_direction", "f32_runs", "f32_direction"):
            r = out["orders"][o][key]
            assert r["odd_memory_over_algorithmic"] == pytest.approx(1.0 + 0.1 * (i + 1), rel=1e-4)
            assert r["even_memory_over_algorithmic"] == pytest.approx(1.0, rel=1e-4)
            assert r["odd_l1_l2_over_algorithmic"] == pytest.approx(1.0 + 0.1 * (i + 1), rel=1e-4)


def test_bench_refuses_more_than_one_gpu():
    # one GPU only: the solver has no multi-GPU path, and the bench says so
    import subprocess
    import sys
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr


def test_slot_bits_threshold():
    # 32-bit slot offsets while 19 * ldf <= 2^31 - 1 (ldf = N rounded up to 64)
    top = (2 ** 31 - 1) // 19 // 64 * 64
    assert bench.slot_bits(top) == 32 and bench.slot_bits(top + 1) == 64
    assert bench.slot_bits(48_129_638) == 32 and bench.slot_bits(114_085_068) == 64
