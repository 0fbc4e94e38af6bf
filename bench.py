"""Throughput of the sparse-lattice D3Q19 propagation steps on one MI355X.

One benchmark step is one full AA cycle of AA-RIA in FP64: the direct even
time step followed by the indirect odd time step (two lattice updates of every
fluid node), on the 512x128x128 sphere pack at porosity 0.40 (radius-8
spheres, LS enumeration with blocking factor 64, tau = 0.6). Lattice tables
and PDFs are resident in HBM before timing starts.

Also reported: the other propagation variants (AA-IA, OS-NT-IA, OS-NT-RIA),
GPU analogues of the paper's bandwidth micro-benchmarks (Sect. 5.2, Table 3),
per-kernel durations from HIP events, the loop-balance Roofline (Sect. 4,
Sect. 5.2) and the oracle timed on the host CPU.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MFLUP/s and % of HBM roofline (GB/s ÷ B/FLUP), FP64 vs FP32 AA-RIA, 1 GPU"
HBM_PEAK_GBS = 8000.0
WORKLOAD = "spherepack-512x128x128"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_bytes(kind, n, r, w, s=8):
    """Algorithmic HBM bytes of one launch (PDFs read + written once, plus indices)."""
    pdf = 38 * s * n
    if kind == "even":
        return pdf
    if kind in ("odd_ia", "osnt_ia"):
        return pdf + 72 * n
    if kind in ("odd_ria", "osnt_ria"):
        return pdf + 72 * r + 12 * w
    raise KeyError(kind)


def source_digest():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1410_0412_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode() + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from committed rocprofv3 counter runs, if the
    kernel sources have not changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            doc = json.load(fh)
    except (OSError, ValueError):
        return None
    e = doc.get("kernels", {}).get(kernel)
    if not e or e.get("workload") != workload or doc.get("source_digest") != source_digest():
        return None
    return e.get("hbm_bytes_per_launch")


def time_variant(torch, lat, p, pattern, ria, precision, steps, warmup):
    from paper_1410_0412_amd import Solver

    s = Solver(lat, p["tau"], p["force"], pattern=pattern, ria=ria, precision=precision)
    s.init()
    s.step(2 * warmup)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for i in range(steps):
        s.step(1)
        ev[2 * i + 1].record()
        s.step(1)
        ev[2 * i + 2].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    d = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(2 * steps)]) * 1e-3
    _, _, tot = s.moments()
    if not np.isfinite(tot.cpu().numpy()).all():
        raise RuntimeError("non-finite totals after the timed run")
    del s
    return wall, d[0::2], d[1::2]


def microbench(torch, n_nodes):
    from paper_1410_0412_amd import bench_stream

    out = {}
    ld = (n_nodes + 63) // 64 * 64
    a = torch.ones(19 * ld, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    cases = {"copy": (0, 19 * ld, 2 * 8 * 19 * ld), "CNT-19A": (1, n_nodes, 2 * 8 * 19 * n_nodes),
             "U-19A": (2, n_nodes, 2 * 8 * 19 * n_nodes), "U-1A": (3, 19 * ld, 2 * 8 * 19 * ld)}
    for name, (kind, n, nbytes) in cases.items():
        for _ in range(3):
            bench_stream(kind, a, b, n, ld)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        e0.record()
        for _ in range(reps):
            bench_stream(kind, a, b, n, ld)
        e1.record()
        torch.cuda.synchronize()
        out[name] = round(nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    del a, b
    return out


def cpu_baseline(mask, p, steps=2):
    from oracle import dense

    solid = mask.astype(bool)
    f = dense.initial_state(solid)
    t0 = time.perf_counter()
    for _ in range(steps):
        f = dense.step(f, solid, p["periodic"], p["tau"], p["force"])
    dt = time.perf_counter() - t0
    n = int((~solid).sum())
    return {"value": round(n * steps / dt / 1e6, 4), "unit": "MFLUP/s", "cores": 1, "kind": "oracle",
            "sample": "%d time steps of the full-array FP64 numpy oracle on the same %s lattice "
                      "(single process, one thread; it updates all %d cells, MFLUP/s counts the %d fluid nodes)"
                      % (steps, WORKLOAD, solid.size, n)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500, help="timed AA cycles (2 time steps each)")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    from lbm_inputs import workload
    from paper_1410_0412_amd import Lattice

    log("generating", WORKLOAD)
    mask, p = workload(WORKLOAD, seed=args.seed)
    t0 = time.perf_counter()
    lat = Lattice(mask, p["periodic"], p["order"], p["block"])
    t_build = time.perf_counter() - t0
    N, R, W = lat.n_fluid, lat.n_runs, lat.n_waves
    r = R / N
    log("lattice N=%d R=%d r=%.4f built in %.2fs" % (N, R, r, t_build))

    variants = [("aa", True, "f64"), ("aa", True, "f32")]
    if not args.no_variants:
        variants += [("aa", False, "f64"), ("osnt", False, "f64"), ("osnt", True, "f64"),
                     ("aa", True, "f16")]
    res = {}
    for pattern, ria, prec in variants:
        key = "%s_%s_%s" % (pattern, "ria" if ria else "ia", prec)
        log("timing", key)
        wall, d_a, d_b = time_variant(torch, lat, p, pattern, ria, prec, args.steps, args.warmup)
        mflups = 2 * N * args.steps / wall / 1e6
        sb = {"f64": 8, "f32": 4, "f16": 2}[prec]
        if pattern == "aa":
            kinds = ("even", "odd_ria" if ria else "odd_ia")
            avg = (kernel_bytes(kinds[0], N, R, W, sb) + kernel_bytes(kinds[1], N, R, W, sb)) / 2
        else:
            kinds = ("osnt_ria" if ria else "osnt_ia",) * 2
            avg = kernel_bytes(kinds[0], N, R, W, sb)
        bl = avg / N
        res[key] = {
            "mflups": round(mflups, 1),
            "ms_per_time_step": round(wall / (2 * args.steps) * 1e3, 4),
            "kernel_us": {kinds[0]: round(float(np.mean(d_a)) * 1e6, 2),
                          kinds[1] + ("" if kinds[0] != kinds[1] else "_b"): round(float(np.mean(d_b)) * 1e6, 2)},
            "loop_balance_B_per_FLUP": round(bl, 3),
            "hbm_gbs_model": round(mflups * bl / 1e3, 1),
            "frac_of_hbm_roofline": round(mflups / (HBM_PEAK_GBS * 1e3 / bl), 4),
        }
        if key == "aa_ria_f64":
            main_wall, main_odd = wall, d_b
        log(key, res[key])

    micro = microbench(torch, N)
    log("micro-benchmarks GB/s", micro)

    aa = res["aa_ria_f64"]
    odd_bytes = kernel_bytes("odd_ria", N, R, W)
    odd_s = float(np.mean(main_odd))
    achieved = odd_bytes / odd_s / 1e9
    traffic = measured_traffic("aa_odd_f64<IndexRIA>", WORKLOAD)
    out = {
        "metric": METRIC,
        "value": aa["mflups"],
        "unit": "MFLUP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": WORKLOAD,
            "variant": "AA-RIA",
            "step": "one AA cycle: direct even step + indirect odd step (2 time steps)",
            "fluid_nodes": N, "runs": R, "runs_per_node": round(r, 5),
            "porosity": round(float(1.0 - mask.mean()), 5),
            "tau": p["tau"], "force": list(p["force"]),
            "enumeration": "lex B=%d" % p["block"],
            "lattice_build_s": round(t_build, 3),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "aa_odd_f64<IndexRIA>",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": int(odd_bytes),
            "avg_launch_us": round(odd_s * 1e6, 2),
        },
        "hbm_roofline_mflups": {
            "loop_balance_B_per_FLUP": aa["loop_balance_B_per_FLUP"],
            "roofline_mflups_at_8TBs": round(HBM_PEAK_GBS * 1e3 / aa["loop_balance_B_per_FLUP"], 1),
            "frac": aa["frac_of_hbm_roofline"],
            "paper_model_B_l_aa_r": round(304 + 38 * r, 3),
        },
        "variants": res,
        "microbench_GBs": micro,
    }
    if not args.no_cpu_baseline:
        log("timing the oracle on the host")
        out["cpu_baseline"] = cpu_baseline(mask, p)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
