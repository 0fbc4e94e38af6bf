"""Throughput of the sparse-lattice D3Q19 propagation steps on one MI355X.

One benchmark step is one full AA cycle of AA-RIA in FP64: the direct even
time step followed by the indirect odd time step (two lattice updates of every
fluid node), on the 384^3 foam (smoothed Gaussian noise thresholded to
porosity 0.85, 48.1M fluid nodes, lexicographic order without blocking,
tau = 0.7). Lattice tables and PDFs are resident in HBM before timing starts.
Each variant is timed as the median of 5 runs of ``--steps`` cycles.

Also reported: FP32 AA-RIA on the same lattice, the other propagation
variants (AA-IA, OS-NT-IA, OS-NT-RIA, FP16), AA-RIA on the 512x128x128
sphere pack, GPU analogues of the paper's bandwidth micro-benchmarks
(Sect. 5.2, Table 3), per-kernel durations from HIP events, the loop-balance
Roofline (Sect. 4, Sect. 5.2) and the oracle timed on the host CPU.

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
WORKLOAD = "foam-384"
SIDE_WORKLOAD = "spherepack-512x128x128"
REPEATS = 5  # timed runs per variant of the default line; the median counts


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_bytes(kind, n, idx, s=8):
    """Algorithmic HBM bytes of one launch: the PDFs read and written once,
    plus, for an indirect step, ``idx`` index bytes per node (72 for the
    adjacency list; the run tables' bytes per node for RIA)."""
    pdf = 38 * s * n
    if kind == "even":
        return pdf
    if kind in ("odd", "osnt"):
        return pdf + idx * n
    raise KeyError(kind)


# kernel names of the odd step per index source (as rocprofv3 prints them)
ODD_KERNEL = {"adjacency": "aa_odd<double, IndexIA, false>", "runs": "aa_odd<double, IndexRIA, false>",
              "direction": "aa_odd<double, IndexRIADir, false>"}


def _strip_comments(text):
    """C/C++ source without comments and blank-line or indentation changes."""
    out, i, n = [], 0, len(text)
    while i < n:
        if text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        elif text[i] == '"':
            j = i + 1
            while j < n and text[j] != '"':
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        else:
            out.append(text[i])
            i += 1
    lines = (" ".join(l.split()) for l in "".join(out).splitlines())
    return "\n".join(l for l in lines if l)


def source_digest(read=None):
    """Digest of the kernel sources (comments and layout ignored), so that
    counter results are only reused for the code they were taken on."""
    from paper_1410_0412_amd.build import DEVICE_SOURCES

    csrc = os.path.join(ROOT, "paper_1410_0412_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(DEVICE_SOURCES):
        if read is None:
            with open(os.path.join(csrc, name), encoding="utf-8") as fh:
                text = fh.read()
        else:
            text = read(name)
        h.update(name.encode() + _strip_comments(text).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from committed rocprofv3 counter runs
    (profiles/traffic_<workload>.json), if the kernel sources have not
    changed since the counters were taken."""
    for name in ("traffic_%s.json" % workload,):
        try:
            with open(os.path.join(ROOT, "profiles", name)) as fh:
                doc = json.load(fh)
        except (OSError, ValueError):
            continue
        if doc.get("workload") != workload:
            continue
        e = doc.get("kernels", {}).get(kernel)
        if not e or doc.get("source_digest") != source_digest():
            return None
        return e.get("hbm_bytes_per_launch")
    return None


def kernel_key(name):
    """Short kernel name of a demangled rocprofv3 kernel name. The time-step
    kernels take the slot type (int: 32-bit element offsets, long: 64-bit)
    as their last template argument; the short name leaves it out, since the
    lattice size fixes it (``slot_bits``)."""
    name = name.replace("(anonymous namespace)::", "").replace("lbm::", "").replace("void ", "")
    depth, out = 0, []
    for ch in name:
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    key = "".join(out).strip()
    for slot in (", int>", ", long>"):
        if key.endswith(slot):
            return key[: -len(slot)] + ">"
    return key


#: --odd-schedule choices as the solver's odd_schedule argument
SCHEDULES = {"auto": "auto", "band": "band", "chunked": None}
#: the --odd-schedule choice of this run (set by main)
ODD_SCHEDULE = ["auto"]


def odd_schedule_name(lat, precision, index_bytes):
    """The AA odd step's workgroup order of the default line's solver."""
    from paper_1410_0412_amd import choose_odd_schedule
    from paper_1410_0412_amd.solver import BAND_ROWS

    if ODD_SCHEDULE[0] == "chunked":
        return "chunked"
    if ODD_SCHEDULE[0] == "band":
        return "band/%d" % BAND_ROWS
    rows = choose_odd_schedule(lat, "aa", precision, index_bytes)
    return "band/%d" % rows if rows else "chunked"


def slot_bits(n_fluid):
    """Width of the time-step kernels' slot offsets for a lattice of n_fluid
    nodes: 32 while a grid (19 * ldf elements) fits in 2^31 - 1, else 64."""
    ldf = (max(int(n_fluid), 1) + 63) // 64 * 64
    return 32 if 19 * ldf <= 2 ** 31 - 1 else 64


def _counter_clusters(path, counters):
    """Per kernel: the averages of ``counters`` over each cluster of
    consecutive dispatch ids of one rocprofv3 --pmc csv file. The variants
    run one after the other, so a kernel shared by two variants (the odd
    step with and without the XCD remap) shows up as separate clusters; each
    cluster is averaged on its own."""
    import csv

    acc = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] not in counters:
            continue
        k = kernel_key(r["Kernel_Name"])
        acc.setdefault(k, {}).setdefault(int(r["Dispatch_Id"]), {})[r["Counter_Name"]] = float(r["Counter_Value"])
    out = {}
    for k, per in acc.items():
        ids = sorted(per)
        clusters = [[ids[0]]]
        for d0, d1 in zip(ids, ids[1:]):
            if d1 - d0 > 4:
                clusters.append([])
            clusters[-1].append(d1)
        out[k] = [({c: sum(per[i].get(c, 0.0) for i in cl) / len(cl) for c in counters}, len(cl))
                  for cl in clusters]
    return out


def traffic_from(fetch_csv, write_csv, workload_name, command, out_path=None, rdreq_csv=None, wrreq_csv=None):
    """Write profiles/traffic_<workload>.json (or out_path) from two rocprofv3 --pmc runs
    (FETCH_SIZE, WRITE_SIZE; KiB per dispatch). Both counters are scaled by
    what they read for the copy micro-benchmark, whose bytes are known.

    With request counts (``rdreq_csv``: TCC_EA0_RDREQ_sum, TCC_EA0_RDREQ_32B_sum,
    TCC_BUBBLE_sum; ``wrreq_csv``: TCC_EA0_WRREQ_sum, TCC_EA0_WRREQ_64B_sum)
    the same bytes are also formed from the number and size of the requests
    the L2 sends to memory, as a check of the scale factors: read requests
    of 128 B (the copy's bytes over its request count), writes of 64 B or
    32 B."""
    fetch = {k: [(v["FETCH_SIZE"] * 1024.0, n) for v, n in cl]
             for k, cl in _counter_clusters(fetch_csv, ("FETCH_SIZE",)).items()}
    write = {k: [(v["WRITE_SIZE"] * 1024.0, n) for v, n in cl]
             for k, cl in _counter_clusters(write_csv, ("WRITE_SIZE",)).items()}
    mask, p = __import__("lbm_inputs").workload(workload_name)
    n = int((mask == 0).sum())
    ld = (n + 63) // 64 * 64
    copy_bytes = 8 * 19 * ld  # read once and written once by the copy kernel
    sf = copy_bytes / fetch["bench_copy"][0][0]
    sw = copy_bytes / write["bench_copy"][0][0]
    rd = wr = None
    if rdreq_csv and wrreq_csv:
        rd = _counter_clusters(rdreq_csv, ("TCC_EA0_RDREQ_sum", "TCC_EA0_RDREQ_32B_sum", "TCC_BUBBLE_sum"))
        wr = _counter_clusters(wrreq_csv, ("TCC_EA0_WRREQ_sum", "TCC_EA0_WRREQ_64B_sum"))
        c = rd["bench_copy"][0][0]
        read_req_bytes = copy_bytes / c["TCC_EA0_RDREQ_sum"]
    kernels = {}
    for k in sorted(set(fetch) & set(write)):
        if k.startswith("bench_") or k.startswith("at::"):
            continue
        # the first cluster belongs to the first variant that runs the kernel
        fb, wb = fetch[k][0][0] * sf, write[k][0][0] * sw
        kernels[k] = {"fetch_bytes": int(fb), "write_bytes": int(wb), "hbm_bytes_per_launch": int(fb + wb),
                      "dispatches": fetch[k][0][1]}
        if len(fetch[k]) > 1 and len(fetch[k]) == len(write[k]):
            kernels[k]["later_clusters"] = [
                {"fetch_bytes": int(f * sf), "write_bytes": int(w * sw), "dispatches": n}
                for (f, n), (w, _) in zip(fetch[k][1:], write[k][1:])]
        if rd is not None and k in rd and k in wr:
            r, w = rd[k][0][0], wr[k][0][0]
            kernels[k]["requests"] = {
                "read": int(r["TCC_EA0_RDREQ_sum"]), "read_32B": int(r["TCC_EA0_RDREQ_32B_sum"]),
                "read_128B_bubble": int(r["TCC_BUBBLE_sum"]),
                "write": int(w["TCC_EA0_WRREQ_sum"]), "write_64B": int(w["TCC_EA0_WRREQ_64B_sum"]),
                "read_bytes": int(r["TCC_EA0_RDREQ_32B_sum"] * 32
                                  + (r["TCC_EA0_RDREQ_sum"] - r["TCC_EA0_RDREQ_32B_sum"]) * read_req_bytes),
                "write_bytes": int(w["TCC_EA0_WRREQ_64B_sum"] * 64
                                   + (w["TCC_EA0_WRREQ_sum"] - w["TCC_EA0_WRREQ_64B_sum"]) * 32)}
    doc = {"workload": workload_name, "source_digest": source_digest(),
           "scale": {"fetch": round(sf, 4), "write": round(sw, 4),
                     "reference": "copy micro-benchmark of %d bytes" % copy_bytes},
           "command": command, "kernels": kernels}
    if rd is not None:
        doc["request_check"] = {
            "read_request_bytes": round(read_req_bytes, 3),
            "note": "bytes per L2-to-memory read request of the copy kernel (its bytes over TCC_EA0_RDREQ_sum); "
                    "FETCH_SIZE counts a request as 64 B unless TCC_BUBBLE marks it as 128 B, and TCC_BUBBLE "
                    "reads 0 here, hence the fetch scale of 2"}
    with open(out_path or os.path.join(ROOT, "profiles", "traffic_%s.json" % workload_name), "w") as fh:
        json.dump(doc, fh, indent=1)
    return doc


def trace_summary(trace_csv):
    """Per-launch statistics of a rocprofv3 kernel trace (k_kernel_trace.csv),
    one row per run of consecutive dispatches of one kernel at one grid size
    (a bench variant on one lattice): calls, mean and minimum duration."""
    import csv

    rows = sorted(csv.DictReader(open(trace_csv)), key=lambda r: int(r["Dispatch_Id"]))
    groups = []
    last = {}
    for r in rows:
        key = (kernel_key(r["Kernel_Name"]), int(r["Grid_Size_X"]))
        d = int(r["Dispatch_Id"])
        us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3
        g = last.get(key)
        if g is None or d - g["last"] > 6:
            g = {"kernel": key[0], "grid": key[1], "first": d, "last": d, "us": []}
            groups.append(g)
            last[key] = g
        g["last"] = d
        g["us"].append(us)
    return [{"kernel": g["kernel"], "grid": g["grid"], "first_dispatch": g["first"], "calls": len(g["us"]),
             "avg_us": round(float(np.mean(g["us"])), 2), "min_us": round(float(np.min(g["us"])), 2)}
            for g in groups]


def order_traffic(sweep_json, fetch_csv, write_csv, tcp_csv, scale_fetch=2.0, scale_write=1.0):
    """Counter traffic of the AA step kernels per enumeration: the GPU form of
    the in-cache loop balance of Sect. 5.6. The counter files come from
    rocprofv3 --pmc runs of the same --orders sweep that wrote ``sweep_json``
    (FETCH_SIZE; WRITE_SIZE; TCP_TCC_READ_REQ_sum and TCP_TCC_WRITE_REQ_sum).
    The sweep runs, per order, the paper's runs in FP64 and FP32, then
    per-direction runs in FP64 and FP32, so the k-th cluster of a kernel's
    dispatches belongs to the k-th variant that runs it. Memory bytes use the
    FETCH_SIZE and WRITE_SIZE scales of the copy kernel (from
    profiles/traffic_foam-384.json); L1-to-L2 request sizes are those that put the
    FP64 even step of the first order on its algorithmic bytes."""
    sweep = json.load(open(sweep_json))
    orders = list(sweep["orders"])
    N = sweep["orders"][orders[0]]["fluid_nodes"]
    fetch = _counter_clusters(fetch_csv, ("FETCH_SIZE",))
    write = _counter_clusters(write_csv, ("WRITE_SIZE",))
    tcp = _counter_clusters(tcp_csv, ("TCP_TCC_READ_REQ_sum", "TCP_TCC_WRITE_REQ_sum"))
    ev64 = tcp["aa_even<double, false>"][0][0]
    rd_req = 38 * 8 * N / 2 / ev64["TCP_TCC_READ_REQ_sum"]
    wr_req = 38 * 8 * N / 2 / ev64["TCP_TCC_WRITE_REQ_sum"]
    out = {"workload": sweep["config"]["workload"], "fluid_nodes": N,
           "l1_to_l2_request_bytes": {"read": round(rd_req, 2), "write": round(wr_req, 2)},
           "memory_scale": {"fetch": scale_fetch, "write": scale_write}, "orders": {}}
    for i, spec in enumerate(orders):
        row = sweep["orders"][spec]
        ib = row["index_bytes_per_node"]
        res = {"runs_per_node": row["runs_per_node"], "index_bytes_per_node": ib}
        for prec, S, s in (("f64", "double", 8), ("f32", "float", 4)):
            for ria, idx, cl_even in (("runs", "IndexRIA", 2 * i), ("direction", "IndexRIADir", 2 * i + 1)):
                odd_k = "aa_odd<%s, %s, false>" % (S, idx)
                even_k = "aa_even<%s, false>" % S
                alg_odd = 38 * s * N + ib[ria] * N
                alg_even = 38 * s * N
                o_mem = (fetch[odd_k][i][0]["FETCH_SIZE"] * scale_fetch
                         + write[odd_k][i][0]["WRITE_SIZE"] * scale_write) * 1024.0
                e_mem = (fetch[even_k][cl_even][0]["FETCH_SIZE"] * scale_fetch
                         + write[even_k][cl_even][0]["WRITE_SIZE"] * scale_write) * 1024.0
                t = tcp[odd_k][i][0]
                l1 = t["TCP_TCC_READ_REQ_sum"] * rd_req + t["TCP_TCC_WRITE_REQ_sum"] * wr_req
                v = row[prec if ria == "runs" else prec + "_direction"]
                res["%s_%s" % (prec, ria)] = {
                    "mflups": v["mflups"], "odd_us": v["odd_us"], "even_us": v["even_us"],
                    "odd_memory_B_per_node": round(o_mem / N, 2), "odd_algorithmic_B_per_node": round(alg_odd / N, 2),
                    "odd_memory_over_algorithmic": round(o_mem / alg_odd, 4),
                    "even_memory_over_algorithmic": round(e_mem / alg_even, 4),
                    "odd_l1_l2_B_per_node": round(l1 / N, 2),
                    "odd_l1_l2_over_algorithmic": round(l1 / alg_odd, 4)}
        out["orders"][spec] = res
    return out


class Timing:
    """Timed cycles of one variant: host-clock seconds of each repeat, and
    HIP-event durations of the first and second step of sampled cycles."""

    def __init__(self, walls, first, second, index):
        self.walls, self.first, self.second, self.index = walls, first, second, index

    @property
    def wall(self):
        """Seconds of all repeats together."""
        return float(sum(self.walls))

    def median_wall(self):
        return float(np.median(self.walls))

    # (wall, first, second, index), for callers that time one repeat
    def __iter__(self):
        return iter((self.wall, self.first, self.second, self.index))


def time_variant(torch, lat, p, pattern, ria, precision, steps, warmup, xcd_remap=True, sample_every=16,
                 repeats=1, trt_magic=None):
    """Time ``repeats`` runs of ``steps`` cycles of two time steps each, queued
    back to back, each run bracketed by synchronisations.

    Kernel durations come from HIP events on the solver's stream around
    single launches inside the timed runs: the first step of every
    `sample_every`-th cycle and the second step of the cycle half-way
    between (with ``sample_every=1``: both steps of every cycle). An event
    pair adds about 2 us to a run; around every launch that is 4 % of the
    run on the 3.3M-node sphere pack (steps of 0.2 ms) and under 0.1 % on
    the 48M-node foam (steps of 2.4-2.9 ms)."""
    from paper_1410_0412_amd import Solver

    s = Solver(lat, p["tau"], p["force"], pattern=pattern, ria=ria, precision=precision, xcd_remap=xcd_remap,
               trt_magic=trt_magic, odd_schedule=SCHEDULES[ODD_SCHEDULE[0]] if pattern == "aa" else None)
    index = s.index
    s.init()
    s.step(2 * warmup)
    torch.cuda.synchronize()
    every = max(1, int(sample_every))
    half = every // 2
    pairs = ([], [])  # (start, end) events around first / second steps
    walls = []
    for _ in range(max(1, int(repeats))):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            k = i % every
            sample = (k == 0, k == half if every > 1 else True)
            if not any(sample):
                s.step(2)
                continue
            for j in (0, 1):
                if not sample[j]:
                    s.step(1)
                    continue
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                s.step(1)
                b.record()
                pairs[j].append((a, b))
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
    d = [np.array([a.elapsed_time(b) for a, b in pr]) * 1e-3 for pr in pairs]
    _, _, tot = s.moments()
    if not np.isfinite(tot.cpu().numpy()).all():
        raise RuntimeError("non-finite totals after the timed run")
    del s
    return Timing(walls, d[0], d[1], index)


def microbench(torch, n_nodes):
    from paper_1410_0412_amd import bench_stream

    out = {}
    ld = (n_nodes + 63) // 64 * 64
    a = torch.ones(19 * ld, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    cases = {"copy": (0, 19 * ld, 2 * 8 * 19 * ld), "CNT-19A": (1, n_nodes, 2 * 8 * 19 * n_nodes),
             "U-19A": (2, n_nodes, 2 * 8 * 19 * n_nodes), "U-1A": (3, 19 * ld, 2 * 8 * 19 * ld),
             "U-19T": (5, n_nodes, 2 * 8 * 19 * n_nodes), "CNT-19T": (6, n_nodes, 2 * 8 * 19 * n_nodes),
             "U-19T-L": (7, n_nodes, 2 * 8 * 19 * n_nodes), "CNT-19T-L": (8, n_nodes, 2 * 8 * 19 * n_nodes)}
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


def host_cpu():
    """Model name and logical CPU counts of the host (as the OS reports them)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def host_mem_available():
    """Bytes of host memory the OS reports as available (None if unknown)."""
    try:
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemAvailable:"):
                    return int(line.split()[1]) * 1024
    except (OSError, ValueError, IndexError):
        pass
    return None


def cpu_baseline(mask, p, workload_name, cell_budget=5e7):
    """The full-array FP64 oracle on the host, on a bounded sample of the
    workload: about ``cell_budget`` cell updates (one time step of the 384^3
    foam, six of the 512x128x128 sphere pack), on an x-crop of the box if
    host memory cannot hold about five full PDF arrays."""
    from oracle import dense

    solid = mask.astype(bool)
    steps = max(1, int(round(cell_budget / solid.size)))
    crop = ""
    avail = host_mem_available()
    plane = 19 * 8 * solid.shape[1] * solid.shape[2]
    if avail is not None and 5 * plane * solid.shape[0] > avail:
        nx = max(1, int(avail // (5 * plane)))
        solid = np.ascontiguousarray(solid[:nx])
        crop = "; x-crop of %d of %d planes (host memory)" % (nx, mask.shape[0])
    f = dense.initial_state(solid)
    t0 = time.perf_counter()
    for _ in range(steps):
        f = dense.step(f, solid, p["periodic"], p["tau"], p["force"])
    dt = time.perf_counter() - t0
    del f
    n = int((~solid).sum())
    return {"value": round(n * steps / dt / 1e6, 4), "unit": "MFLUP/s", "cores": 1, "kind": "oracle",
            "sample": "%d time step(s) of the full-array FP64 numpy oracle on the %s lattice%s "
                      "(single process, one thread; it updates all %d cells, MFLUP/s counts the %d fluid nodes), "
                      "%.1f s" % (steps, workload_name, crop, solid.size, n, dt),
            "host": host_cpu()}


def order_sweep(torch, args):
    """Sect. 5.6 analogue: AA-RIA throughput and run density per enumeration."""
    from lbm_inputs import workload
    from paper_1410_0412_amd import Lattice, choose_index

    log("generating", args.workload)
    mask, p = workload(args.workload, seed=args.seed)
    out = {"metric": METRIC + " (enumeration sweep)", "unit": "MFLUP/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "data": "synthetic",
           "config": {"workload": args.workload, "porosity": round(float(1 - mask.mean()), 5), "tau": p["tau"]},
           "orders": {}}
    for spec in args.orders.split(","):
        order, _, blk = spec.partition(":")
        blk = int(blk or 0)
        t0 = time.perf_counter()
        lat = Lattice(mask, p["periodic"], order, blk)
        tb = time.perf_counter() - t0
        N, R = lat.n_fluid, lat.n_runs
        ib = lat.index_bytes()
        row = {"fluid_nodes": N, "runs_per_node": round(R / N, 5), "lattice_build_s": round(tb, 2),
               "index_bytes_per_node": {k: round(v, 3) for k, v in ib.items()}}
        # the paper's runs, then per-direction runs; "auto" names the choice
        # the library makes between the two
        row["auto"] = {prec: choose_index(lat, "aa", prec) for prec in ("f64", "f32")}
        for ria in ("runs", "direction"):
            for prec in ("f64", "f32"):
                wall, d_e, d_o, index = time_variant(torch, lat, p, "aa", ria, prec, args.steps, args.warmup)
                key = prec if ria == "runs" else prec + "_direction"
                sb = 8 if prec == "f64" else 4
                mflups = 2 * N * args.steps / wall / 1e6
                bl = (kernel_bytes("even", N, ib[index], sb) + kernel_bytes("odd", N, ib[index], sb)) / 2 / N
                row[key] = {"index": index, "mflups": round(mflups, 1),
                            "even_us": round(float(np.mean(d_e)) * 1e6, 1),
                            "odd_us": round(float(np.mean(d_o)) * 1e6, 1),
                            "loop_balance_B_per_FLUP": round(bl, 2),
                            "frac_of_hbm_roofline": round(mflups / (HBM_PEAK_GBS * 1e3 / bl), 4)}
        if args.with_ia_osnt:
            # FP64 AA-IA and OS-NT with each index source (the Sect. 5.1 RIA comparison)
            for pattern, ria in (("aa", False), ("osnt", False), ("osnt", "runs"), ("osnt", "direction")):
                wall, _, _, index = time_variant(torch, lat, p, pattern, ria, "f64", args.steps, args.warmup)
                mflups = 2 * N * args.steps / wall / 1e6
                if pattern == "aa":
                    bl = (kernel_bytes("even", N, ib[index]) + kernel_bytes("odd", N, ib[index])) / 2 / N
                else:
                    bl = kernel_bytes("osnt", N, ib[index]) / N
                row["%s_%s_f64" % (pattern, index)] = {
                    "mflups": round(mflups, 1), "loop_balance_B_per_FLUP": round(bl, 2),
                    "frac_of_hbm_roofline": round(mflups / (HBM_PEAK_GBS * 1e3 / bl), 4)}
        log(spec, row)
        out["orders"][spec] = row
        del lat
    print(json.dumps(out), flush=True)


def size_sweep(torch, args):
    """AA-RIA throughput against lattice size: steps queued back to back, as a
    caller runs them, timed with events around the whole run."""
    from lbm_inputs import workload
    from paper_1410_0412_amd import Lattice, Solver

    out = {"metric": "MFLUP/s against lattice size (AA-RIA, automatic index choice)", "unit": "MFLUP/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "data": "synthetic", "workloads": {}}
    for name in args.size_sweep.split(","):
        log("generating", name)
        mask, p = workload(name, seed=args.seed)
        lat = Lattice(mask, p["periodic"], p["order"], p["block"])
        N = lat.n_fluid
        row = {"fluid_nodes": N}
        for prec in ("f64", "f32"):
            s = Solver(lat, p["tau"], p["force"], pattern="aa", ria="auto", precision=prec,
                       odd_schedule=SCHEDULES[args.odd_schedule])
            s.init()
            s.step(2 * args.warmup)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            s.step(2 * args.steps)
            e1.record()
            torch.cuda.synchronize()
            sec = e0.elapsed_time(e1) * 1e-3
            row[prec] = {"index": s.index, "mflups": round(2 * args.steps * N / sec / 1e6, 1),
                         "us_per_time_step": round(sec / (2 * args.steps) * 1e6, 2),
                         "odd_schedule": "band/%d" % s.band_rows if s.band_rows else "chunked"}
            del s
        log(name, row)
        out["workloads"][name] = row
        del lat, mask
    print(json.dumps(out), flush=True)


def pattern_study(torch, args):
    """AA against OS-NT (RIA, automatic index choice) per storage precision
    on each workload of --pattern-study."""
    from lbm_inputs import workload
    from paper_1410_0412_amd import Lattice

    out = {"metric": "MFLUP/s of AA-RIA and OS-NT-RIA per storage precision", "unit": "MFLUP/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "data": "synthetic", "workloads": {}}
    for name in args.pattern_study.split(","):
        log("generating", name)
        mask, p = workload(name, seed=args.seed)
        lat = Lattice(mask, p["periodic"], p["order"], p["block"])
        N = lat.n_fluid
        row = {"fluid_nodes": N}
        for prec in ("f64", "f32", "f16"):
            for pattern in ("aa", "osnt"):
                wall, d_a, d_b, index = time_variant(torch, lat, p, pattern, "auto", prec, args.steps, args.warmup)
                row["%s_%s" % (pattern, prec)] = {
                    "index": index, "mflups": round(2 * N * args.steps / wall / 1e6, 1),
                    "kernel_us": [round(float(np.mean(d_a)) * 1e6, 2), round(float(np.mean(d_b)) * 1e6, 2)]}
        log(name, row)
        out["workloads"][name] = row
        del lat, mask
    print(json.dumps(out), flush=True)


def precision_study(torch, args):
    """FP32 / FP16 deviation storage against the FP64 path on one workload."""
    from lbm_inputs import workload
    from paper_1410_0412_amd import Lattice, Solver

    log("generating", args.workload)
    mask, p = workload(args.workload, seed=args.seed)
    lat = Lattice(mask, p["periodic"], p["order"], p["block"])
    steps = args.steps
    res, ref = {}, None
    for prec in ("f64", "f32", "f16"):
        s = Solver(lat, p["tau"], p["force"], pattern="aa", ria=True, precision=prec)
        s.init()
        _, _, t0 = s.moments()
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for k in range(0, steps, 1000):
            s.step(min(1000, steps - k))
            torch.cuda.synchronize()
            log(prec, "step", min(k + 1000, steps))
        wall = time.perf_counter() - w0
        rho, u, t1 = s.moments()
        row = {"mflups": round(lat.n_fluid * steps / wall / 1e6, 1),
               "mass_drift_rel": abs(t1[0].item() - t0[0].item()) / t0[0].item()}
        if ref is None:
            ref = (rho, u)
        else:
            scale = torch.sqrt((ref[1] ** 2).sum(0)).max()
            du = torch.sqrt(((u - ref[1]) ** 2).sum(0)).max() / scale
            row.update({"u_normwise_rel_err_vs_f64": du.item(),
                        "rho_max_abs_err_vs_f64": (rho - ref[0]).abs().max().item()})
            # per component: max |u_a - u_a,f64| over nodes, relative to max |u_f64|
            for a, name in enumerate(("ux", "uy", "uz")):
                row[name + "_max_err_rel_to_umax_vs_f64"] = ((u[a] - ref[1][a]).abs().max() / scale).item()
        row["u_max"] = u.abs().max().item()
        res[prec] = row
        log(prec, row)
        del s
    out = {"metric": "error of deviation storage vs the FP64 GPU path", "n_gpus": 1, "steps": steps,
           "data": "synthetic", "config": {"workload": args.workload, "fluid_nodes": lat.n_fluid,
                                           "variant": "AA-RIA (paper's runs)", "tau": p["tau"],
                                           "force": list(p["force"])},
           "precisions": res}
    print(json.dumps(out), flush=True)


def adjoint_bench(torch, args):
    """Differentiation extension on the 128^3 sphere pack: the forward PBB
    step, the adjoint step and one whole gradient of the outlet flux (T
    steps, checkpoints every 20), with their algorithmic bytes."""
    from lbm_inputs import workload, pbb_fraction
    from paper_1410_0412_amd import Lattice, Solver, outlet_flux

    name = "spherepack-128"
    mask, p = workload(name, seed=args.seed)
    lat = Lattice(mask, p["periodic"], p["order"], p["block"])
    N, T, every = lat.n_fluid, p["steps"], 20
    nv = lat.node_voxel().astype(np.int64)
    ns = torch.from_numpy(pbb_fraction(mask, seed=1).reshape(-1)[nv]).cuda()
    wv = np.zeros(mask.shape)
    wv[-1] = 1.0
    w = torch.from_numpy(wv.reshape(-1)[nv]).cuda()
    s = Solver(lat, p["tau"], p["force"], pattern="aa", ria="auto", pbb=True)
    ib = lat.index_bytes()[s.index]
    ev = lambda: torch.cuda.Event(enable_timing=True)
    # forward PBB steps
    s.set_solid_fraction(ns)
    s.init()
    s.step(2 * args.warmup)
    e0, e1 = ev(), ev()
    e0.record()
    s.step(T)
    e1.record()
    torch.cuda.synchronize()
    fwd_s = e0.elapsed_time(e1) * 1e-3 / T
    # adjoint steps over stored states of one checkpoint segment
    states = []
    s.init()
    for _ in range(every):
        states.append(s.pdf[0].clone())
        s.step(1)
    lam = torch.empty_like(s.pdf[0])
    grad = torch.zeros(N, dtype=torch.float64, device="cuda")
    s.adjoint_seed(w, 0, every, lam)
    for t in range(every - 1, -1, -1):  # warm-up pass
        s.adjoint_step(states[t], t, lam, grad)
    s.adjoint_seed(w, 0, every, lam)
    torch.cuda.synchronize()
    e0, e1 = ev(), ev()
    e0.record()
    for t in range(every - 1, -1, -1):
        s.adjoint_step(states[t], t, lam, grad)
    e1.record()
    torch.cuda.synchronize()
    adj_s = e0.elapsed_time(e1) * 1e-3 / every
    del states
    # one whole gradient: forward with checkpoints, recomputation, adjoint;
    # the first call also allocates its buffers, the second finds them in
    # torch's cache
    walls = []
    for _ in range(2):
        x = ns.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J = outlet_flux(x, s, T, every, w)
        J.backward()
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
    first_s, grad_s = walls
    # algorithmic bytes per node: PBB forward reads and writes 19 PDFs and
    # reads ns; the adjoint reads the forward state and lambda, writes lambda,
    # reads ns and updates the gradient; odd steps add the index bytes
    fwd_b = 38 * 8 + 8 + ib / 2
    adj_b = 57 * 8 + 8 + 16 + ib / 2
    out = {"metric": "adjoint AA step (PBB, FP64): MFLUP/s and % of HBM roofline", "n_gpus": 1,
           "data": "synthetic", "unit": "MFLUP/s",
           "config": {"workload": name, "fluid_nodes": N, "steps": T, "checkpoint_every": every, "index": s.index,
                      "tau": p["tau"], "force": list(p["force"])},
           "forward_pbb": {"mflups": round(N / fwd_s / 1e6, 1), "us_per_step": round(fwd_s * 1e6, 2),
                           "B_per_FLUP": round(fwd_b, 2),
                           "frac_of_hbm_roofline": round(N / fwd_s * fwd_b / (HBM_PEAK_GBS * 1e9), 4)},
           "adjoint": {"mflups": round(N / adj_s / 1e6, 1), "us_per_step": round(adj_s * 1e6, 2),
                       "B_per_FLUP": round(adj_b, 2),
                       "frac_of_hbm_roofline": round(N / adj_s * adj_b / (HBM_PEAK_GBS * 1e9), 4)},
           "gradient": {"seconds": round(grad_s, 4), "first_call_seconds": round(first_s, 4), "J": J.item(),
                        "forward_step_equivalents": round(grad_s / fwd_s / T, 2),
                        "note": "forward with checkpoints + recomputation of every segment + adjoint, "
                                "wall clock including host-side launch, checkpoint copies and the save and "
                                "restore of the solver's state; the second of two calls (the first also "
                                "allocates its buffers)"}}
    log(out)
    print(json.dumps(out), flush=True)


def stride_sweep(torch, args):
    """U-19A (19-stream in-place update, the AA even-step traffic) for stream
    strides padded by different amounts: the effect of the paper's padding
    (Sect. 4.3) on the GPU."""
    from paper_1410_0412_amd import bench_stream

    n = 3336242
    base = (n + 63) // 64 * 64
    mib2 = (2 << 20) // 8
    strides = [base + k * 64 for k in (0, 1, 2, 3, 5, 8, 16, 32, 64, 128, 256, 1024)]
    strides += [(n + mib2 - 1) // mib2 * mib2]
    out = {"metric": "U-19A GB/s vs stream stride (2 * 19 * 8 B per node)", "n_gpus": 1, "nodes": n, "rows": []}
    cap = 19 * (max(strides) + mib2)
    buf = torch.zeros(cap, dtype=torch.float64, device="cuda")
    off = (-buf.data_ptr() % (2 << 20)) // 8
    a = buf[off:]
    for ld in strides:
        for _ in range(3):
            bench_stream(2, a, a, n, ld)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(30):
            bench_stream(2, a, a, n, ld)
        e1.record()
        torch.cuda.synchronize()
        gbs = 2 * 8 * 19 * n * 30 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        row = {"stride": ld, "pad_elems": ld - base, "stride_bytes_mod_2MiB": (ld * 8) % (2 << 20), "GBs": round(gbs, 1)}
        out["rows"].append(row)
        log(row)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20,
                    help="timed AA cycles (2 time steps each) per repeat; the default line takes the median of 5")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--odd-schedule", choices=("auto", "band", "chunked"), default="auto",
                    help="workgroup order of the AA odd step in every AA line of the run "
                         "(auto: the solver's choice)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--workload", default=WORKLOAD,
                    help="named synthetic workload of the default line (default: the 384^3 foam)")
    ap.add_argument("--orders", default=None,
                    help="enumeration sweep instead of the default line, e.g. lex:0,lex:8,morton,hilbert")
    ap.add_argument("--with-ia-osnt", action="store_true",
                    help="with --orders: also time FP64 AA-IA and OS-NT with every index source")
    ap.add_argument("--order-traffic", nargs=4, metavar=("SWEEP_JSON", "FETCH_CSV", "WRITE_CSV", "TCP_CSV"),
                    help="per-enumeration counter traffic of an --orders sweep (one JSON document) and exit")
    ap.add_argument("--trace-summary", default=None, metavar="KERNEL_TRACE_CSV",
                    help="print per-variant launch statistics of a rocprofv3 kernel trace and exit")
    ap.add_argument("--traffic-requests", nargs=2, metavar=("RDREQ_CSV", "WRREQ_CSV"),
                    help="with --traffic-from: request-count counter files for the cross-check")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic_<workload>.json from two rocprofv3 --pmc counter files and exit")
    ap.add_argument("--traffic-command", default="", help="command recorded with --traffic-from")
    ap.add_argument("--traffic-out", default=None, help="with --traffic-from: write here instead of profiles/traffic_<workload>.json")
    ap.add_argument("--adjoint", action="store_true",
                    help="time the forward PBB step, the adjoint step and one gradient on the 128^3 sphere pack")
    ap.add_argument("--micro-sizes", default=None,
                    help="micro-benchmarks only, at these node counts (comma separated), one JSON line")
    ap.add_argument("--stride-sweep", action="store_true",
                    help="U-19A bandwidth against the padding of the stream stride")
    ap.add_argument("--pattern-study", default=None,
                    help="AA and OS-NT (RIA) in FP64/FP32/FP16 on these workloads (comma separated), one JSON line")
    ap.add_argument("--size-sweep", default=None,
                    help="AA-RIA FP64/FP32 MFLUP/s on these workloads (comma separated), one JSON line")
    ap.add_argument("--precision-study", action="store_true",
                    help="FP32/FP16 deviation storage vs FP64 after --steps time steps on --workload")
    args = ap.parse_args()
    ODD_SCHEDULE[0] = args.odd_schedule
    if args.order_traffic:
        print(json.dumps(order_traffic(*args.order_traffic), indent=1))
        return
    if args.trace_summary:
        for row in trace_summary(args.trace_summary):
            print(json.dumps(row))
        return
    if args.traffic_from:
        req = args.traffic_requests or (None, None)
        doc = traffic_from(args.traffic_from[0], args.traffic_from[1], args.workload, args.traffic_command,
                           out_path=args.traffic_out, rdreq_csv=req[0], wrreq_csv=req[1])
        print(json.dumps(doc["kernels"], indent=1))
        return
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the solver has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    from lbm_inputs import workload
    from paper_1410_0412_amd import Lattice

    if args.orders:
        return order_sweep(torch, args)
    if args.precision_study:
        return precision_study(torch, args)
    if args.size_sweep:
        return size_sweep(torch, args)
    if args.pattern_study:
        return pattern_study(torch, args)
    if args.stride_sweep:
        return stride_sweep(torch, args)
    if args.adjoint:
        return adjoint_bench(torch, args)
    if args.micro_sizes:
        rows = {}
        for n in (int(x) for x in args.micro_sizes.split(",")):
            rows[n] = microbench(torch, n)
            log(n, rows[n])
        print(json.dumps({"metric": "micro-benchmark GB/s vs node count (2 * 19 * 8 B per node; copy: 2 * 19 * ld * 8 B)",
                          "n_gpus": 1, "data": "synthetic", "sizes": rows}), flush=True)
        return
    return main_line(torch, args)


def time_line(torch, lat, p, pattern, ria, prec, args, remap=True, trt_magic=None):
    """One variant of the default line: ``REPEATS`` runs of ``args.steps``
    cycles; events around every launch on lattices whose steps take
    milliseconds, around sampled launches on smaller ones."""
    every = 1 if lat.n_fluid >= 10_000_000 else 16
    return time_variant(torch, lat, p, pattern, ria, prec, args.steps, args.warmup, remap, sample_every=every,
                        repeats=REPEATS, trt_magic=trt_magic)


def line_row(tm, N, idx_bytes, pattern, prec, steps, workload_name=None):
    """Rates and Roofline fractions of one timed variant (median repeat)."""
    med = tm.median_wall()
    mflups = 2 * N * steps / med / 1e6
    sb = {"f64": 8, "f32": 4, "f16": 2}[prec]
    idx = idx_bytes[tm.index]
    if pattern == "aa":
        kinds = ("even", "odd")
        avg = (kernel_bytes("even", N, idx, sb) + kernel_bytes("odd", N, idx, sb)) / 2
    else:
        kinds = ("osnt", "osnt_b")
        avg = kernel_bytes("osnt", N, idx, sb)
    bl = avg / N
    rates = sorted(2 * N * steps / w / 1e6 for w in tm.walls)
    row = {
        "mflups": round(mflups, 1),
        "index": tm.index,
        "repeats_mflups": [round(r, 1) for r in rates],
        "ms_per_time_step": round(med / (2 * steps) * 1e3, 4),
        "kernel_us": {kinds[0]: round(float(np.mean(tm.first)) * 1e6, 2),
                      kinds[1]: round(float(np.mean(tm.second)) * 1e6, 2)},
        "kernel_samples": [int(len(tm.first)), int(len(tm.second))],
        "loop_balance_B_per_FLUP": round(bl, 3),
        "hbm_gbs_model": round(mflups * bl / 1e3, 1),
        "frac_of_hbm_roofline": round(mflups / (HBM_PEAK_GBS * 1e3 / bl), 4),
    }
    if workload_name:
        row["workload"] = workload_name
        row["fluid_nodes"] = N
    return row


def main_line(torch, args):
    """The default line: AA-RIA FP64 (value) and FP32 on ``args.workload``,
    the other propagation variants beside them, AA-RIA FP64/FP32 on the
    sphere pack, the matched micro-benchmarks, the dominant kernel's
    Roofline and the oracle on the host."""
    from lbm_inputs import workload
    from paper_1410_0412_amd import Lattice

    name = args.workload
    log("generating", name)
    mask, p = workload(name, seed=args.seed)
    t0 = time.perf_counter()
    lat = Lattice(mask, p["periodic"], p["order"], p["block"])
    t_build = time.perf_counter() - t0
    N, R = lat.n_fluid, lat.n_runs
    r = R / N
    log("lattice N=%d R=%d r=%.4f built in %.2fs" % (N, R, r, t_build))

    idx_bytes = lat.index_bytes()
    log("index bytes per node and indirect step", {k: round(v, 3) for k, v in idx_bytes.items()})
    # RIA lines use the library's choice between the paper's runs and
    # per-direction runs ("auto"); the paper's runs are also timed on their own
    # (pattern, index, storage, XCD-aware tile order, TRT collision)
    variants = [("aa", "auto", "f64", True, False), ("aa", "auto", "f32", True, False)]
    if not args.no_variants:
        variants += [("aa", "runs", "f64", True, False), ("aa", False, "f64", True, False),
                     ("osnt", False, "f64", True, False), ("osnt", "auto", "f64", True, False),
                     ("osnt", "runs", "f64", True, False), ("aa", "auto", "f16", True, False),
                     ("aa", "auto", "f64", False, False), ("aa", "auto", "f64", True, True),
                     ("aa", "auto", "f32", True, True)]
    names = {"auto": "ria", "runs": "ria_runs", False: "ia"}
    res = {}
    for pattern, ria, prec, remap, trt in variants:
        key = "%s_%s_%s%s%s" % (pattern, names[ria], "trt_" if trt else "", prec, "" if remap else "_no_xcd_remap")
        log("timing", key)
        # the paper's TRT operator with the magic parameter 3/16 (Sect. 2)
        tm = time_line(torch, lat, p, pattern, ria, prec, args, remap, trt_magic=3.0 / 16.0 if trt else None)
        res[key] = line_row(tm, N, idx_bytes, pattern, prec, args.steps)
        if key == "aa_ria_f64":
            main_tm = tm
        log(key, res[key])

    micro = microbench(torch, N)
    log("micro-benchmarks GB/s", micro)
    # Sect. 5.2: the Roofline with the access-pattern-matched micro-benchmark
    # as the bandwidth: the 19-row update (AA) or copy (OS-NT) in the
    # tile-major layout the grids use, in plain launch order or launched as
    # the step kernel is (U-19T / U-19T-L, CNT-19T / CNT-19T-L), whichever
    # is faster
    matched = {"aa": max(micro["U-19T"], micro["U-19T-L"]), "osnt": max(micro["CNT-19T"], micro["CNT-19T-L"])}
    for key, row in res.items():
        bw = matched["aa" if key.startswith("aa") else "osnt"]
        row["frac_of_matched_roofline"] = round(row["mflups"] / (bw * 1e3 / row["loop_balance_B_per_FLUP"]), 4)

    side = SIDE_WORKLOAD if name != SIDE_WORKLOAD else None
    if side and not args.no_variants:
        # the sphere pack (short runs, r = 0.67) beside the foam
        log("generating", side)
        smask, sp = workload(side, seed=args.seed)
        slat = Lattice(smask, sp["periodic"], sp["order"], sp["block"])
        sib = slat.index_bytes()
        for prec in ("f64", "f32"):
            key = "spherepack_aa_ria_" + prec
            log("timing", key)
            tm = time_line(torch, slat, sp, "aa", "auto", prec, args)
            res[key] = line_row(tm, slat.n_fluid, sib, "aa", prec, args.steps, side)
            log(key, res[key])
        del slat, smask

    aa = res["aa_ria_f64"]
    main_index = main_tm.index
    odd_bytes = kernel_bytes("odd", N, idx_bytes[main_index])
    odd_s = float(np.mean(main_tm.second))
    achieved = odd_bytes / odd_s / 1e9
    odd_kernel = ODD_KERNEL[main_index]
    traffic = measured_traffic(odd_kernel, name)
    enum = "lex B=%d" % p["block"] if p["block"] > 1 else "lex (no blocking)"
    out = {
        "metric": METRIC,
        "value": aa["mflups"],
        "unit": "MFLUP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_tm.median_wall() / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": name,
            "variant": "AA-RIA",
            "ria_index": main_index,
            "index_bytes_per_node": {k: round(v, 3) for k, v in idx_bytes.items()},
            "direction_runs": lat.n_direction_runs,
            "step": "one AA cycle: direct even step + indirect odd step (2 time steps)",
            "timing": "median of %d repeats of `steps` cycles, each between two synchronisations; "
                      "kernel durations from HIP events on the solver's stream" % REPEATS,
            "fluid_nodes": N, "runs": R, "runs_per_node": round(r, 5),
            "box": list(mask.shape),
            "porosity": round(float(1.0 - mask.mean()), 5),
            "tau": p["tau"], "force": list(p["force"]),
            "enumeration": enum,
            "odd_schedule": odd_schedule_name(lat, "f64", idx_bytes[main_index]),
            "lattice_build_s": round(t_build, 3),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": odd_kernel,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": int(odd_bytes),
            "slot_bits": slot_bits(N),
            "avg_launch_us": round(odd_s * 1e6, 2),
            "launch_samples": int(len(main_tm.second)),
            # the counter-measured bytes (traffic) per launch over the same duration
            "traffic_GBs": round(traffic / odd_s / 1e9, 1) if traffic else None,
        },
        "hbm_roofline_mflups": {
            "loop_balance_B_per_FLUP": aa["loop_balance_B_per_FLUP"],
            "roofline_mflups_at_8TBs": round(HBM_PEAK_GBS * 1e3 / aa["loop_balance_B_per_FLUP"], 1),
            "frac": aa["frac_of_hbm_roofline"],
            "matched_benchmark": "U-19T" if micro["U-19T"] >= micro["U-19T-L"] else "U-19T-L",
            "matched_bandwidth_GBs": matched["aa"],
            "matched_roofline_mflups": round(matched["aa"] * 1e3 / aa["loop_balance_B_per_FLUP"], 1),
            "frac_of_matched_roofline": aa["frac_of_matched_roofline"],
            "paper_model_B_l_aa_r": round(304 + 38 * r, 3),
            "frac_of_paper_model_roofline": round(aa["mflups"] / (HBM_PEAK_GBS * 1e3 / (304 + 38 * r)), 4),
        },
        "fp32": {"value": res["aa_ria_f32"]["mflups"], "unit": "MFLUP/s",
                 "index": res["aa_ria_f32"]["index"],
                 "frac_of_hbm_roofline": res["aa_ria_f32"]["frac_of_hbm_roofline"],
                 "frac_of_matched_roofline": res["aa_ria_f32"]["frac_of_matched_roofline"],
                 "loop_balance_B_per_FLUP": res["aa_ria_f32"]["loop_balance_B_per_FLUP"],
                 "kernel_us": res["aa_ria_f32"]["kernel_us"],
                 "storage": "d_q = f_q - w_q rho0 in FP32, FP32 arithmetic"},
        "variants": res,
        "microbench_GBs": micro,
    }
    del lat
    if not args.no_cpu_baseline:
        log("timing the oracle on the host")
        out["cpu_baseline"] = cpu_baseline(mask, p, name)
    print(json.dumps(out), flush=True)

if __name__ == "__main__":
    main()
