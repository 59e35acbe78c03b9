"""Benchmark: MRG32k3a multi-stream generation on one MI355X.

One step = create 262,144 streams on the device from a seeded random 6-word
seed (2^127 jump-ahead) + generate 2^30 fp64 uniforms from them (4,096 per
stream, element k*S + s = draw k of stream s) + the state write-back.
Inputs and outputs stay in HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--copy-probe] [--serve-seconds T]
    python bench.py --pmc-summary FETCH_CSV WRITE_CSV BENCH_LOG
    python bench.py --trace-summary KERNEL_TRACE_CSV BENCH_LOG
    python bench.py --valu-summary VALU_CSV BENCH_LOG
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

S_STREAMS = 262144
PER_STREAM = 4096
N = S_STREAMS * PER_STREAM
HBM_PEAK_GBPS = 8000.0
# every source the profiled kernels are compiled or planned from: counters
# taken before a change to any of them no longer describe the kernels
KERNEL_SRCS = [os.path.join(ROOT, "paper_2201_06604_amd", "csrc", f)
               for f in ("mrg_kernels.hip", "mrg_engine.h", "mrg_math.h", "mrg_internal.h", "mrg_logtab.h",
                         "mrg_sincostab.h", "mrg_tuned.h", "mrg_tables.hip", "mrg_hyper.h", "mrg_batch.cpp")]
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "gen_kernel_uniform_f64_262144x4096_traffic.json")
COPY_PROBE_BYTES = 1 << 30
# VALU issue ceiling: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one lane-instruction
# per lane per cycle; gfx950 issues fp64 FMA at full rate)
VALU_PEAK_LANE_INSTR = 256 * 4 * 16 * 2.4e9
# Op model: lane-instructions per draw of each kind, counted with SQ_INSTS_VALU
# on the 2^30-draw launches of the first complete kernels and frozen here as
# the algorithmic work of a draw, so that a kernel that does the same work in
# fewer instructions shows as a higher fraction rather than a smaller model;
# issued_frac (the kernel's own measured instructions over the same time and
# ceiling) is reported beside it.  The fp32 normals and exponentials changed
# method (fp32 series on the fp64 tables instead of the fp64 transform rounded),
# so theirs are the new kernels' counts: VALU instructions of the main loop of
# the gfx950 assembly over the draws one iteration stores (the same count gives
# 18.17 for fp64 uniforms, measured 18.18, and 19.17 for fp32 uniforms,
# measured 19.29)
OPS_PER_DRAW = {"f64_uniform": 18.2, "f32_uniform": 19.6, "f64_normal": 54.9, "f64_exponential": 48.3,
                "f32_normal": 36.1, "f32_exponential": 32.2}
# The same for the contingency-table kernels: lane-instructions per table of
# the 10^6-table mix and per Fisher replicate of the 7 x 12 table, counted with
# SQ_INSTS_VALU on the tables kernel with 6 checkpoints and the Fisher kernel
# with 8 (their inversion loops' trip counts depend on the margins), frozen
OPS_PER_TABLE = {"tables_kernel": 43136.9, "fisher_kernel": 692654.1}
VALU_JSON = os.path.join(ROOT, "profiles", "gen_kernels_valu_262144x4096.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle cpu_baseline leg")
    ap.add_argument("--no-variants", action="store_true", help="skip f32/normal/exponential timings")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-plain comparison")
    ap.add_argument("--no-tables", action="store_true", help="skip the contingency-table / Fisher timings")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-loop measurement")
    ap.add_argument("--no-paper", action="store_true",
                    help="skip the MRG31k3p and paper-geometry (rnormGpu example) timings")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="seconds of Poisson arrivals per serving rate and mode")
    ap.add_argument("--trace-summary", nargs=2, metavar=("KERNEL_TRACE_CSV", "BENCH_LOG"), default=None,
                    help="per-kernel duration statistics of a rocprofv3 --kernel-trace run of bench.py "
                         "(markdown on stdout), with the timed launches of the headline kernel "
                         "separated from its warm-up ones, then exit")
    ap.add_argument("--valu-summary", nargs=2, metavar=("VALU_CSV", "BENCH_LOG"), default=None,
                    help="turn a rocprofv3 --pmc SQ_INSTS_VALU run of bench.py into the per-unit "
                         "instruction counts under profiles/, then exit")
    ap.add_argument("--pmc-summary", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "BENCH_LOG"), default=None,
                    help="turn two rocprofv3 --pmc counter CSVs (FETCH_SIZE, WRITE_SIZE) of a "
                         "--copy-probe run into the traffic summary under profiles/, then exit; the "
                         "kernel-source hash is read from the profiled run's own JSON line in BENCH_LOG")
    return ap.parse_args()


def kernel_sha():
    import hashlib
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def pmc_summary(fetch_csv, write_csv, bench_log):
    """HBM bytes per launch of the fp64-uniform generate kernel from the
    FETCH_SIZE and WRITE_SIZE counters (KiB per dispatch), each scaled by what
    the same counter reads for the 1 GiB copy of --copy-probe."""
    import csv

    def per_kernel(path, counter):
        acc = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            acc.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in acc.items()}

    fetch, write = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    sha = None
    with open(bench_log) as f:
        for line in f:
            if line.startswith("{"):
                sha = json.loads(line)["roofline"].get("source_sha256")
    if not sha:
        sys.exit("no kernel-source hash in " + bench_log)

    def pick(d, pred):
        ks = [k for k in d if pred(k)]
        assert len(ks) == 1, ks
        return d[ks[0]], ks[0]

    # the fp64-uniform generate kernel that writes the most: the 2^30-draw
    # launch (the run also has small-grid launches of another instance)
    gens = [k for k in write if "gen_kernel<0, 0," in k]
    name = max(gens, key=lambda k: write[k])
    is_copy = lambda k: "copyBuffer" in k
    g_f, g_w = fetch[name], write[name]
    c_f, _ = pick(fetch, is_copy)
    c_w, _ = pick(write, is_copy)
    kib = COPY_PROBE_BYTES / 1024.0
    f_fac, w_fac = kib / c_f, kib / c_w
    out = {"kernel": name, "workload": "262144 streams x 4096 fp64 uniforms",
           "fetch_kib": g_f, "write_kib": g_w, "copy_fetch_kib": c_f, "copy_write_kib": c_w,
           "fetch_factor": f_fac, "write_factor": w_fac,
           "bytes_per_launch": (g_f * f_fac + g_w * w_fac) * 1024.0,
           "source_sha256": sha}
    with open(TRAFFIC_JSON, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def measured_traffic():
    """Traffic per launch, only while the kernel source is the one measured."""
    if not os.path.exists(TRAFFIC_JSON):
        return None
    with open(TRAFFIC_JSON) as f:
        t = json.load(f)
    return t["bytes_per_launch"] if t.get("source_sha256") == kernel_sha() else None


def trace_summary(kt_csv, bench_log):
    """Markdown table of per-kernel durations from a rocprofv3 kernel-trace
    CSV of one bench.py run; the headline kernel (the fp64-uniform generate
    launch over 2^30 draws) is also summarised over its last `steps`
    dispatches, the ones inside the timed region, next to the same run's own
    HIP-event figures from its JSON line."""
    import csv
    rows = list(csv.DictReader(open(kt_csv)))
    line = None
    with open(bench_log) as f:
        for ln in f:
            if ln.startswith("{"):
                line = json.loads(ln)
    if line is None:
        sys.exit("no JSON line in " + bench_log)
    by = {}
    for r in rows:
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3  # ns -> us
        by.setdefault(r["Kernel_Name"], []).append((int(r["Start_Timestamp"]), d))
    total = sum(d for v in by.values() for _, d in v)
    print("| Kernel | Calls | Avg (us) | Median (us) | Min (us) | Max (us) | % of GPU time |")
    print("|---|---|---|---|---|---|---|")
    for k, v in sorted(by.items(), key=lambda kv: -sum(d for _, d in kv[1])):
        ds = sorted(d for _, d in v)
        name = k if len(k) <= 90 else k[:87] + "..."
        print(f"| `{name}` | {len(ds)} | {np.mean(ds):.1f} | {np.median(ds):.1f} | {ds[0]:.1f} | {ds[-1]:.1f} | "
              f"{100 * sum(ds) / total:.2f} |")
    gens = [k for k in by if "gen_kernel<0, 0," in k]
    head = max(gens, key=lambda k: max(d for _, d in by[k]))
    steps = int(line["steps"])
    timed = [d for _, d in sorted(by[head])][-steps:]
    alg = line["roofline"]["alg_bytes_per_launch"]
    avg = float(np.mean(timed))
    print()
    print(f"Headline kernel `{head}`: the last {steps} dispatches (the timed region) average "
          f"{avg:.1f} us (median {np.median(timed):.1f}, min {min(timed):.1f}); "
          f"{alg / 1e9:.4f} GB / {avg / 1e3:.4f} ms = {alg / (avg * 1e-6) / 1e9:.1f} GB/s = "
          f"{alg / (avg * 1e-6) / 1e9 / HBM_PEAK_GBPS:.4f} of {HBM_PEAK_GBPS:.0f} GB/s.")
    rf = line["roofline"]
    print(f"The same run's JSON line (HIP events around each timed launch): avg_launch_ms {rf['avg_launch_ms']}, "
          f"median {rf['launch_ms_median']}, min {rf['launch_ms_min']}, achieved {rf['achieved']} GB/s, "
          f"frac {rf['frac']}; ms_per_step {line['ms_per_step']}, value {line['value']}.")


def valu_summary(valu_csv, bench_log):
    """Lane-instructions per unit of the measured kernels from a rocprofv3
    --pmc run of bench.py with SQ_INSTS_VALU and GRBM_GUI_ACTIVE (wave-
    instructions per dispatch x 64 lanes / the units the dispatch processed),
    and each kernel's VALU busy (SQ_INSTS_VALU x 4 cycles over the 1,024 SIMDs
    and the dispatch's busy cycles per XCD, GRBM_GUI_ACTIVE / 8), written to
    the JSON the bench reads while the kernel sources are unchanged.  Units:
    draws for the 2^30-draw generate launches (the dispatch of each kind with
    the most instructions) and for the last batch launch (a graph replay over
    the whole mix); tables for the 10^6-table launch; replicates for the
    largest Fisher launch (Table 2, B = 10,027,008)."""
    import csv
    per = {}
    for r in csv.DictReader(open(valu_csv)):
        key = (int(r["Dispatch_Id"]), r["Kernel_Name"])
        c = per.setdefault(key, {})
        c[r["Counter_Name"]] = c.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    line = None
    with open(bench_log) as f:
        for ln in f:
            if ln.startswith("{"):
                line = json.loads(ln)
    if line is None:
        sys.exit("no JSON line in " + bench_log)

    def busy(c):
        cyc = c.get("GRBM_GUI_ACTIVE", 0.0) / 8
        return c["SQ_INSTS_VALU"] * 4 / (1024 * cyc) if cyc else None

    def biggest(pred):
        """The dispatch with the most instructions, its VALU busy replaced by
        the median over every dispatch of that size (timed repetitions of one
        launch differ only in clock and neighbours)."""
        ks = [(c.get("SQ_INSTS_VALU", 0.0), d, k) for (d, k), c in per.items() if pred(k)]
        if not ks:
            return None
        top, d, k = max(ks)
        same = sorted(b for b in (busy(per[(d2, k2)]) for v, d2, k2 in ks if abs(v - top) <= 1e-3 * top)
                      if b is not None)
        c = dict(per[(d, k)])
        c["busy"] = same[len(same) // 2] if same else None
        return c

    out = {"source_sha256": line["roofline"]["source_sha256"], "per_unit": {}, "valu_busy": {}, "workload": {}}

    def put(name, c, units, what):
        if c is None:
            return
        out["per_unit"][name] = c["SQ_INSTS_VALU"] * 64 / units
        b = c["busy"] if "busy" in c else busy(c)
        out["valu_busy"][name] = round(b, 4) if b is not None else None
        out["workload"][name] = what

    for name, prefix in [("f64_uniform", "gen_kernel<0, 0,"), ("f32_uniform", "gen_kernel<0, 1,"),
                         ("f64_normal", "gen_kernel<1, 0,"), ("f64_exponential", "gen_kernel<2, 0,"),
                         ("f32_normal", "gen_kernel<1, 1,"), ("f32_exponential", "gen_kernel<2, 1,")]:
        put(name, biggest(lambda k, p=prefix: p in k), N, f"{S_STREAMS} streams x {PER_STREAM} draws, per draw")
    put("tables_kernel", biggest(lambda k: "tables_kernel" in k), 1_000_000,
        "10^6 tables of the CFG4 mix, per table")
    put("fisher_kernel", biggest(lambda k: "fisher_kernel" in k), 10027008,
        "Table 2 (7 x 12), B = 10,027,008 replicates, per replicate")
    batch = sorted((d, k) for (d, k) in per
                   if any(n + "(" in k for n in ("batch_kernel", "batch_gang_kernel", "batch_gang_narrow_kernel")))
    if batch and "batched" in line:
        put("batch_kernel", per[batch[-1]], line["batched"]["draws"],
            "the 4,096-request mix (last launch: a graph replay), per draw")
    with open(VALU_JSON, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def valu_profile():
    """Measured lane-instructions per unit of the kernels the committed VALU
    counter profile covers, only while the kernel sources are the ones
    measured (None otherwise)."""
    if not os.path.exists(VALU_JSON):
        return None
    with open(VALU_JSON) as f:
        t = json.load(f)
    return t if t.get("source_sha256") == kernel_sha() else None


def alu_roofline(ops_per_unit, units, ms, measured_per_unit=None):
    """VALU roofline entry: ops_per_unit x units lane-instructions in `ms`
    against the 2.4 GHz issue ceiling."""
    achieved = ops_per_unit * units / (ms * 1e-3)
    out = {"bound": "alu", "achieved": round(achieved / 1e12, 3), "peak": round(VALU_PEAK_LANE_INSTR / 1e12, 2),
           "unit": "T lane-instr/s", "frac": round(achieved / VALU_PEAK_LANE_INSTR, 4),
           "ops_per_unit": ops_per_unit}
    if measured_per_unit is not None:
        out["measured_ops_per_unit"] = round(measured_per_unit, 2)
        out["issued_frac"] = round(measured_per_unit * units / (ms * 1e-3) / VALU_PEAK_LANE_INSTR, 4)
    return out


def timed_median(torch, fn, reps=5, inner=3, warm_ms=50.0):
    """Median over `reps` of the mean time (ms, HIP events on the current
    stream) of `inner` back-to-back calls, after calls for at least `warm_ms`
    of wall time, so that a leg that follows an idle GPU is not timed while
    the clocks are still coming up."""
    t0 = time.perf_counter()
    while True:
        fn()
        torch.cuda.synchronize()
        if (time.perf_counter() - t0) * 1e3 >= warm_ms:
            break
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(inner):
            fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b) / inner)
    return sorted(ts)[len(ts) // 2]


def cpu_baseline(seed):
    """The oracle, as it is, on the host cores: all 262,144 streams x 4,096
    fp64 uniforms (2^30 draws, ~15 s of CPU work), split over threads."""
    import oracle as O
    threads = max(1, min(16, os.cpu_count() or 1))
    S_sample = S_STREAMS
    c = seed.copy()
    rec = O.create_streams(O.MRG32K3A, c, S_sample)
    n = S_sample * PER_STREAM
    t0 = time.perf_counter()
    O.generate(O.MRG32K3A, rec, n, O.UNIFORM, O.F64, 1.0, threads=threads)
    dt = time.perf_counter() - t0
    # one thread, on the first 16,384 streams (1/16 of the workload)
    sub = O.create_streams(O.MRG32K3A, seed.copy(), 16384)
    t1 = time.perf_counter()
    O.generate(O.MRG32K3A, sub, 16384 * PER_STREAM, O.UNIFORM, O.F64, 1.0, threads=1)
    dt1 = time.perf_counter() - t1
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": n / dt / 1e9, "unit": "GSamples/s", "cores": threads, "kind": "oracle",
            "sample": f"{S_sample} streams x {PER_STREAM} fp64 uniforms, the whole workload "
                      f"({n} draws, {dt:.2f} s wall on {threads} threads)",
            "single_thread": {"value": 16384 * PER_STREAM / dt1 / 1e9, "unit": "GSamples/s",
                              "sample": f"16384 streams x {PER_STREAM} fp64 uniforms ({dt1:.2f} s)"},
            "cpu_model": model, "nproc": os.cpu_count()}


def oracle_threads():
    return max(1, min(16, os.cpu_count() or 1))


def oracle_rate(gen_seed, S, per, dist, dtype, param=1.0):
    """The oracle generating `per` draws of each of S streams on the host
    cores (streams split over threads): (GSamples/s, seconds, threads)."""
    import oracle as O
    rec = O.create_streams(O.MRG32K3A, gen_seed.copy(), S)
    th = oracle_threads()
    t0 = time.perf_counter()
    O.generate(O.MRG32K3A, rec, S * per, dist, dtype, param, threads=th)
    dt = time.perf_counter() - t0
    return S * per / dt / 1e9, dt, th


def bench_small(torch, P, workloads, reps=50):
    """The paper-shaped small case: seed 12345 x 6, 1,024 streams created on
    the device, 1,024 fp64 uniforms each (2^20): launch-bound, so latency per
    call (median and min of 50, HIP events), and the oracle on one core."""
    import oracle as O
    st = P.new_streams_tensor(1024)
    out = torch.empty(1 << 20, dtype=torch.float64, device="cuda")

    def create_gen():
        c = P.mrg_creator_init(workloads.PAPER_SEED)
        P.mrg_streams_create_device(c, 1024, out=st)
        P.mrg_generate(st, 1 << 20, P.MRG_UNIFORM, P.MRG_F64, out=out)

    both, gen = [], []
    for _ in range(5):
        create_gen()
    for _ in range(reps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        c = P.mrg_creator_init(workloads.PAPER_SEED)
        P.mrg_streams_create_device(c, 1024, out=st)
        e[1].record()
        P.mrg_generate(st, 1 << 20, P.MRG_UNIFORM, P.MRG_F64, out=out)
        e[2].record()
        torch.cuda.synchronize()
        both.append(e[0].elapsed_time(e[2]) * 1e3)
        gen.append(e[1].elapsed_time(e[2]) * 1e3)
    rec = O.create_streams(O.MRG32K3A, np.array(workloads.PAPER_SEED, dtype=np.uint32), 1024)
    t0 = time.perf_counter()
    O.generate(O.MRG32K3A, rec, 1 << 20, O.UNIFORM, O.F64, 1.0, threads=1)
    oracle_ms = (time.perf_counter() - t0) * 1e3
    return {"workload": "seed 12345 x 6, 1,024 streams created on the device, 1,024 fp64 uniforms each",
            "create_and_generate_us": {"median": round(float(np.median(both)), 1), "min": round(float(min(both)), 1)},
            "generate_us": {"median": round(float(np.median(gen)), 1), "min": round(float(min(gen)), 1)},
            "oracle_one_core_ms": round(oracle_ms, 1)}


def bench_batched(torch, P, workloads, reps=3, with_oracle=True):
    """4,096 generation requests (lengths log-uniform in [1e3, 1e7], 64-1,024
    streams each, random f32/f64 x uniform/normal/exponential) on consecutive
    streams of one creator: 4,096 back-to-back plain launches against one
    autotuned persistent launch replayed from a HIP graph.  Per-request
    latency = completion time from the start of the run (plain: HIP events
    after each launch; batched: device completion stamps)."""
    reqs = workloads.batch_requests()
    total_S = sum(r["n_streams"] for r in reqs)
    total_n = sum(r["n"] for r in reqs)
    c = P.mrg_creator_init(workloads.random_seed())
    streams = P.mrg_streams_create_device(c, total_S)
    dmap = {0: P.MRG_UNIFORM, 1: P.MRG_NORMAL, 2: P.MRG_EXPONENTIAL}
    tmap = {0: (P.MRG_F64, torch.float64), 1: (P.MRG_F32, torch.float32)}
    meta, creqs = [], []
    for r in reqs:
        dist = dmap[r["dist"]]
        dtype, tdt = tmap[r["dtype"]]
        s = streams[r["first_stream"]:r["first_stream"] + r["n_streams"]]
        o = torch.empty(r["n"], dtype=tdt, device="cuda")
        meta.append((s, r["n"], dist, dtype, o))
        creqs.append(P.make_request(s, r["n"], dist, dtype, 1.0, o))
    out_bytes = sum(m[4].numel() * m[4].element_size() for m in meta)

    def plain_once():
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(len(meta) + 1)]
        evs[0].record()
        for i, (s, n, dist, dtype, o) in enumerate(meta):
            P.mrg_generate(s, n, dist, dtype, 1.0, out=o)
            evs[i + 1].record()
        torch.cuda.synchronize()
        return np.array([evs[0].elapsed_time(e) for e in evs[1:]])

    plain_once()
    runs = [plain_once() for _ in range(reps)]
    lat_p = min(runs, key=lambda a: a[-1])

    tune = P.BatchPlan(creqs, dict(tile_units=1024))
    plan = P.BatchPlan(creqs)
    plan.alloc_workspace(max(tune.workspace_size(), plan.workspace_size()))
    del tune
    plan.upload()
    best, _ = plan.autotune()
    g = torch.cuda.CUDAGraph()
    st = torch.cuda.Stream()
    with torch.cuda.graph(g, stream=st):
        plan.launch(stream=st.cuda_stream)
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    best_ms, lat_b = None, None
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        g.replay()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        t = plan.request_times()
        lat = (t[1:].astype(np.float64) - float(t[0])) * 1e-5  # 100 MHz ticks -> ms
        if best_ms is None or ms < best_ms:
            best_ms, lat_b = ms, lat
    del g

    def stats(ms, lat):
        return {"makespan_ms": round(float(ms), 3), "GSamples_per_s": round(total_n / (ms * 1e-3) / 1e9, 2),
                "GB_per_s": round(out_bytes / (ms * 1e-3) / 1e9, 1),
                "p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3)}

    res = {"workload": "4096 requests, lengths log-uniform in [1e3, 1e7], 64-1024 streams each, "
                       "random f32/f64 x uniform/normal/exponential(rate 1)",
           "requests": len(reqs), "streams": total_S, "draws": total_n, "output_bytes": out_bytes,
           "plain": stats(lat_p[-1], lat_p), "batched": stats(best_ms, lat_b),
           "batched_tuning": best}
    kind = {(0, 0): "f64_uniform", (0, 1): "f32_uniform", (1, 0): "f64_normal", (1, 1): "f32_normal",
            (2, 0): "f64_exponential", (2, 1): "f32_exponential"}
    ops = sum(r["n"] * OPS_PER_DRAW[kind[(r["dist"], r["dtype"])]] for r in reqs)
    vp = valu_profile()
    meas = vp["per_unit"].get("batch_kernel") if vp else None
    res["roofline"] = alu_roofline(ops / total_n, total_n, best_ms, meas)
    res["roofline"]["hbm_frac"] = round(out_bytes / (best_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)
    res["roofline"]["kernel"] = ("batch_kernel" if best.get("gang_waves", 1) <= 1 else
                                 "batch_gang_narrow_kernel" if best.get("wide_stores") == 1 else
                                 "batch_gang_kernel") + \
        " (persistent, graph-replayed)"
    if meas is not None:
        # issued_frac counts the algorithmic work plus idle lanes of partial
        # waves, per-tile jumps and tails
        res["roofline"]["valu_busy_profiled"] = vp.get("valu_busy", {}).get("batch_kernel")
    res["speedup_makespan"] = round(res["plain"]["makespan_ms"] / res["batched"]["makespan_ms"], 2)
    res["p99_ratio_plain_over_batched"] = round(res["plain"]["p99_ms"] / res["batched"]["p99_ms"], 2)
    for m in meta:
        del m
    if with_oracle:
        res["oracle"] = batch_oracle_sample(reqs, workloads.random_seed())
    return res


def batch_oracle_sample(reqs, seed, every=16):
    """The oracle on every 16th request of the batch mix (each on its own
    streams, reached by one 2^127-step jump per stream offset), requests
    spread over the host threads."""
    import oracle as O
    from concurrent.futures import ThreadPoolExecutor
    dmap = {0: O.UNIFORM, 1: O.NORMAL, 2: O.EXPONENTIAL}
    tmap = {0: O.F64, 1: O.F32}
    sample = reqs[::every]

    def one(r):
        c = seed.copy()
        O.jump(O.MRG32K3A, c, r["first_stream"] * 2**127)
        rec = O.create_streams(O.MRG32K3A, c, r["n_streams"])
        O.generate(O.MRG32K3A, rec, r["n"], dmap[r["dist"]], tmap[r["dtype"]], 1.0)

    th = oracle_threads()
    t0 = time.perf_counter()
    with ThreadPoolExecutor(th) as ex:
        list(ex.map(one, sample))
    dt = time.perf_counter() - t0
    n = sum(r["n"] for r in sample)
    return {"value": round(n / dt / 1e9, 4), "unit": "GSamples/s", "cores": th, "kind": "oracle",
            "sample": f"every {every}th request ({len(sample)} requests, {n} draws, {dt:.2f} s)"}


def bench_tables(torch, P, workloads, reps=10, with_oracle=True):
    """Section 4 consumer: 1e6 random 2x2..5x5 tables with fixed margins
    (totals 5..200), one stream each, per launch (HIP events); and fisher.sim
    on the two tables the paper tests (12 x 12 with B = 2^20, 7 x 12 with
    B = 10,027,008), one MRG32k3a stream per replicate."""
    def read_golden(name):
        with open(os.path.join(ROOT, "tests", "golden", name)) as f:
            return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]

    n = 1_000_000
    I, J, rows, cols = workloads.contingency_margins(n)
    c = P.mrg_creator_init(workloads.random_seed())
    d = P.mrg_streams_create_device(c, n)
    dI, dJ, dr, dc = [torch.from_numpy(a).cuda() for a in (I, J, rows, cols)]
    tabs = torch.empty((n, 5, 5), dtype=torch.int32, device="cuda")
    stats = torch.empty(n, dtype=torch.float64, device="cuda")
    P.mrg_tables_sample(d, dI, dJ, dr, dc, tables=tabs, stats=stats)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        P.mrg_tables_sample(d, dI, dJ, dr, dc, tables=tabs, stats=stats)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    draws = int(((I - 1) * (J - 1)).sum())
    res = {"workload": "1e6 tables, shapes 2x2..5x5, margins uniform 5..200, 1 stream per table, "
                       "int32 tables + statistic",
           "ms": round(ms, 3), "Mtables_per_s": round(n / ms / 1e3, 1),
           "GUniforms_per_s": round(draws / ms / 1e6, 2)}
    vp = valu_profile()
    meas = vp["per_unit"].get("tables_kernel") if vp else None
    res["roofline"] = alu_roofline(OPS_PER_TABLE["tables_kernel"], n, ms, meas)
    res["roofline"]["kernel"] = "tables_kernel"
    if meas is not None:
        res["roofline"]["valu_busy_profiled"] = vp.get("valu_busy", {}).get("tables_kernel")
    res["roofline"]["note"] = ("ops_per_unit = issued VALU lane-slots per table (wave-instructions x 64, "
                               "SQ_INSTS_VALU, frozen): the inversion loops' trip counts depend on the "
                               "margins, and a wave issues until its longest lane is done")
    del d, tabs, stats
    if with_oracle:
        res["oracle"] = tables_oracle_sample(I, J, rows, cols, workloads.random_seed())
    fis = {}
    for name, B, paper_s in (("fisher_month.txt", 1 << 20, 0.348), ("fisher_week.txt", 10027008, 2.030)):
        tab = np.array([[int(v) for v in r] for r in read_golden(name)], dtype=np.int32)
        c = P.mrg_creator_init(workloads.random_seed(44))
        d = P.mrg_streams_create_device(c, B)
        P.mrg_fisher_sim(d, tab, B=min(B, 4096))
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        cnt, _, _ = P.mrg_fisher_sim(d, tab)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        key = name.split("_")[1].split(".")[0]
        fis[key] = {
            "table": f"{tab.shape[0]}x{tab.shape[1]}", "B": B, "ms": round(ms, 2),
            "Mtables_per_s": round(B / ms / 1e3, 2), "pvalue": round(P.mrg_fisher_pvalue(int(cnt.item()), B), 6),
            "paper_V100_s": paper_s}
        if key == "week":
            meas = vp["per_unit"].get("fisher_kernel") if vp else None
            fis[key]["roofline"] = alu_roofline(OPS_PER_TABLE["fisher_kernel"], B, ms, meas)
            fis[key]["roofline"]["kernel"] = "fisher_kernel"
            if meas is not None:
                fis[key]["roofline"]["valu_busy_profiled"] = vp.get("valu_busy", {}).get("fisher_kernel")
        del d
    res["fisher"] = fis
    if with_oracle:
        tab = np.array([[int(v) for v in r] for r in read_golden("fisher_month.txt")], dtype=np.int32)
        res["fisher"]["oracle"] = fisher_oracle_sample(tab, workloads.random_seed(44))
    return res


def tables_oracle_sample(I, J, rows, cols, seed, n=200_000):
    """The oracle sampling the first 200,000 tables of the mix on the host
    threads (tables split into contiguous blocks)."""
    import oracle as O
    from concurrent.futures import ThreadPoolExecutor
    rec = O.create_streams(O.MRG32K3A, seed.copy(), n)
    th = oracle_threads()
    bounds = np.linspace(0, n, th + 1).astype(int)

    def one(k):
        a, b = bounds[k], bounds[k + 1]
        O.tables(O.MRG32K3A, rec[a:b], I[a:b], J[a:b], rows[a:b], cols[a:b])

    t0 = time.perf_counter()
    with ThreadPoolExecutor(th) as ex:
        list(ex.map(one, range(th)))
    dt = time.perf_counter() - t0
    return {"value": round(n / dt / 1e6, 3), "unit": "Mtables/s", "cores": th, "kind": "oracle",
            "sample": f"first {n} tables of the mix ({dt:.2f} s)"}


def fisher_oracle_sample(tab, seed, B=65536):
    """The oracle's fisher.sim count on the 12 x 12 table with 65,536
    replicates on the host threads."""
    import oracle as O
    from concurrent.futures import ThreadPoolExecutor
    rec = O.create_streams(O.MRG32K3A, seed.copy(), B)
    th = oracle_threads()
    bounds = np.linspace(0, B, th + 1).astype(int)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(th) as ex:
        list(ex.map(lambda k: O.fisher_count(O.MRG32K3A, rec[bounds[k]:bounds[k + 1]], tab), range(th)))
    dt = time.perf_counter() - t0
    return {"value": round(B / dt / 1e6, 3), "unit": "Mtables/s", "cores": th, "kind": "oracle",
            "sample": f"12x12 table, {B} replicates ({dt:.2f} s)"}


def bench_paper(torch, P, workloads, out, reps=5):
    """The paper's own generator and geometry: MRG31k3p fp64 uniforms at the
    throughput size (262,144 streams x 4,096, default launch), and the
    rnormGpu example of Section 3.1 (10^4 x 10^4 fp64 normals from 65,536
    MRG31k3p streams on a 512 x 128 work-item lattice, Listing 2 placement)."""
    G = P.MRG_GEN_MRG31K3P
    c = P.mrg_creator_init(workloads.PAPER_SEED, gen=G)
    st = P.mrg_streams_create_device(c, S_STREAMS, gen=G)

    def timed(fn):
        return timed_median(torch, fn, reps=reps)

    ms = timed(lambda: P.mrg_generate(st, N, P.MRG_UNIFORM, P.MRG_F64, out=out, gen=G))
    res = {"mrg31k3p_uniform_f64": {"GSamples_per_s": round(N / (ms * 1e-3) / 1e9, 1), "ms": round(ms, 4),
                                    "GB_per_s": round((N * 8 + S_STREAMS * 48) / (ms * 1e-3) / 1e9, 1)}}
    del st
    c = P.mrg_creator_init(workloads.PAPER_SEED, gen=G)
    st = P.mrg_streams_create_device(c, 65536, gen=G)
    view = out[:10000 * 10000].view(10000, 10000)
    ms = timed(lambda: P.mrg_generate_paper(st, 10000, 10000, 512, 128, P.MRG_NORMAL, P.MRG_F64, out=view, gen=G))
    res["rnormGpu_10000x10000_512x128"] = {"ms": round(ms, 3), "GSamples_per_s": round(1e8 / (ms * 1e-3) / 1e9, 1),
                                           "paper_s": 0.051}
    return res


def bench_serving(torch, P, workloads, rates=(2000, 5000, 10000, 20000, 50000), duration=10.0):
    """The request loop: Poisson arrivals from 256 sessions (64 device
    streams each), lengths log-uniform in [1e2, 1e6] fp64 normals, a 32 GB
    output pool; continuous batching on 4 HIP streams against one plain
    launch per request.  Latency = completion - arrival."""
    pool = torch.empty(32 << 30, dtype=torch.uint8, device="cuda")
    out = {}
    for rate in rates:
        t, sess, lens = workloads.poisson_arrivals(float(rate), duration, rng_seed=rate)
        row = {}
        for mode, name in ((0, "batched"), (1, "plain")):
            srv = P.Server(256, workloads.random_seed(), pool, mode=mode)
            lat, span = srv.drive((t * 1e9).astype(np.uint64), sess, lens)
            st = srv.stats()
            srv.close()
            lat_ms = lat / 1e6
            row[name] = {"GSamples_per_s": round(float(lens.sum()) / (span / 1e9) / 1e9, 3),
                         "p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
                         "p99_ms": round(float(np.percentile(lat_ms, 99)), 3),
                         "p999_ms": round(float(np.percentile(lat_ms, 99.9)), 3),
                         "pool_peak_MB": round(st["pool_peak"] / 1e6, 1),
                         "launches": int(st["launches"]), "max_in_flight": int(st["max_in_flight"]),
                         "max_lanes_busy": int(st["max_lanes_busy"])}
            print(f"serving {rate}/s {name}: p50 {row[name]['p50_ms']} ms p99 {row[name]['p99_ms']} ms",
                  file=sys.stderr, flush=True)
        out[f"{rate}_per_s"] = dict(requests=int(len(t)), **row)
    del pool
    return {"workload": f"Poisson arrivals for {duration:g} s, 256 sessions x 64 streams, lengths log-uniform "
                        "in [1e2, 1e6] fp64 normals, 32 GB pool", "rates": out}


def main():
    args = parse()
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary)
        return
    if args.trace_summary:
        trace_summary(*args.trace_summary)
        return
    if args.valu_summary:
        valu_summary(*args.valu_summary)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported in this build "
              "(streams shard by block across GPUs with no exchange; see the design notes).",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2201_06604_amd as P
    import workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    seed = workloads.random_seed()
    streams = P.new_streams_tensor(S_STREAMS)
    out = torch.empty(N, dtype=torch.float64, device=dev)

    def step():
        c = P.mrg_creator_init(seed)
        P.mrg_streams_create_device(c, S_STREAMS, out=streams)
        P.mrg_generate(streams, N, P.MRG_UNIFORM, P.MRG_F64, out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: K whole steps; the generate launch is bracketed by events
    # on the stream it runs on (torch's current stream)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        c = P.mrg_creator_init(seed)
        P.mrg_streams_create_device(c, S_STREAMS, out=streams)
        ev[i][0].record()
        P.mrg_generate(streams, N, P.MRG_UNIFORM, P.MRG_F64, out=out)
        ev[i][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gen_ms = [a.elapsed_time(b) for a, b in ev]
    ms_per_step = wall * 1e3 / args.steps
    value = N / (ms_per_step * 1e-3) / 1e9
    gen_avg_ms = float(np.mean(gen_ms))
    alg_bytes = N * 8 + S_STREAMS * 48  # output + state read and written
    achieved = alg_bytes / (gen_avg_ms * 1e-3) / 1e9

    traffic = measured_traffic()

    res = {
        "metric": "GSamples/s MRG32k3a fp64 uniforms (bit-exact); p99 latency, batched vs plain",
        "value": round(value, 3),
        "unit": "GSamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "MRG32k3a: 262,144 streams created on device by 2^127 jump-ahead "
                               "from a seeded random 6-word seed, 4,096 fp64 uniforms each "
                               "(2^30 per step), interleaved output k*S+s",
                   "streams": S_STREAMS, "per_stream": PER_STREAM, "dist": "uniform",
                   "out_dtype": "f64"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": None if traffic is None else int(round(traffic)),
                     "traffic_unit": "bytes per launch",
                     "kernel": "gen_kernel<uniform,f64>", "alg_bytes_per_launch": alg_bytes,
                     "avg_launch_ms": round(gen_avg_ms, 4),
                     "launch_ms_median": round(float(np.median(gen_ms)), 4),
                     "launch_ms_min": round(float(min(gen_ms)), 4), "source_sha256": kernel_sha()},
    }

    # store-only ceiling: torch's fill of the same 8 GiB buffer
    fe = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    out.fill_(0.5)
    fe[0].record()
    for _ in range(5):
        out.fill_(0.5)
    fe[1].record()
    torch.cuda.synchronize()
    fill_ms = fe[0].elapsed_time(fe[1]) / 5
    res["store_only_fill_GBps"] = round(N * 8 / (fill_ms * 1e-3) / 1e9, 1)
    res["achieved_vs_store_only"] = round(achieved / res["store_only_fill_GBps"], 3)

    # store-only ceiling of the generate kernel's own layout (same grid, store
    # width, row order, barriers, cache policy; no numbers computed), timed
    # like the headline launches
    for _ in range(args.warmup):
        P.mrg_store_ceiling(S_STREAMS, N, P.MRG_F64, out=out)
    cev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for a, b in cev:
        a.record()
        P.mrg_store_ceiling(S_STREAMS, N, P.MRG_F64, out=out)
        b.record()
    torch.cuda.synchronize()
    c_ms = [a.elapsed_time(b) for a, b in cev]
    c_avg = float(np.mean(c_ms))
    res["store_ceiling"] = {"kernel": "store_ceiling_kernel (the generate kernel's launch shape)",
                            "avg_launch_ms": round(c_avg, 4), "launch_ms_median": round(float(np.median(c_ms)), 4),
                            "GBps": round(N * 8 / (c_avg * 1e-3) / 1e9, 1)}
    res["achieved_vs_store_ceiling"] = round(achieved / res["store_ceiling"]["GBps"], 3)
    res["roofline"]["frac_of_store_ceiling"] = res["achieved_vs_store_ceiling"]

    if not args.no_variants:
        var = {}
        out32 = torch.empty(N, dtype=torch.float32, device=dev)
        for name, dist, dt, o, esz in [("f32_uniform", P.MRG_UNIFORM, P.MRG_F32, out32, 4),
                                       ("f64_normal", P.MRG_NORMAL, P.MRG_F64, out, 8),
                                       ("f64_exponential", P.MRG_EXPONENTIAL, P.MRG_F64, out, 8),
                                       ("f32_normal", P.MRG_NORMAL, P.MRG_F32, out32, 4),
                                       ("f32_exponential", P.MRG_EXPONENTIAL, P.MRG_F32, out32, 4)]:
            ms = timed_median(torch, lambda: P.mrg_generate(streams, N, dist, dt, 1.0, out=o))
            gbps = N * esz / (ms * 1e-3) / 1e9
            var[name] = {"GSamples_per_s": round(N / (ms * 1e-3) / 1e9, 2),
                         "GB_per_s": round(gbps, 1), "hbm_frac": round(gbps / HBM_PEAK_GBPS, 4),
                         "ms": round(ms, 4)}
            vp = valu_profile()
            meas = vp["per_unit"].get(name) if vp else None
            var[name]["roofline"] = alu_roofline(OPS_PER_DRAW[name], N, ms, meas)
        del out32
        if not args.no_cpu:
            import oracle as O
            for name, od, odt in [("f32_uniform", O.UNIFORM, O.F32), ("f64_normal", O.NORMAL, O.F64),
                                  ("f64_exponential", O.EXPONENTIAL, O.F64), ("f32_normal", O.NORMAL, O.F32),
                                  ("f32_exponential", O.EXPONENTIAL, O.F32)]:
                rate, dt_s, th = oracle_rate(seed, 16384, PER_STREAM, od, odt)
                var[name]["oracle"] = {"value": round(rate, 4), "unit": "GSamples/s", "cores": th,
                                       "kind": "oracle",
                                       "sample": f"16384 streams x {PER_STREAM} ({dt_s:.2f} s)"}
        res["variants"] = var

    res["small"] = bench_small(torch, P, workloads)

    if not args.no_batch:
        res["batched"] = bench_batched(torch, P, workloads, with_oracle=not args.no_cpu)
        torch.cuda.empty_cache()

    if not args.no_tables:
        res["tables"] = bench_tables(torch, P, workloads, with_oracle=not args.no_cpu)
        torch.cuda.empty_cache()

    if not args.no_serving:
        res["serving"] = bench_serving(torch, P, workloads, duration=args.serve_seconds)
        torch.cuda.empty_cache()

    if not args.no_paper:
        res["paper_generator_geometry"] = bench_paper(torch, P, workloads, out)

    if args.copy_probe:
        a = torch.empty(COPY_PROBE_BYTES // 8, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        res["copy_probe_bytes"] = a.numel() * 8

    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(seed)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
