"""Benchmark: one step = one plain deterministic sample sort (every step of Algorithm 1) of
2^28 uint32 keys, uniform over [0, 2^32) from the seeded SplitMix64 stream (seed 8), keys only,
on one MI355X.  Inputs are resident in HBM before timing starts: one copy per step, so every
timed sort sees the same unsorted input and nothing but sorting happens in the timed region.

Prints one JSON line with the throughput (Mkeys/s), the per-stage kernel times measured with
HIP events on the sort's stream over the timed region, the HBM roofline of the dominant kernel,
and the CPU oracle timed on a bounded sample of the same stream.

A second leg ("batched") times the batched workload -- 4096 independent float32 sorts, sizes
log-uniform in [2^8, 2^20], N(0,1) keys with 1% exact duplicates and signed zeros -- as one
segmented call per step, beside the same segments sorted back to back, one plain sort call
each, on the same stream.

A third leg ("served") runs the served-stream workload: requests of sizes log-uniform in
[2^10, 2^26], half uint32 keys only and half uint64 keys with uint32 values, keys uniform or
bucket-clustered, through the library's server (device arena as the memory budget, continuous
batching of small requests into segmented launches).  It reports throughput when all requests
are waiting (saturated) and p50/p99 request latency under Poisson arrivals at a stated fraction
of the back-to-back capacity, beside the same requests sorted back to back with plain calls.
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
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue peak: one wave64 VALU instruction per CU per clock (four SIMDs of 16 lanes, each
# taking four clocks per wave instruction), 256 CUs at 2.4 GHz.
VALU_PEAK_G = 256 * 2.4
METRIC = "Mkeys/s + HBM GB/s (2^28 u32); p50/p99 latency, batched/served vs plain sort"
# device sources whose hash keys the recorded counter files (profiles/*.json)
KERNEL_SRCS = [os.path.join(ROOT, "paper_1002_4464_amd", "csrc", f)
               for f in ("kernels.hip", "steps.h", "sort_primitives.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
TRAFFIC_C3B_FILE = os.path.join(ROOT, "profiles", "traffic_c3b.json")
VALU_FILE = os.path.join(ROOT, "profiles", "valu.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Pipeline stages as timed by the library (kernel launches grouped by the step they implement).
STAGE_GROUPS = {
    "steps1-3 local sort + sampling": ["s123_local_sort"],
    "step4 sample sort": ["s4_sample_sort", "s4_sample_merge"],
    "steps5-6 rank": ["s56_rank"],
    "step7 scan": ["s7_scan_colsum", "s7_scan_mid", "s7_scan_update", "s7_scan"],
    "step8 + level2 steps1-3": ["s8_l2_s123_gather_sort"],
    "level2 step4": ["l2_s4_sample_sort", "l2_s4_sample_merge"],
    "level2 steps5-6": ["l2_s56_rank"],
    "level2 step7": ["l2_s7_scan"],
    "steps8-9 gather + bucket sort": ["s89_gather_sort", "s89_gather_merge", "s9_bucket_sort"],
}


def group_bytes(group: str, n: int, g, kb: int) -> float:
    """Algorithmic HBM bytes one step of a stage group must move:
    a sort or move of the data reads and writes n keys once; ranking reads the sorted sublists
    once plus the splitters and writes the counts; the scan reads the m x s counts twice (column
    sums, then the update) and writes the offsets, piece destinations and piece sources.
    Where a level's chunks hold w = L/s of 64 to 1024 items (a multiple of 16, chunk-end
    samples), its tile sort also writes the rank index (every 16th key, n/16 keys) and each
    (sublist, splitter) rank reads w/16 index entries and one block of 16 keys instead of the
    chunk."""
    sb = g.sample_bytes
    m1s1 = g.sublists * g.samples
    m2s2 = -(-n // max(g.sublist_len2, 1)) * g.samples2 if g.levels == 2 else 0

    def index_w(L, s):
        w = L // s if s else 0
        return w if (w % 16 == 0 and 64 <= w <= 1024) else 0

    # randomized plans bisect their level-1 ranks; their level 2 has chunk-end samples
    w1 = 0 if g.sampling else index_w(g.sublist_len, g.samples)
    w2 = index_w(g.sublist_len2, g.samples2) if g.levels == 2 else 0
    rank1 = m1s1 * (w1 // 16 + 16) * kb if w1 else n * kb
    rank2 = m2s2 * (w2 // 16 + 16) * kb if w2 else n * kb
    return {
        "steps1-3 local sort + sampling": 2 * n * kb + m1s1 * sb + (n * kb // 16 if w1 else 0),
        "step4 sample sort": 2 * m1s1 * sb,
        "steps5-6 rank": rank1 + m1s1 * (sb + 4),
        "step7 scan": 5 * m1s1 * 4,
        "step8 + level2 steps1-3": (2 * n * kb + 2 * m1s1 * 4 + m2s2 * sb
                                    + (n * kb // 16 if w2 else 0)),
        "level2 step4": 2 * m2s2 * sb,
        "level2 steps5-6": rank2 + m2s2 * (sb + 4),
        "level2 step7": 5 * m2s2 * 4,
        "steps8-9 gather + bucket sort": 2 * n * kb,
    }.get(group, 0.0)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_for(stage: str, path: str = TRAFFIC_FILE):
    """Measured HBM bytes per step of a stage group (rocprofv3 FETCH_SIZE + WRITE_SIZE, each
    scaled by a copy kernel of known size), if recorded for the current kernel source."""
    try:
        with open(path) as f:
            t = json.load(f)
    except OSError:
        return None
    if t.get("kernel_source_sha256_16") != kernel_hash():
        return None
    v = t.get("bytes_per_step", {}).get(stage)
    return float(v) if v is not None else None


def valu_for(stage: str):
    """VALU wave instructions per step of a stage group (rocprofv3 SQ_INSTS_VALU), if
    recorded for the current kernel source."""
    try:
        with open(VALU_FILE) as f:
            t = json.load(f)
    except OSError:
        return None
    if t.get("kernel_source_sha256_16") != kernel_hash():
        return None
    v = t.get("valu_wave_instr_per_step", {}).get(stage)
    return float(v) if v is not None else None


def cpu_model() -> str:
    """The host CPU as /proc/cpuinfo names it (model name, family / model / stepping, clock)."""
    fields = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if not line.strip():
                    break  # the first processor's block is enough
                k, _, v = line.partition(":")
                fields[k.strip()] = v.strip()
    except OSError:
        return "unknown"
    name = fields.get("model name", "unknown")
    extra = ", ".join(f"{k} {fields[k]}" for k in ("cpu family", "model", "stepping", "cpu MHz")
                      if k in fields)
    return f"{name} ({extra})" if extra else name


def cpu_baseline(seed: int, sample_log2: int, L: int, s: int, full_log2: int):
    """The single-threaded C oracle of Algorithm 1, pinned to one host core, on the first
    2^sample_log2 keys of the benchmark's stream."""
    import oracle
    n = 1 << sample_log2
    keys = __import__("synth").uniform_u32(n, seed)
    oracle.build(force=False)
    old = os.sched_getaffinity(0)
    core = min(old)
    os.sched_setaffinity(0, {core})
    try:
        t0 = time.perf_counter()
        out, _, _ = oracle.dss(keys, L, s)
        dt = time.perf_counter() - t0
    finally:
        os.sched_setaffinity(0, old)
    assert (out[1:] >= out[:-1]).all()
    return {"value": round(n / dt / 1e6, 3), "unit": "Mkeys/s", "cores": 1, "kind": "oracle",
            "cpu": cpu_model(), "host_cpus": len(old),
            "sample": (f"the benchmark's own input (2^{sample_log2} keys, seed {seed}), one run"
                       if sample_log2 == full_log2 else
                       f"first 2^{sample_log2} keys of the same uniform stream (seed {seed})") +
                      f"; single-threaded C oracle of Algorithm 1 with L={L}, s={s}, pinned to "
                      f"core {core}; {dt:.1f} s"}


def path_roofline(n: int, kb: int, ms: float) -> dict:
    """Whole-sort HBM fractions: measured bytes of all passes (rocprofv3 counters recorded for
    this kernel source) over the sort time, and the one-level algorithmic floor of 7 n b bytes
    (Steps 2, 8 and 9 read and write the data, Step 6 reads it once)."""
    rec = {"floor_7nb_gbs": round(7 * n * kb / (ms * 1e-3) / 1e9, 1)}
    rec["floor_frac"] = round(rec["floor_7nb_gbs"] / HBM_PEAK_GBS, 4)
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        if t.get("kernel_source_sha256_16") == kernel_hash():
            tot = sum(t["bytes_per_step"].values())
            rec["measured_bytes"] = round(tot)
            rec["measured_gbs"] = round(tot / (ms * 1e-3) / 1e9, 1)
            rec["measured_frac"] = round(rec["measured_gbs"] / HBM_PEAK_GBS, 4)
    except (OSError, KeyError, ValueError):
        pass
    return rec


def time_sorts(plan, torch, dev, k, v, reps, warm=1, timing_reps=0):
    """Median / min / max ms of `reps` sorts, each on its own resident copy of (k, v), with HIP
    events recorded on the sort's stream between them (after `warm` untimed sorts); then, if
    asked, the library's per-kernel events over `timing_reps` more sorts."""
    ws = plan.workspace(dev)
    st = torch.cuda.current_stream(dev)
    tot = warm + reps + timing_reps
    bufs = [k.clone() for _ in range(tot)]
    vb = [v.clone() for _ in range(tot)] if v is not None else None

    def one(i):
        if vb is None:
            plan.sort_keys(bufs[i], ws, st)
        else:
            plan.sort_pairs(bufs[i], vb[i], ws, st)

    for i in range(warm):
        one(i)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record(st)
    for j in range(reps):
        one(warm + j)
        ev[j + 1].record(st)
    torch.cuda.synchronize()
    ms = sorted(ev[j].elapsed_time(ev[j + 1]) for j in range(reps))
    stages = {}
    if timing_reps:
        plan.set_timing(True)
        for i in range(warm + reps, tot):
            one(i)
        torch.cuda.synchronize()
        stages = plan.stage_times()
        plan.set_timing(False)
    status = ws[:256].cpu().numpy().view(np.uint32)
    assert int(status[0]) == 0, f"kernel status flags {int(status[0]):#x}"
    last = bufs[-1]
    del bufs, vb
    return {"median": ms[len(ms) // 2], "min": ms[0], "max": ms[-1], "stages": stages,
            "routed": int(status[40]), "last": last}


C2_SEEDS = {"uniform": 2, "gaussian": 3, "bucket": 4, "staggered": 5, "sorted": 6, "equal": 7}


def distributions_leg(args, ds, torch, dev):
    """The six 2^26 uint32 distributions, each sorted by Algorithm 1 (deterministic samples)
    and by the randomized-splitter comparison method (random sample positions, last bucket
    closed by +infinity) with the same plan: time per distribution and the spread across them
    (Section 5's distribution-independence claim, measured on both methods)."""
    import synth
    n = 1 << args.dist_log2
    det = ds.Plan(ds.U32, False, n)
    tu = ds.Tuning(0, 0, 0, 0, 0)
    tu.sampling = 1
    tu.seed = args.random_seed
    rnd = ds.Plan(ds.U32, False, n, tu)
    g = det.geometry(n)
    out = {"workload": f"2^{args.dist_log2} uint32 keys, keys only, six distributions (seeds "
                       f"{C2_SEEDS})", "n": n,
           "plan": {"levels": g.levels, "L": g.sublist_len, "s": g.samples,
                    "L2": g.sublist_len2, "s2": g.samples2},
           "random_seed": args.random_seed, "reps": args.dist_reps,
           "deterministic": {}, "randomized": {}}
    for dist, seed in C2_SEEDS.items():
        log(f"[bench] distributions: {dist}")
        src = torch.from_numpy(synth.make_u32(dist, n, seed).view(np.int32)).to(dev)
        for mode, plan in (("deterministic", det), ("randomized", rnd)):
            r = time_sorts(plan, torch, dev, src, None, args.dist_reps)
            last = r["last"][: 1 << 20].cpu().numpy().view(np.uint32)
            assert (last[1:] >= last[:-1]).all(), f"{mode} {dist}: prefix not sorted"
            rec = {"ms": round(r["median"], 4), "min_ms": round(r["min"], 4),
                   "max_ms": round(r["max"], 4), "mkeys_s": round(n / r["median"] / 1e3, 1)}
            if mode == "randomized":
                rec["routed_buckets"] = r["routed"]
            out[mode][dist] = rec
        del src
        torch.cuda.empty_cache()
    for mode in ("deterministic", "randomized"):
        ms = [v["ms"] for v in out[mode].values()]
        out[mode + "_spread"] = {"min_ms": min(ms), "max_ms": max(ms),
                                 "rel": round((max(ms) - min(ms)) / min(ms), 4)}
    return out


def c3b_leg(args, ds, torch, dev):
    """2^27 (uint64 key, uint32 value = input index) pairs, keys uniform or Zipf(1.1) over 2^20
    values: time per sort, per-stage kernel times, and the dominant stage against the HBM
    roofline (12 bytes per item; measured traffic from profiles/traffic_c3b.json)."""
    import synth
    n = 1 << 27
    kb = 12
    plan = ds.Plan(ds.U64, True, n)
    g = plan.geometry(n)
    vals = torch.arange(n, dtype=torch.int32, device=dev)
    out = {"workload": "2^27 uint64 keys with uint32 values (input index), uniform (seed 9) "
                       "or Zipf(1.1) over 2^20 values (seed 10), stable", "n": n,
           "plan": {"levels": g.levels, "L": g.sublist_len, "s": g.samples,
                    "L2": g.sublist_len2, "s2": g.samples2}}
    for dist in ("uniform",) if args.c3b_uniform_only else ("uniform", "zipf"):
        log(f"[bench] c3b: generating {dist}")
        keys = synth.uniform_u64(n, 9) if dist == "uniform" else synth.zipf_u64(n, 10)
        src = torch.from_numpy(keys.view(np.int64)).to(dev)
        del keys
        log(f"[bench] c3b: timing {dist}")
        r = time_sorts(plan, torch, dev, src, vals, args.c3b_reps,
                       timing_reps=args.c3b_reps if dist == "uniform" else 0)
        last = r["last"][: 1 << 20].cpu().numpy().view(np.uint64)
        assert (last[1:] >= last[:-1]).all(), f"c3b {dist}: prefix not sorted"
        out[dist] = {"ms": round(r["median"], 4), "min_ms": round(r["min"], 4),
                     "max_ms": round(r["max"], 4), "mkeys_s": round(n / r["median"] / 1e3, 1),
                     "floor_7nb_frac": round(7 * n * kb / (r["median"] * 1e-3) / 1e9
                                             / HBM_PEAK_GBS, 4)}
        if r["stages"]:
            reps = args.c3b_reps
            groups = {}
            for grp, names in STAGE_GROUPS.items():
                t = sum(r["stages"][nm][0] * r["stages"][nm][1] for nm in names
                        if nm in r["stages"]) / reps
                if t > 0:
                    groups[grp] = round(t, 4)
            out["stage_ms"] = groups
            dom = max(groups, key=groups.get)
            alg = group_bytes(dom, n, g, kb)
            ach = alg / (groups[dom] * 1e-3) / 1e9
            out["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1),
                               "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": round(ach / HBM_PEAK_GBS, 4),
                               "traffic": traffic_for(dom, TRAFFIC_C3B_FILE),
                               "algorithmic_bytes": alg, "ms_per_step": groups[dom]}
        del src
        torch.cuda.empty_cache()
    if "zipf" in out:
        out["zipf_vs_uniform"] = round(out["zipf"]["ms"] / out["uniform"]["ms"], 4)
    return out


def sweep(args, ds, torch, dev):
    """Mkeys/s against n for each layout (the paper's constant-rate experiment), and time
    against the samples per sublist s at fixed n (its s experiment), at this GPU's sizes."""
    import synth
    out = {"n_sweep": [], "s_sweep": []}

    def timed(plan, k, v, reps=5):
        ws = plan.workspace(dev)
        bufs = [k.clone() for _ in range(reps + 1)]
        vb = [v.clone() for _ in range(reps + 1)] if v is not None else None
        st = torch.cuda.current_stream(dev)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        for i in range(reps + 1):
            if i == 1:
                ev[0].record(st)
            if vb is None:
                plan.sort_keys(bufs[i], ws, st)
            else:
                plan.sort_pairs(bufs[i], vb[i], ws, st)
            if i >= 1:
                ev[i].record(st)
        torch.cuda.synchronize()
        ms = sorted(ev[i - 1].elapsed_time(ev[i]) for i in range(1, reps + 1))
        return ms[len(ms) // 2]

    layouts = [("u32", ds.U32, False, 28), ("u32 pairs", ds.U32, True, 27),
               ("u64", ds.U64, False, 27), ("u64 pairs", ds.U64, True, 27)]
    for name, kt, vals, top in layouts:
        for lg in range(16, top + 1, 2 if top % 2 == 0 else 1):
            n = 1 << lg
            if kt == ds.U64:
                k = torch.from_numpy(synth.uniform_u64(n, 9).view(np.int64)).to(dev)
            else:
                k = torch.from_numpy(synth.uniform_u32(n, 2).view(np.int32)).to(dev)
            v = torch.arange(n, dtype=torch.int32, device=dev) if vals else None
            plan = ds.Plan(kt, vals, n)
            ms = timed(plan, k, v)
            g = plan.geometry(n)
            out["n_sweep"].append({"layout": name, "n": n, "ms": round(ms, 4),
                                   "mkeys_s": round(n / ms / 1e3, 1), "levels": g.levels})
            log(f"[bench] sweep {name} 2^{lg}: {ms:.3f} ms")
            del k, v, plan
            torch.cuda.empty_cache()
    for lg in (25, 26, 27):
        n = 1 << lg
        k = torch.from_numpy(synth.uniform_u32(n, 2).view(np.int32)).to(dev)
        for s in (16, 32, 64, 128, 256, 512, 1024):
            try:
                plan = ds.Plan(ds.U32, False, n, ds.Tuning(16384, s, 0, 0, 2))
            except ds.DsortError:
                continue
            ms = timed(plan, k, None)
            g = plan.geometry(n)
            out["s_sweep"].append({"n": n, "s": s, "s2": g.samples2, "ms": round(ms, 4),
                                   "mkeys_s": round(n / ms / 1e3, 1)})
            log(f"[bench] s sweep 2^{lg} s={s}: {ms:.3f} ms")
            del plan
            torch.cuda.empty_cache()
        del k
    return out


def batched_leg(args, ds, torch, dev):
    """One step = one segmented call over the whole batch; the reference point is the same
    batch sorted by back-to-back plain calls (one per segment) on the same stream."""
    import synth
    S = args.batched_segments
    sizes = synth.segment_sizes(S, args.batched_seed, 8, 20)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n = int(offs[-1])
    log(f"[bench] batched: generating {S} float32 segments, {n} keys (seed {args.batched_seed})")
    x = synth.normal_f32_segments(sizes, args.batched_seed)
    src = torch.from_numpy(x.view(np.int32)).to(dev)
    del x
    t_off = torch.from_numpy(offs).to(dev)
    K, W = args.batched_steps, 2
    bufs = [src.clone() for _ in range(W + K)]
    max_seg = int(sizes.max())
    plan = ds.Plan(ds.F32, False, n, max_segments=S)
    geo = plan.segmented_geometry(n, S, max_seg)
    ws = plan.workspace(dev)
    stream = torch.cuda.current_stream(dev)
    torch.cuda.synchronize()
    for i in range(W):
        plan.sort_segmented(bufs[i], t_off, max_segment=max_seg, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    log(f"[bench] batched: timing {K} segmented calls")
    t0 = time.perf_counter()
    for i in range(W, W + K):
        plan.sort_segmented(bufs[i], t_off, max_segment=max_seg, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    dt_default = (time.perf_counter() - t0) / K
    # autotune (L, s) per length class on the pristine batch, then time again
    log("[bench] batched: autotuning")
    t0 = time.perf_counter()
    tuning = plan.autotune_segmented(src, t_off, max_segment=max_seg, repeats=2, workspace=ws,
                                     stream=stream)
    torch.cuda.synchronize()
    t_tune = time.perf_counter() - t0
    geo = plan.segmented_geometry(n, S, max_seg)
    for b in bufs:
        b.copy_(src)
    for i in range(W):
        plan.sort_segmented(bufs[i], t_off, max_segment=max_seg, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    log(f"[bench] batched: timing {K} tuned segmented calls")
    t0 = time.perf_counter()
    for i in range(W, W + K):
        plan.sort_segmented(bufs[i], t_off, max_segment=max_seg, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / K
    # the same call captured once into a HIP graph (with the copy that refills its buffer) and
    # replayed, against the same copy + call issued eagerly; a captured call keeps every size
    # class on the capturing stream, the eager call spreads them over side streams
    gbuf = bufs[0]
    cap_stream = torch.cuda.Stream(dev)
    graph = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=cap_stream):
        gbuf.copy_(src)
        plan.sort_segmented(gbuf, t_off, max_segment=max_seg, workspace=ws,
                            stream=torch.cuda.current_stream(dev))
    torch.cuda.synchronize()

    def timed_loop(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(K):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / K

    dt_graph = timed_loop(graph.replay)
    graph_out = gbuf.clone()

    def eager():
        gbuf.copy_(src)
        plan.sort_segmented(gbuf, t_off, max_segment=max_seg, workspace=ws, stream=stream)

    dt_eager = timed_loop(eager)
    assert torch.equal(gbuf, graph_out), "graph replay differs from the eager call"
    del graph, graph_out
    # per-kernel times on K more calls with the library's HIP events switched on
    for b in bufs[W:]:
        b.copy_(src)
    torch.cuda.synchronize()
    plan.set_timing(True)
    for i in range(W, W + K):
        plan.sort_segmented(bufs[i], t_off, max_segment=max_seg, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    stages = plan.stage_times()
    plan.set_timing(False)
    status = int(ws[:4].cpu().numpy().view(np.uint32)[0])
    assert status == 0, f"kernel status flags {status:#x}"
    for g in (int(np.argmax(sizes)), int(np.argmin(sizes)), S // 2):
        seg = bufs[-1][int(offs[g]):int(offs[g + 1])].cpu().numpy().view(np.uint32).astype(
            np.int64)
        img = np.where(seg >= 1 << 31, 0xFFFFFFFF - seg, seg + (1 << 31))
        assert (img[1:] >= img[:-1]).all(), f"segment {g} not sorted"
    del bufs

    # back to back: one plain call per segment, same stream, same device-resident input
    pplan = ds.Plan(ds.F32, False, max_seg)
    pws = pplan.workspace(dev)
    Kp = args.batched_plain_steps
    pbufs = [src.clone() for _ in range(1 + Kp)]
    bounds = [(int(offs[g]), int(offs[g + 1])) for g in range(S)]

    def plain_step(buf):
        for lo, hi in bounds:
            pplan.sort_keys(buf[lo:hi], pws, stream)

    plain_step(pbufs[0])
    torch.cuda.synchronize()
    log(f"[bench] batched: timing {Kp} back-to-back passes of {S} plain calls")
    t0 = time.perf_counter()
    for i in range(1, 1 + Kp):
        plain_step(pbufs[i])
    torch.cuda.synchronize()
    dtp = (time.perf_counter() - t0) / Kp
    assert torch.equal(pbufs[-1], pbufs[0])
    del pbufs, src
    return {
        "workload": f"{S} independent float32 sorts, sizes log-uniform in [2^8, 2^20] (seed "
                    f"{args.batched_seed}), N(0,1) keys with 1% duplicates and signed zeros, "
                    f"IEEE totalOrder, keys only",
        "n": n, "segments": S, "max_segment": max_seg,
        "small_capacity": geo.small_capacity,
        "tuning": {"class_upper": geo.class_upper, "L": geo.sublist_len, "s": geo.samples},
        "autotune_s": round(t_tune, 2),
        "value": round(n / dt / 1e6, 1), "unit": "Mkeys/s", "steps": K,
        "ms_per_step": round(dt * 1e3, 4),
        "untuned_ms_per_step": round(dt_default * 1e3, 4),
        "graph": {"what": "copy into the buffer + one segmented call, captured once",
                  "replay_ms": round(dt_graph * 1e3, 4), "eager_ms": round(dt_eager * 1e3, 4)},
        "back_to_back_mkeys_s": round(n / dtp / 1e6, 1),
        "back_to_back_ms": round(dtp * 1e3, 3),
        "speedup_vs_back_to_back": round(dtp / dt, 2),
        "kernel_ms": {k: round(v[0] * v[1] / K, 4) for k, v in stages.items()},
    }


def _request_keys(torch, dev, i, n, seed, out_k, out_v):
    """Request i of the served trace, generated on the device from its own seeded generator
    (so every run starts from identical inputs without keeping pristine copies): even requests
    uint32 keys only, odd ones uint64 keys with uint32 values (the input index); keys uniform or
    clustered in 64 consecutive groups (group g in subrange g), alternating in pairs."""
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed * 7919 + i)
    bucket = (i >> 1) % 2 == 1
    lo = torch.randint(0, 1 << 32, (n,), dtype=torch.int64, device=dev, generator=gen)
    if i % 2 == 0:
        if bucket:
            grp = torch.arange(n, dtype=torch.int64, device=dev) * 64 // n
            lo = (grp << 26) | (lo >> 6)
        out_k.copy_(lo.to(torch.int32))  # low 32 bits
    else:
        hi = torch.randint(0, 1 << 32, (n,), dtype=torch.int64, device=dev, generator=gen)
        k = (hi << 32) | lo  # wraps into the int64 view of a uint64
        if bucket:
            grp = torch.arange(n, dtype=torch.int64, device=dev) * 64 // n
            k = (grp << 58) | ((k >> 6) & ((1 << 58) - 1))
        out_k.copy_(k)
        torch.arange(n, dtype=torch.int32, device=dev, out=out_v)


def _fingerprint(torch, t):
    """Order-sensitive digest of a device tensor (wrapping int64 arithmetic)."""
    x = t.to(torch.int64)
    w = torch.arange(1, x.numel() + 1, dtype=torch.int64, device=t.device) * 0x9E3779B1
    return int((x * w).sum()), int((x ^ (w >> 7)).sum())


def served_leg(args, ds, torch, dev):
    import synth
    R = args.served_requests
    sizes = synth.segment_sizes(R, args.served_seed, 10, 26)
    bytes_per = [int(n) * (4 if i % 2 == 0 else 12) for i, n in enumerate(sizes.tolist())]
    free, _ = torch.cuda.mem_get_info(dev)
    budget = args.served_budget_gb << 30
    room = free - budget - (8 << 30)  # arena, plan workspaces and digests
    note = None
    if sum(bytes_per) > room:  # keep the trace's prefix that fits beside the arena
        keep = int(np.searchsorted(np.cumsum(bytes_per), room))
        note = (f"{R} requests need {sum(bytes_per) / 2**30:.0f} GiB of resident buffers; "
                f"{keep} fit beside the {args.served_budget_gb} GiB arena")
        R = keep
        sizes = sizes[:R]
    log(f"[bench] served: {R} requests, {int(sizes.sum())} items (seed {args.served_seed})")
    work, layouts = [], []
    for i, n in enumerate(sizes.tolist()):
        if i % 2 == 0:
            work.append((torch.empty(n, dtype=torch.int32, device=dev), None))
            layouts.append(ds.U32)
        else:
            work.append((torch.empty(n, dtype=torch.int64, device=dev),
                         torch.empty(n, dtype=torch.int32, device=dev)))
            layouts.append(ds.U64)
    total = int(sizes.sum())

    def reset():
        for i, (wk, wv) in enumerate(work):
            _request_keys(torch, dev, i, wk.numel(), args.served_seed, wk, wv)
        torch.cuda.synchronize()

    # back to back: one plain call per request, in arrival order, one stream
    stream = torch.cuda.current_stream(dev)
    plans = {ds.U32: ds.Plan(ds.U32, False, int(sizes.max())),
             ds.U64: ds.Plan(ds.U64, True, int(sizes.max()))}
    wss = {kt: p.workspace(dev) for kt, p in plans.items()}

    def b2b():
        for (wk, wv), kt in zip(work, layouts):
            if wv is None:
                plans[kt].sort_keys(wk, wss[kt], stream)
            else:
                plans[kt].sort_pairs(wk, wv, wss[kt], stream)

    reset()
    b2b()
    torch.cuda.synchronize()
    reset()
    t0 = time.perf_counter()
    b2b()
    torch.cuda.synchronize()
    t_b2b = time.perf_counter() - t0
    ref = [(_fingerprint(torch, wk), None if wv is None else _fingerprint(torch, wv))
           for wk, wv in work]
    del wss, plans
    torch.cuda.empty_cache()

    srv = ds.Server(budget, max_inflight=args.served_inflight, lanes=args.served_lanes)

    def check():
        for (wk, wv), (rk, rv) in zip(work, ref):
            assert _fingerprint(torch, wk) == rk, "served != plain"
            assert wv is None or _fingerprint(torch, wv) == rv, "served != plain"

    def run(gaps):
        reset()
        tickets = []
        t_start = time.perf_counter()
        t_next = t_start
        for (wk, wv), kt, gap in zip(work, layouts, gaps):
            t_next += gap
            while time.perf_counter() < t_next:
                pass
            tickets.append(srv.submit(wk, wv, key_type=kt, sync=False))
        res = [srv.wait(t, timeout_s=600) for t in tickets]
        span = (max(r.t_done_ns for r in res) - min(r.t_submit_ns for r in res)) * 1e-9
        lat = np.array([r.latency_s for r in res])
        for t in tickets:
            srv.release(t)
        return span, lat

    run(np.zeros(R))  # warm-up
    log("[bench] served: saturated run")
    span_sat, lat_sat = run(np.zeros(R))
    check()
    u = (synth.draws64(args.served_seed + 1, R) >> np.uint64(11)).astype(np.float64) / 2.0**53
    poisson = []
    for load in args.served_loads:
        rate = load * R / t_b2b  # requests per second
        gaps = -np.log(1.0 - u) / rate
        log(f"[bench] served: Poisson run at {load:.2f} x back-to-back capacity")
        span_p, lat_p = run(gaps)
        check()
        poisson.append({"offered_load": load, "mkeys_s": round(total / span_p / 1e6, 1),
                        "vs_back_to_back": round(t_b2b / span_p, 3),
                        "p50_ms": round(float(np.percentile(lat_p, 50)) * 1e3, 3),
                        "p99_ms": round(float(np.percentile(lat_p, 99)) * 1e3, 3)})
    st = srv.stats()
    srv.close()
    del work
    torch.cuda.empty_cache()
    bound = args.served_p99_bound_ms
    held = [p for p in poisson if p["p99_ms"] <= bound]
    best = max(held, key=lambda p: p["offered_load"]) if held else None
    head = poisson[0]
    return {
        "workload": f"{R} requests, sizes log-uniform in [2^10, 2^26] (seed {args.served_seed}), "
                    f"alternating uint32 keys-only and uint64-key/uint32-value pairs, uniform or "
                    f"bucket-clustered keys generated on the device; device arena "
                    f"{args.served_budget_gb} GiB, {args.served_lanes} lanes",
        "requests": R, "requests_note": note,
        "items": total,
        "back_to_back_mkeys_s": round(total / t_b2b / 1e6, 1),
        "back_to_back_ms": round(t_b2b * 1e3, 3),
        "saturated_mkeys_s": round(total / span_sat / 1e6, 1),
        "saturated_speedup_vs_back_to_back": round(t_b2b / span_sat, 3),
        "saturated_p50_ms": round(float(np.percentile(lat_sat, 50)) * 1e3, 3),
        "saturated_p99_ms": round(float(np.percentile(lat_sat, 99)) * 1e3, 3),
        "offered_load": head["offered_load"],
        "poisson_mkeys_s": head["mkeys_s"],
        "poisson_p50_ms": head["p50_ms"],
        "poisson_p99_ms": head["p99_ms"],
        "p99_bound_ms": bound,
        "max_load_at_p99": best["offered_load"] if best else None,
        "max_load_mkeys_s": best["mkeys_s"] if best else None,
        "max_load_vs_back_to_back": best["vs_back_to_back"] if best else None,
        "poisson_runs": poisson,
        "units": st["units"], "batched_units": st["batched_units"],
        "batched_requests": st["batched_requests"], "max_batch": st["max_batch"],
        "peak_arena_gib": round(st["peak_arena_bytes"] / 2**30, 3),
    }


def _group_of(kernel: str, seen: dict) -> str:
    """Maps a rocprofv3 kernel name of one sort to its stage group; the Step 1-3 tile kernels
    run once per level, so their first launch in a sort is level 1 and the second level 2."""
    name = kernel.replace("dsort::(anonymous namespace)::", "")
    if name.startswith("k_tile_radix") or name.startswith("void k_tile_radix") or \
            (name.startswith("void k_tile<") and ", 0," in name):
        seen["tile"] = seen.get("tile", 0) + 1
        return "steps1-3 local sort + sampling" if seen["tile"] % 2 == 1 else \
            "step8 + level2 steps1-3"
    for key, grp in (("k_gather", "steps8-9 gather + bucket sort"),
                     ("k_tile<", "steps8-9 gather + bucket sort"),
                     ("k_rank", "steps5-6 rank"),
                     ("k_sort_samples", "step4 sample sort"),
                     ("k_merge_round", "step4 sample sort"),
                     ("k_scan", "step7 scan"),
                     ("k_init", "init")):
        if key in name:
            return grp
    return "other"


def ingest_pmc(fetch_csv: str, write_csv: str, copy_bytes: int, sorts: int, out_json: str):
    """Turns two rocprofv3 --pmc runs of `bench.py --copy-calibration` (FETCH_SIZE, then
    WRITE_SIZE; KiB per dispatch) into measured HBM bytes per sort for each stage group, each
    counter scaled by what it reads for the calibration copy of `copy_bytes` bytes."""
    import csv
    import collections

    def load(path, counter):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        return rows

    res = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = load(path, counter)
        last_sort = max((int(r["Dispatch_Id"]) for r in rows if "dsort" in r["Kernel_Name"]),
                        default=0)
        copies = [float(r["Counter_Value"]) * 1024 for r in rows
                  if int(r["Dispatch_Id"]) > last_sort and
                  ("copyBuffer" in r["Kernel_Name"] or "elementwise" in r["Kernel_Name"])]
        # the calibration copy is the largest copy kernel after the sorts (the others are the
        # small device-to-host reads of the result checks)
        big = max(copies, default=0.0)
        scale = copy_bytes / big if big > 0 else 1.0
        per = collections.defaultdict(float)
        seen = {}
        started = False
        for r in rows:
            name = r["Kernel_Name"]
            if "dsort" not in name:
                continue
            grp = _group_of(name, seen)
            if grp == "init":
                started = True
                continue
            if started:
                per[grp] += float(r["Counter_Value"]) * 1024 * scale
        res[counter] = ({k: v / sorts for k, v in per.items()}, scale)
    groups = set(res["FETCH_SIZE"][0]) | set(res["WRITE_SIZE"][0])
    traffic = {g: res["FETCH_SIZE"][0].get(g, 0.0) + res["WRITE_SIZE"][0].get(g, 0.0)
               for g in groups}
    rec = {"kernel_source_sha256_16": kernel_hash(),
           "copy_bytes": copy_bytes, "fetch_scale": res["FETCH_SIZE"][1],
           "write_scale": res["WRITE_SIZE"][1], "sorts": sorts,
           "bytes_per_step": traffic,
           "fetch_bytes": res["FETCH_SIZE"][0], "write_bytes": res["WRITE_SIZE"][0]}
    with open(out_json, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
    print(json.dumps(rec, indent=1, sort_keys=True))


def ingest_valu(csv_path: str, sorts: int, out_json: str):
    """Turns a rocprofv3 --pmc run that holds SQ_INSTS_VALU into VALU wave instructions per sort
    for each stage group (profiles/valu.json), for the issue-bound view of the roofline."""
    import csv
    import collections
    rows = [r for r in csv.DictReader(open(csv_path)) if r["Counter_Name"] == "SQ_INSTS_VALU"]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    per = collections.defaultdict(float)
    seen = {}
    started = False
    for r in rows:
        name = r["Kernel_Name"]
        if "dsort" not in name:
            continue
        grp = _group_of(name, seen)
        if grp == "init":
            started = True
            continue
        if started:
            per[grp] += float(r["Counter_Value"])
    rec = {"kernel_source_sha256_16": kernel_hash(), "sorts": sorts,
           "valu_wave_instr_per_step": {k: v / sorts for k, v in per.items()}}
    with open(out_json, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
    print(json.dumps(rec, indent=1, sort_keys=True))


def calibration_copy(args, torch, dev):
    """With --copy-calibration BYTES: one device copy of that many bytes after the sorts, the
    kernel of known size by which ingest_pmc scales the counters."""
    if args.copy_calibration:
        cs = torch.empty(args.copy_calibration // 4, dtype=torch.int32, device=dev)
        cd = torch.empty_like(cs)
        cd.copy_(cs)
        torch.cuda.synchronize()
        del cs, cd


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--seed", type=int, default=8)
    ap.add_argument("--cpu-sample-log2", type=int, default=28,
                    help="the oracle runs on the first 2^k keys of the benchmark's input "
                         "(default: all of it, one run)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stage-timing", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="after timing, copy BYTES bytes with torch (a kernel of known size for "
                         "scaling rocprofv3 FETCH_SIZE/WRITE_SIZE)")
    ap.add_argument("--ingest-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn two rocprofv3 counter CSVs of a --copy-calibration run into "
                         "profiles/traffic.json (CPU only)")
    ap.add_argument("--traffic-file", default=TRAFFIC_FILE,
                    help="where --ingest-pmc writes (profiles/traffic_c3b.json for a run of "
                         "--only c3b --c3b-uniform-only)")
    ap.add_argument("--ingest-valu", metavar="PMC_CSV",
                    help="turn a rocprofv3 counter CSV holding SQ_INSTS_VALU into "
                         "profiles/valu.json (CPU only)")
    ap.add_argument("--sorts", type=int, default=1, help="sorts in the ingested runs")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched leg")
    ap.add_argument("--batched-segments", type=int, default=4096)
    ap.add_argument("--batched-seed", type=int, default=4)
    ap.add_argument("--batched-steps", type=int, default=10)
    ap.add_argument("--batched-plain-steps", type=int, default=2)
    ap.add_argument("--no-served", action="store_true", help="skip the served leg")
    ap.add_argument("--no-distributions", action="store_true",
                    help="skip the six-distribution leg (deterministic and randomized)")
    ap.add_argument("--dist-log2", type=int, default=26)
    ap.add_argument("--dist-reps", type=int, default=5)
    ap.add_argument("--random-seed", type=int, default=2024,
                    help="seed of the randomized-splitter runs")
    ap.add_argument("--no-c3b", action="store_true", help="skip the 2^27 uint64-pair leg")
    ap.add_argument("--c3b-reps", type=int, default=5)
    ap.add_argument("--c3b-uniform-only", action="store_true",
                    help="the 2^27 uint64-pair leg without its Zipf input (for counter runs)")
    ap.add_argument("--only", choices=["batched", "served", "sweep", "distributions", "c3b"],
                    help="run only that leg and print its record (for profiling)")
    ap.add_argument("--served-requests", type=int, default=4000)
    ap.add_argument("--served-seed", type=int, default=12)
    ap.add_argument("--served-loads", type=float, nargs="+",
                    default=[0.7, 0.5, 0.9, 1.0, 1.1, 1.25, 1.5],
                    help="offered loads of the Poisson runs (first one is the headline)")
    ap.add_argument("--served-p99-bound-ms", type=float, default=25.0,
                    help="p99 latency bound for the highest sustained offered load")
    ap.add_argument("--served-budget-gb", type=int, default=64)
    ap.add_argument("--served-lanes", type=int, default=4)
    ap.add_argument("--served-inflight", type=int, default=1024)
    args = ap.parse_args()
    if args.ingest_pmc:
        ingest_pmc(args.ingest_pmc[0], args.ingest_pmc[1], args.copy_calibration, args.sorts,
                   args.traffic_file)
        return
    if args.ingest_valu:
        ingest_valu(args.ingest_valu, args.sorts, VALU_FILE)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the library has no multi-GPU path "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1002_4464_amd as ds
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.only:
        leg = {"batched": batched_leg, "served": served_leg, "sweep": sweep,
               "distributions": distributions_leg, "c3b": c3b_leg}[args.only]
        rec = leg(args, ds, torch, dev)
        calibration_copy(args, torch, dev)
        print(json.dumps({args.only: rec}), flush=True)
        return
    n = 1 << args.log2n
    K, W = args.steps, args.warmup

    log(f"[bench] generating 2^{args.log2n} uniform u32 keys (seed {args.seed})")
    keys = synth.uniform_u32(n, args.seed)
    src = torch.from_numpy(keys.view(np.int32)).to(dev)
    # W warm-up, K timed, and (with stage timing) K more instrumented steps, each on its own
    # resident copy of the unsorted input
    nb = W + K + (0 if args.no_stage_timing else K)
    bufs = [src.clone() for _ in range(nb)]
    del src
    plan = ds.Plan(ds.U32, False, n)
    g = plan.geometry(n)
    ws = plan.workspace(dev)
    stream = torch.cuda.current_stream(dev)
    torch.cuda.synchronize()

    log(f"[bench] plan: levels={g.levels} L={g.sublist_len} s={g.samples} m={g.sublists} "
        f"L2={g.sublist_len2} s2={g.samples2}; warmup {W}")
    for i in range(W):
        plan.sort_keys(bufs[i], ws, stream)
    torch.cuda.synchronize()
    log(f"[bench] timing {K} steps")
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    t0 = time.perf_counter()
    evs[0].record(stream)
    for j, i in enumerate(range(W, W + K)):
        plan.sort_keys(bufs[i], ws, stream)
        evs[j + 1].record(stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    step_ms = sorted(evs[j].elapsed_time(evs[j + 1]) for j in range(K))
    stages = {}
    dt_instr = None
    if not args.no_stage_timing:
        # per-kernel HIP events (the library brackets every launch) on K more sorts, kept out
        # of the headline region because the events themselves cost time
        log(f"[bench] timing {K} instrumented steps")
        plan.set_timing(True)
        t1 = time.perf_counter()
        for i in range(W + K, W + 2 * K):
            plan.sort_keys(bufs[i], ws, stream)
        torch.cuda.synchronize()
        dt_instr = time.perf_counter() - t1
        stages = plan.stage_times()
        plan.set_timing(False)
    calibration_copy(args, torch, dev)

    out = bufs[-1][: 1 << 20].cpu().numpy().view(np.uint32)
    assert (out[1:] >= out[:-1]).all(), "output prefix not sorted"
    status = int(ws[:4].cpu().numpy().view(np.uint32)[0])
    assert status == 0, f"kernel status flags {status:#x}"

    ms_per_step = dt / K * 1e3
    mkeys = n / (dt / K) / 1e6
    stage_ms = {k: round(v[0] * v[1] / K, 4) for k, v in stages.items()}
    kb = 4
    groups = {}
    for grp, names in STAGE_GROUPS.items():
        t = sum(stages[nm][0] * stages[nm][1] for nm in names if nm in stages) / K
        if t > 0:
            groups[grp] = t
    roofline = None
    whole_bytes = sum(group_bytes(gname, n, g, kb) for gname in groups)
    if groups:
        dom = max(groups, key=groups.get)
        t_ms = groups[dom]
        alg = group_bytes(dom, n, g, kb)
        achieved = alg / (t_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_for(dom),
                    "algorithmic_bytes": alg, "ms_per_step": round(t_ms, 4),
                    "launches_per_step": sum(stages[nm][1] for nm in STAGE_GROUPS[dom]
                                             if nm in stages) // K,
                    "alu": None}
        # The same kernels against their instruction-issue bound: VALU wave instructions per
        # step (counted by rocprofv3 on this kernel source) over the live kernel time.
        vi = valu_for(dom)
        if vi:
            ach = vi / (t_ms * 1e-3) / 1e9
            roofline["alu"] = {"bound": "alu", "achieved": round(ach, 1), "peak": VALU_PEAK_G,
                               "unit": "G VALU wave instructions/s",
                               "frac": round(ach / VALU_PEAK_G, 4),
                               "valu_wave_instructions": vi}
    del bufs
    torch.cuda.empty_cache()
    dists = None
    if not args.no_distributions:
        dists = distributions_leg(args, ds, torch, dev)
    c3b = None
    if not args.no_c3b:
        c3b = c3b_leg(args, ds, torch, dev)
    batched = None
    if not args.no_batched:
        batched = batched_leg(args, ds, torch, dev)
    served = None
    if not args.no_served:
        served = served_leg(args, ds, torch, dev)
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        L = g.sublist_len
        s = g.samples
        cpu = cpu_baseline(args.seed, min(args.cpu_sample_log2, args.log2n), L, s, args.log2n)

    if batched:
        # the honest peer of the batched rate: the plain sort's own rate at 2^28
        batched["vs_plain_rate"] = round(batched["value"] / mkeys, 3)
    rec = {
        "metric": METRIC,
        "value": round(mkeys, 1),
        "unit": "Mkeys/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"plain sort of 2^{args.log2n} uint32 keys, uniform (SplitMix64 "
                               f"seed {args.seed}), keys only", "n": n,
                   "levels": g.levels, "L": g.sublist_len, "s": g.samples, "m": g.sublists,
                   "L2": g.sublist_len2, "s2": g.samples2},
        "step_ms": {"median": round(step_ms[K // 2], 4), "min": round(step_ms[0], 4),
                    "spread": round(step_ms[-1] - step_ms[0], 4)},
        "instrumented_ms_per_step": round(dt_instr / K * 1e3, 4) if dt_instr else None,
        "path_hbm_gbs": round(whole_bytes / (ms_per_step * 1e-3) / 1e9, 1) if stages else None,
        "path": path_roofline(n, kb, ms_per_step),
        "stage_ms": {k: round(v, 4) for k, v in groups.items()},
        "kernel_ms": stage_ms,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "distributions": dists,
        "c3b": c3b,
        "batched": batched,
        "served": served,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
