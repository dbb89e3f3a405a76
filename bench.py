"""Benchmark: one step = one plain deterministic sample sort (every step of Algorithm 1) of
2^28 uint32 keys, uniform over [0, 2^32) from the seeded SplitMix64 stream (seed 8), keys only,
on one MI355X.  Inputs are resident in HBM before timing starts: one copy per step, so every
timed sort sees the same unsorted input and nothing but sorting happens in the timed region.

Prints one JSON line with the throughput (Mkeys/s), the per-stage kernel times measured with
HIP events on the sort's stream over the timed region, the HBM roofline of the dominant kernel,
and the CPU oracle timed on a bounded sample of the same stream.
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
METRIC = "Mkeys/s + HBM GB/s (2^28 u32); p50/p99 latency, batched/served vs plain sort"
KERNEL_SRC = os.path.join(ROOT, "paper_1002_4464_amd", "csrc", "kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Pipeline stages as timed by the library (kernel launches grouped by the step they implement).
STAGE_GROUPS = {
    "steps1-3 local sort + sampling": ["s123_local_sort"],
    "step4 sample sort": ["s4_sample_sort", "s4_sample_merge"],
    "steps5-6 rank": ["s56_rank"],
    "step7 scan": ["s7_scan_colsum", "s7_scan_mid", "s7_scan_update", "s7_scan"],
    "step8 relocate": ["s8_relocate"],
    "level2 steps1-3": ["l2_s123_local_sort"],
    "level2 step4": ["l2_s4_sample_sort", "l2_s4_sample_merge"],
    "level2 steps5-6": ["l2_s56_rank"],
    "level2 step7": ["l2_s7_scan"],
    "steps8-9 gather + bucket sort": ["s89_gather_sort", "s89_gather_merge", "s9_bucket_sort"],
}


def group_bytes(group: str, n: int, g, kb: int) -> float:
    """Algorithmic HBM bytes one step of a stage group must move (the design doc lists them):
    a sort or move of the data reads and writes n keys once; ranking reads the sorted sublists
    once plus the splitters and writes the counts; samples, counts and offsets are small."""
    sb = g.sample_bytes
    m1s1 = g.sublists * g.samples
    m2s2 = -(-n // max(g.sublist_len2, 1)) * g.samples2 if g.levels == 2 else 0
    return {
        "steps1-3 local sort + sampling": 2 * n * kb + m1s1 * sb,
        "step4 sample sort": 2 * m1s1 * sb,
        "steps5-6 rank": n * kb + m1s1 * (sb + 4),
        "step8 relocate": 2 * n * kb + 2 * m1s1 * 4,
        "level2 steps1-3": 2 * n * kb + m2s2 * sb,
        "level2 steps5-6": n * kb + m2s2 * (sb + 4),
        "steps8-9 gather + bucket sort": 2 * n * kb,
    }.get(group, 0.0)


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_for(stage: str):
    """Measured HBM bytes per step of a stage group (rocprofv3 FETCH_SIZE + WRITE_SIZE, each
    scaled by a copy kernel of known size), if recorded for the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except OSError:
        return None
    if t.get("kernel_source_sha256_16") != kernel_hash():
        return None
    v = t.get("bytes_per_step", {}).get(stage)
    return float(v) if v is not None else None


def cpu_baseline(seed: int, sample_log2: int, L: int, s: int):
    import oracle
    n = 1 << sample_log2
    keys = __import__("synth").uniform_u32(n, seed)
    t0 = time.perf_counter()
    out, _, _ = oracle.dss(keys, L, s)
    dt = time.perf_counter() - t0
    assert (out[1:] >= out[:-1]).all()
    return {"value": round(n / dt / 1e6, 3), "unit": "Mkeys/s", "cores": 1, "kind": "oracle",
            "sample": f"first 2^{sample_log2} keys of the same uniform stream (seed {seed}); "
                      f"single-threaded C oracle of Algorithm 1 with L={L}, s={s}; {dt:.1f} s"}


def _group_of(kernel: str, seen: dict) -> str:
    """Maps a rocprofv3 kernel name of one sort to its stage group; the Step 1-3 tile kernels
    run once per level, so their first launch in a sort is level 1 and the second level 2."""
    name = kernel.replace("dsort::(anonymous namespace)::", "")
    if name.startswith("k_tile_radix") or name.startswith("void k_tile_radix") or \
            (name.startswith("void k_tile<") and ", 0," in name):
        seen["tile"] = seen.get("tile", 0) + 1
        return "steps1-3 local sort + sampling" if seen["tile"] % 2 == 1 else "level2 steps1-3"
    for key, grp in (("k_gather", "steps8-9 gather + bucket sort"),
                     ("k_tile<", "steps8-9 gather + bucket sort"),
                     ("k_relocate", "step8 relocate"),
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
        copies = [float(r["Counter_Value"]) * 1024 for r in rows
                  if "copyBuffer" in r["Kernel_Name"] or "elementwise" in r["Kernel_Name"]]
        # the calibration copy is the last copy kernel in the run
        scale = copy_bytes / copies[-1] if copies and copies[-1] > 0 else 1.0
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--seed", type=int, default=8)
    ap.add_argument("--cpu-sample-log2", type=int, default=26)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stage-timing", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="after timing, copy BYTES bytes with torch (a kernel of known size for "
                         "scaling rocprofv3 FETCH_SIZE/WRITE_SIZE)")
    ap.add_argument("--ingest-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn two rocprofv3 counter CSVs of a --copy-calibration run into "
                         "profiles/traffic.json (CPU only)")
    ap.add_argument("--sorts", type=int, default=1, help="sorts in the ingested runs")
    args = ap.parse_args()
    if args.ingest_pmc:
        ingest_pmc(args.ingest_pmc[0], args.ingest_pmc[1], args.copy_calibration, args.sorts,
                   TRAFFIC_FILE)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1002_4464_amd as ds
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    n = 1 << args.log2n
    K, W = args.steps, args.warmup

    log(f"[bench] generating 2^{args.log2n} uniform u32 keys (seed {args.seed})")
    keys = synth.uniform_u32(n, args.seed)
    src = torch.from_numpy(keys.view(np.int32)).to(dev)
    bufs = [src.clone() for _ in range(W + K)]
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
    plan.set_timing(not args.no_stage_timing)
    log(f"[bench] timing {K} steps")
    t0 = time.perf_counter()
    for i in range(W, W + K):
        plan.sort_keys(bufs[i], ws, stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stages = plan.stage_times() if not args.no_stage_timing else {}
    plan.set_timing(False)
    if args.copy_calibration:
        cs = torch.empty(args.copy_calibration // 4, dtype=torch.int32, device=dev)
        cd = torch.empty_like(cs)
        cd.copy_(cs)
        torch.cuda.synchronize()
        del cs, cd

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
                                             if nm in stages) // K}
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        L = g.sublist_len
        s = g.samples
        cpu = cpu_baseline(args.seed, args.cpu_sample_log2, L, s)

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
        "path_hbm_gbs": round(whole_bytes / (ms_per_step * 1e-3) / 1e9, 1) if stages else None,
        "stage_ms": {k: round(v, 4) for k, v in groups.items()},
        "kernel_ms": stage_ms,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
