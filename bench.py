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


def stage_bytes(stage: str, n: int, g, kb: int) -> float:
    """Algorithmic HBM bytes of one launch of a stage (the minimum the stage must move)."""
    sb = g.sample_bytes
    m1s1 = g.sublists * g.samples
    m2s2 = (n // max(g.sublist_len2, 1)) * g.samples2 if g.levels == 2 else 0
    if stage == "s123_local_sort":
        return 2 * n * kb + m1s1 * sb
    if stage == "l2_s123_local_sort":
        return 2 * n * kb + m2s2 * sb
    if stage in ("s8_relocate",):
        return 2 * n * kb + 2 * m1s1 * 4
    if stage in ("l2_s8_relocate",):
        return 2 * n * kb + 2 * m2s2 * 4
    if stage == "s9_bucket_sort":
        return 2 * n * kb
    if stage == "s56_rank":
        return n * kb + m1s1 * (sb + 4)
    if stage == "l2_s56_rank":
        return n * kb + m2s2 * (sb + 4)
    return 0.0


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_for(stage: str):
    """Measured HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by a copy
    kernel), if recorded for the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except OSError:
        return None
    if t.get("kernel_source_sha256_16") != kernel_hash():
        return None
    v = t.get("bytes_per_launch", {}).get(stage)
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
    args = ap.parse_args()
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

    out = bufs[-1][: 1 << 20].cpu().numpy().view(np.uint32)
    assert (out[1:] >= out[:-1]).all(), "output prefix not sorted"
    status = int(ws[:4].cpu().numpy().view(np.uint32)[0])
    assert status == 0, f"kernel status flags {status:#x}"

    ms_per_step = dt / K * 1e3
    mkeys = n / (dt / K) / 1e6
    stage_ms = {k: round(v[0] * v[1] / K, 4) for k, v in stages.items()}
    kb = 4
    roofline = None
    if stages:
        dom = max(stages, key=lambda k: stages[k][0] * stages[k][1])
        avg_ms, launches = stages[dom]
        alg = stage_bytes(dom, n, g, kb)
        achieved = alg / (avg_ms * 1e-3) / 1e9 if alg else 0.0
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": traffic_for(dom), "algorithmic_bytes": alg,
                    "avg_launch_ms": round(avg_ms, 4)}
    whole_bytes = sum(stage_bytes(k, n, g, kb) * v[1] / K for k, v in stages.items())
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
        "stage_ms": stage_ms,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
