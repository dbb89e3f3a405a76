"""GPU tests of the served sort stream: mixed requests (uint32 keys, uint64 key/value pairs,
float32 keys; sizes spanning the batched and the alone classes) submitted in bursts and as a
Poisson stream, each result bit-exact against the oracle and identical alone and in the mix;
admission by a small memory budget; capacity errors."""
import threading
import time

import numpy as np
import pytest

import oracle
import synth
from helpers import from_dev, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ds():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1002_4464_amd as d
    d.load_library()
    return d


def make_requests(count, seed, lo_log2=10, hi_log2=22):
    """(keys, values or None) host arrays; layouts alternate u32 keys / u64 pairs / f32 keys."""
    sizes = synth.segment_sizes(count, seed, lo_log2, hi_log2)
    reqs = []
    for i, n in enumerate(sizes.tolist()):
        kind = i % 3
        if kind == 0:
            keys = synth.make_u32("uniform" if i % 2 else "bucket", n, seed * 1000 + i)
            reqs.append((keys, None))
        elif kind == 1:
            keys = synth.zipf_u64(n, seed * 1000 + i) if i % 2 else synth.uniform_u64(
                n, seed * 1000 + i)
            reqs.append((keys, synth.index_values(n)))
        else:
            sz = np.array([n], dtype=np.int64)
            reqs.append((synth.normal_f32_segments(sz, seed * 1000 + i, 0.05, 6), None))
    return reqs


KT = {np.dtype(np.uint32): 1, np.dtype(np.uint64): 2, np.dtype(np.float32): 3}


def submit_all(srv, dev, reqs, sync=False):
    return [srv.submit(tk, tv, key_type=KT[k.dtype], sync=sync)
            for (tk, tv), (k, _) in zip(dev, reqs)]


def expected(reqs):
    return [oracle.stable_sort(k, v) for k, v in reqs]


def check(got, want, i):
    gk, gv = got
    wk, wv = want
    assert (gk.view(np.uint8) == wk.view(np.uint8)).all(), f"request {i} keys"
    if wv is not None:
        assert (gv == wv).all(), f"request {i} values"


def to_device(reqs):
    dev = []
    for k, v in reqs:
        dev.append((to_dev(k), to_dev(v) if v is not None else None))
    return dev


def fetch(dev_reqs, reqs):
    out = []
    for (tk, tv), (k, v) in zip(dev_reqs, reqs):
        out.append((from_dev(tk, k.dtype), from_dev(tv, np.uint32) if tv is not None else None))
    return out


def test_burst_mixed_layouts(ds):
    import torch
    reqs = make_requests(60, 3)
    want = expected(reqs)
    dev = to_device(reqs)
    torch.cuda.synchronize()
    srv = ds.Server(2 << 30, max_inflight=256, lanes=4)
    say("[server] burst of", len(reqs), "requests")
    tickets = submit_all(srv, dev, reqs)
    results = [srv.wait(t) for t in tickets]
    stats = srv.stats()
    say("[server] stats", stats)
    got = fetch(dev, reqs)
    for i in range(len(reqs)):
        check(got[i], want[i], i)
    assert stats["completed"] == len(reqs) and stats["failed"] == 0
    assert stats["batched_units"] > 0, "a burst of small requests should be batched"
    assert stats["peak_arena_bytes"] <= 2 << 30
    assert all(r.t_submit_ns <= r.t_admit_ns <= r.t_done_ns for r in results)
    for t in tickets:
        srv.release(t)
    srv.close()


def test_alone_equals_in_mix(ds):
    """Each request sorted alone through the server equals the same request sorted inside a
    mixed burst, bit for bit (and both equal the oracle)."""
    import torch
    reqs = make_requests(24, 5, 8, 20)
    srv = ds.Server(1 << 30, max_inflight=128, lanes=3)
    dev_mix = to_device(reqs)
    torch.cuda.synchronize()
    tickets = submit_all(srv, dev_mix, reqs)
    units = [srv.wait(t).unit for t in tickets]
    mix = fetch(dev_mix, reqs)
    alone = []
    for k, v in reqs:
        (tk, tv), = to_device([(k, v)])
        srv.wait(srv.submit(tk, tv, key_type=KT[k.dtype]))
        alone.append((from_dev(tk, k.dtype), from_dev(tv, np.uint32) if tv is not None else None))
    want = expected(reqs)
    for i in range(len(reqs)):
        check(mix[i], alone[i], i)
        check(alone[i], want[i], i)
    assert len(set(units)) < len(units), "the mixed burst should share launches"
    srv.close()


def test_small_budget_admission(ds):
    """With an arena too small to hold every request's workspace at once, requests wait for
    memory and still all finish correctly; the arena is never exceeded."""
    import torch
    reqs = [(synth.uniform_u32(3 << 20, 70 + i), None) for i in range(6)]
    reqs += [(synth.uniform_u64(1 << 19, 80 + i), synth.index_values(1 << 19)) for i in range(4)]
    budget = 48 << 20
    srv = ds.Server(budget, max_inflight=64, lanes=4)
    dev = to_device(reqs)
    torch.cuda.synchronize()
    tickets = submit_all(srv, dev, reqs)
    for t in tickets:
        srv.wait(t, timeout_s=120)
    stats = srv.stats()
    got = fetch(dev, reqs)
    want = expected(reqs)
    for i in range(len(reqs)):
        check(got[i], want[i], i)
    assert stats["peak_arena_bytes"] <= budget
    srv.close()


def test_capacity_and_argument_errors(ds):
    import torch
    srv = ds.Server(4 << 20, max_inflight=8, lanes=1)
    big = torch.zeros(1 << 24, dtype=torch.int32, device="cuda")
    with pytest.raises(ds.DsortError) as e:
        srv.submit(big)
    assert e.value.status == ds.E_CAPACITY
    with pytest.raises(ds.DsortError) as e:
        srv.poll(12345)
    assert e.value.status == ds.E_TICKET
    tiny = torch.tensor([3, 1, 2], dtype=torch.int32, device="cuda")
    t = srv.submit(tiny)
    srv.wait(t)
    assert tiny.cpu().tolist() == [1, 2, 3]
    srv.release(t)
    with pytest.raises(ds.DsortError):
        srv.release(t)
    empty = torch.zeros(0, dtype=torch.int32, device="cuda")
    srv.wait(srv.submit(empty))
    srv.close()


def test_poisson_stream(ds):
    """Requests submitted from another thread at Poisson arrival times while earlier ones run;
    every result matches the oracle and latencies are recorded."""
    import torch
    reqs = make_requests(80, 9, 10, 21)
    want = expected(reqs)
    dev = to_device(reqs)
    torch.cuda.synchronize()
    srv = ds.Server(2 << 30, max_inflight=256, lanes=4)
    gaps = -np.log(1.0 - (synth.draws64(99, len(reqs)) >> np.uint64(11)).astype(np.float64)
                   / float(1 << 53)) * 2e-4  # mean 0.2 ms between arrivals
    tickets = [None] * len(reqs)

    def producer():
        t_next = time.perf_counter()
        for i, ((tk, tv), (k, _)) in enumerate(zip(dev, reqs)):
            t_next += gaps[i]
            while time.perf_counter() < t_next:
                pass
            tickets[i] = srv.submit(tk, tv, key_type=KT[k.dtype], sync=False)

    th = threading.Thread(target=producer)
    th.start()
    th.join()
    lat = np.array([srv.wait(t).latency_s for t in tickets])
    got = fetch(dev, reqs)
    for i in range(len(reqs)):
        check(got[i], want[i], i)
    say(f"[server] poisson: p50 {np.percentile(lat, 50) * 1e3:.3f} ms, "
        f"p99 {np.percentile(lat, 99) * 1e3:.3f} ms, stats {srv.stats()}")
    srv.close()
