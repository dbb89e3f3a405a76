"""HIP graph capture of whole sorts: the launches of one plain or segmented call are recorded
once and replayed on new inputs.  Every replay is checked against the oracle and against an
eager call on the same input, with eager work and synchronisations between replays."""
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


def _capture(torch, fn):
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()  # eager warm-up on a side stream, as torch's capture recipe asks
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


def test_segmented_graph_replays(ds):
    import torch
    sizes = synth.segment_sizes(96, 5, 6, 18)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n = int(offs[-1])
    plan = ds.Plan(3, False, n, max_segments=sizes.size)
    ws = plan.workspace("cuda")
    t_off = torch.from_numpy(offs).cuda()
    static = torch.zeros(n, dtype=torch.int32, device="cuda")
    g = _capture(torch, lambda: plan.sort_segmented(static, t_off, max_segment=int(sizes.max()),
                                                    workspace=ws))
    for seed in range(4):
        x = synth.normal_f32_segments(sizes, 100 + seed, dup_frac=0.05, zero_log2=6)
        want, _ = oracle.segmented_sort(x, offs)
        say("[graph] segmented replay", seed, "n =", n)
        static.copy_(to_dev(x))
        g.replay()
        torch.cuda.synchronize()
        got = from_dev(static, np.float32)
        assert (got.view(np.uint32) == want.view(np.uint32)).all(), f"replay {seed}"
        eager = to_dev(x)
        plan.sort_segmented(eager, t_off, max_segment=int(sizes.max()), workspace=ws)
        torch.cuda.synchronize()
        assert torch.equal(eager, static)


@pytest.mark.parametrize("n", [30_000, (1 << 20) + 5, 5_000_000])
def test_plain_graph_replays(ds, n):
    import torch
    plan = ds.Plan(1, True, n)
    ws = plan.workspace("cuda")
    k = torch.zeros(n, dtype=torch.int32, device="cuda")
    v = torch.zeros(n, dtype=torch.int32, device="cuda")
    g = _capture(torch, lambda: plan.sort_pairs(k, v, ws))
    for seed in range(3):
        keys = synth.make_u32(["uniform", "bucket", "equal"][seed], n, 60 + seed)
        vals = synth.index_values(n)
        want_k, want_v = oracle.stable_sort(keys, vals)
        say("[graph] plain replay", seed, "n =", n)
        k.copy_(to_dev(keys))
        v.copy_(to_dev(vals))
        g.replay()
        torch.cuda.synchronize()
        assert (from_dev(k, np.uint32) == want_k).all()
        assert (from_dev(v, np.uint32) == want_v).all()
        ek, ev = to_dev(keys), to_dev(vals)
        plan.sort_pairs(ek, ev, ws)
        torch.cuda.synchronize()
        assert torch.equal(ek, k) and torch.equal(ev, v)
