"""sof_find_splits_noalloc (static per-device scratch, no allocation) against
sof_find_splits (caller workspace) through the C ABI: identical records and
histograms on two calls in a row, the second on a smaller frontier, so stale
scratch contents of the first call must not leak into the second."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

from paper_2603_00326_amd import workloads as W
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


def _run_both(S, ctx, wl, **kw):
    import torch
    dev = S.to_device(wl, "cuda:0")
    ref, Href = S.find_splits(ctx, dev, bins=wl.bins, sort_threshold=wl.sort_threshold, hist=True, **kw)
    out = torch.full_like(ref, -7)
    H = torch.full_like(Href, -7)
    got, Hgot = S.find_splits_noalloc(ctx, dev, bins=wl.bins, sort_threshold=wl.sort_threshold, hist=H,
                                      out=out, **kw)
    torch.cuda.synchronize()
    n = wl.n_nodes
    a = got[:n].cpu().numpy()
    b = ref[:n].cpu().numpy()
    assert np.array_equal(a, b), f"records differ: first node {int(np.nonzero((a != b).any(1))[0][0])}"
    assert np.array_equal(Hgot.cpu().numpy(), Href.cpu().numpy()), "histograms differ"
    return int((S.splits_to_numpy(got)[:n]["proj"] >= 0).sum())


@pytest.mark.parametrize("criterion", [0, 1])
def test_noalloc_equals_workspace_call_twice(criterion):
    from paper_2603_00326_amd import sof as S
    ctx = S.Context(0)
    big = W.random_frontier(21, n_rows=60000, d=24, n_classes=3,
                            sizes=[3, 40, 64, 65, 300, 512, 513, 2000, 4097, 8192, 8193, 30001],
                            k=9, z=4, bins=256, sort_threshold=0 if criterion else 100, layout="b")
    small = W.random_frontier(22, n_rows=20000, d=24, n_classes=3, sizes=[7, 600, 9000, 100],
                              k=5, z=3, bins=128, sort_threshold=0 if criterion else 50, layout="a")
    for name, wl in (("first call (12 nodes, up to 30001 samples)", big),
                     ("second call (4 nodes, up to 9000 samples)", small)):
        say(f"[noalloc] criterion {criterion}: {name}")
        n_split = _run_both(S, ctx, wl, criterion=criterion)
        assert n_split > 0


def test_noalloc_fp16_random_bins():
    from paper_2603_00326_amd import sof as S
    ctx = S.Context(0)
    wl = W.random_frontier(23, n_rows=50000, d=16, n_classes=2, sizes=[20, 700, 5000, 20000],
                           k=6, z=5, bins=200, sort_threshold=30, layout="b", dtype=np.float16)
    say("[noalloc] FP16, random-width bins")
    _run_both(S, ctx, wl, bin_mode=S.SOF_BINS_RANDOM, bin_seed=99)


def test_noalloc_under_graph_capture():
    """The callers it is for capture it: sof_find_splits_noalloc recorded in a
    HIP graph and replayed three times, with eager calls on another frontier
    (which reuse the same static scratch) between the replays, gives the
    workspace call's records and histograms every time."""
    import torch
    from paper_2603_00326_amd import sof as S
    ctx = S.Context(0)
    wl = W.random_frontier(24, n_rows=60000, d=16, n_classes=3, sizes=[5, 300, 2000, 9000, 20000], k=6, z=3,
                           bins=256, sort_threshold=64, layout="b")
    other = W.random_frontier(25, n_rows=20000, d=16, n_classes=3, sizes=[40, 3000, 12000], k=4, z=2,
                              bins=128, sort_threshold=64, layout="a")
    say("[noalloc] graph capture")
    dev, odev = S.to_device(wl, "cuda:0"), S.to_device(other, "cuda:0")
    ref, Href = S.find_splits(ctx, dev, bins=wl.bins, sort_threshold=64, hist=True)
    torch.cuda.synchronize()
    out = torch.empty_like(ref)
    H = torch.empty_like(Href)
    oout = torch.empty((other.n_nodes, 10), dtype=torch.int32, device="cuda:0")
    S.find_splits_noalloc(ctx, dev, bins=wl.bins, sort_threshold=64, hist=H, out=out)   # warm-up, eager
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        S.find_splits_noalloc(ctx, dev, bins=wl.bins, sort_threshold=64, hist=H, out=out)
    torch.cuda.synchronize()
    for rep in range(3):
        out.fill_(-7)
        H.fill_(-7)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out[:wl.n_nodes], ref[:wl.n_nodes]), f"replay {rep}: records"
        assert torch.equal(H, Href), f"replay {rep}: histograms"
        S.find_splits_noalloc(ctx, odev, bins=other.bins, sort_threshold=64, out=oout)
        torch.cuda.synchronize()
    del g


def test_noalloc_rejects_sizes_above_the_scratch():
    from paper_2603_00326_amd import sof as S
    from paper_2603_00326_amd import sof
    ctx = S.Context(0)
    fake = 0x10000   # never dereferenced: the size check runs before any launch
    d = sof.sof_data(fake, fake, 4_000_000, 4_000_000, 512, 3, sof.SOF_F32)
    f = sof.sof_frontier(fake, fake, 4_000_000, 4096, 100_000)
    p = sof.sof_proj(fake, fake, fake, fake, 4 * 262144, 262144, 64, None)
    q = sof.sof_params(None, 256, 4, 0, 0, 0)
    L = sof.lib()
    rc = L.sof_find_splits_noalloc(ctx.handle, ctypes.byref(d), ctypes.byref(f), ctypes.byref(p),
                                   ctypes.byref(q), fake, None, None)
    assert rc == sof.SOF_ERR_WORKSPACE
    assert b"static" in L.sof_last_error()
