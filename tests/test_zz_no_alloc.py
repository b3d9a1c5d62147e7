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
