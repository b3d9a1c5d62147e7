"""The batched split search and the partition captured into one HIP graph
(PyTorch's capture on its side stream; the library's fork onto the context's
two streams becomes graph branches) and replayed: every replay, with eager
library work and synchronisations between replays, reproduces the eager
call's split records, histograms and partition."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2603_00326_amd import workloads as W
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("T,criterion", [(100, 0), (0, 1)])
def test_find_and_partition_graph_replays(T, criterion):
    import torch
    from paper_2603_00326_amd import sof as S
    ctx = S.Context(0)
    other_ctx = S.Context(0)   # the eager work between replays keeps its own workspace
    wl = W.random_frontier(41, n_rows=80000, d=20, n_classes=3,
                           sizes=[2, 30, 64, 65, 300, 512, 513, 2000, 4097, 8192, 8193, 20000], k=7, z=3,
                           bins=256, sort_threshold=T, layout="b")
    other = W.random_frontier(42, n_rows=30000, d=20, n_classes=3, sizes=[10, 700, 9000], k=5, z=3, bins=128,
                              sort_threshold=T, layout="r")
    say(f"[gpu] graph replays T={T} criterion={criterion}")
    dev, odev = S.to_device(wl), S.to_device(other)
    N = wl.n_nodes
    out = torch.empty((N, 10), dtype=torch.int32, device="cuda:0")

    def step():
        S.find_splits(ctx, dev, bins=wl.bins, sort_threshold=T, out=out, hist=False, criterion=criterion)
        return S.partition(ctx, dev, out, bins=wl.bins)

    idx_e, coff_e = step()
    torch.cuda.synchronize()
    ref = (out.clone(), idx_e.clone(), coff_e.clone())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        idx_g, coff_g = step()
    torch.cuda.synchronize()
    for rep in range(3):
        for t in (out, idx_g, coff_g):
            t.fill_(-7)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref[0]), f"replay {rep}: records"
        assert torch.equal(idx_g, ref[1]) and torch.equal(coff_g, ref[2]), f"replay {rep}: partition"
        # eager library work between replays
        S.find_splits(other_ctx, odev, bins=other.bins, sort_threshold=T, criterion=criterion)
        torch.cuda.synchronize()
    del g
