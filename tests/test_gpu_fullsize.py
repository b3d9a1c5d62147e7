"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times (one batched call over the whole frontier, the autotuned sort
threshold, then the partition of every node): every node's split record and
the whole partition against the oracle run over the same frontier, plus the
properties that hold at any size (each node's output block is a permutation
of its samples, split into a left block of the measured size that matches
the split's left count)."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_00326_amd import workloads as W
from tests.gpu_helpers import assert_splits_match, say

pytestmark = pytest.mark.gpu

@pytest.fixture(scope="module")
def ctx():
    from paper_2603_00326_amd import sof as S
    return S.Context(0)


def tune(ctx, wl):
    """The benchmark's tuning: the crossover microbenchmark on the workload's
    own matrix and labels."""
    from paper_2603_00326_amd import sof as S
    return S.autotune(ctx, wl.n_classes, int(wl.meta.get("k", 64)), int(wl.meta.get("z", 3)), wl.bins,
                      data=S.to_device(wl))


def tuned_threshold(ctx, wl):
    return int(tune(ctx, wl)["sort_threshold"])


def tuned_config3(ctx, wl):
    """The benchmark's configuration of a config-3 frontier: the autotuned
    switch, half the bins below the autotuned size (128-256 bins), and the
    autotuned wave tile (passed on by run_full)."""
    t = tune(ctx, wl)
    if t["bins_switch"] > 0:
        n = np.diff(wl.node_offsets.astype(np.int64))
        wl.node_bins = np.where(n < t["bins_switch"], t["bins_small"], wl.bins).astype(np.int32)
    return int(t["sort_threshold"]), t


def run_full(ctx, wl, T, bin_mode=0, bin_seed=0, criterion=0, tune=None):
    import torch
    from paper_2603_00326_amd import sof as S
    dev = S.to_device(wl)
    tiles = dict(small_max=tune["small_max"], mid_split=tune["mid_split"]) if tune else {}
    out, _ = S.find_splits(ctx, dev, bins=wl.bins, sort_threshold=T, bin_mode=bin_mode, bin_seed=bin_seed,
                           criterion=criterion, **tiles)
    out_idx, coff = S.partition(ctx, dev, out, bins=wl.bins)
    torch.cuda.synchronize()
    got = S.splits_to_numpy(out)[:wl.n_nodes]
    res = got.copy(), out_idx.cpu().numpy(), coff.cpu().numpy()
    del dev, out, out_idx, coff
    torch.cuda.empty_cache()
    return res


def check_partition_properties(wl, got, out_idx, coff):
    N = wl.n_nodes
    no = wl.node_offsets.astype(np.int64)
    n = np.diff(no)
    assert coff[2 * N] == no[-1]
    assert np.array_equal(coff[0:2 * N:2], no[:-1]), "child block starts"
    n_left = coff[1:2 * N:2].astype(np.int64) - no[:-1]
    split = got["proj"] >= 0
    assert np.array_equal(n_left[split], got["n_left"][split]), "measured left count vs the split's"
    assert np.array_equal(n_left[~split], n[~split]), "an unsplit node keeps every sample on the left"
    node_of = np.repeat(np.arange(N), n)
    a = np.lexsort((wl.sample_idx, node_of))
    b = np.lexsort((out_idx, node_of))
    assert np.array_equal(wl.sample_idx[a], out_idx[b]), "per-node permutation"


def check_all(wl, T, got, out_idx, coff, tag, bin_mode=0, bin_seed=0, criterion=0):
    """Every node's record and the whole partition against the oracle run
    over the same frontier."""
    ref, _ = O.find_splits_w(wl, sort_threshold=T, bin_mode=bin_mode, bin_seed=bin_seed, criterion=criterion)
    assert_splits_match(got, ref, tag)
    want_idx, want_coff = O.partition(wl.X, wl.node_offsets, wl.sample_idx, wl.proj_offsets, wl.nz_offsets,
                                      wl.nz_feature, wl.nz_weight, ref, bins=wl.bins, node_bins=wl.node_bins)
    bad = np.nonzero(coff != want_coff)[0]
    assert bad.size == 0, f"{tag}: child offset {bad[0]} differs: {coff[bad[0]]} vs {want_coff[bad[0]]}"
    bad = np.nonzero(out_idx != want_idx)[0]
    assert bad.size == 0, f"{tag}: partition differs at position {bad[0]} ({bad.size} positions)"


@pytest.mark.parametrize("layout", ["a", "b"])
def test_frontier_4096_lognormal_nodes(ctx, layout):
    wl = W.config3(layout)
    T0, t = tuned_config3(ctx, wl)
    for T in sorted({T0, 48}):
        say(f"[gpu] full frontier layout={layout} nodes={wl.n_nodes} samples={wl.n_samples} T={T} "
            f"bins {t['bins_small']} below n={t['bins_switch']}, wave tile {t['small_max']}/{t['mid_split']}")
        got, out_idx, coff = run_full(ctx, wl, T, tune=t)
        check_partition_properties(wl, got, out_idx, coff)
        check_all(wl, T, got, out_idx, coff, f"c3{layout} T={T}")


def test_root_1m_rows_256_projections(ctx):
    wl = W.config2()
    T = tuned_threshold(ctx, wl)
    say(f"[gpu] root n={wl.n_samples} k={wl.n_proj} T={T}")
    got, out_idx, coff = run_full(ctx, wl, T)
    check_partition_properties(wl, got, out_idx, coff)
    check_all(wl, T, got, out_idx, coff, "c2")


def test_root_10m_rows_fp16_equals_fp32_and_oracle(ctx):
    w16 = W.config5(fp16=True)
    T = tuned_threshold(ctx, w16)
    say(f"[gpu] root n={w16.n_samples} FP16 T={T}")
    g16, i16, c16 = run_full(ctx, w16, T)
    check_partition_properties(w16, g16, i16, c16)
    check_all(w16, T, g16, i16, c16, "c5 fp16")
    del w16
    w32 = W.config5(fp16=False)
    say(f"[gpu] root n={w32.n_samples} FP32 T={T}")
    g32, i32, c32 = run_full(ctx, w32, T)
    assert g16.tobytes() == g32.tobytes(), "FP16 and FP32 storage give different split records"
    assert np.array_equal(i16, i32) and np.array_equal(c16, c32), "FP16 and FP32 partitions differ"


@pytest.mark.parametrize("T", [0, 2**31 - 1])
def test_root_4096_rows_both_paths(ctx, T):
    wl = W.config1(sort=T != 0)
    say(f"[gpu] root n={wl.n_samples} T={T}")
    got, out_idx, coff = run_full(ctx, wl, T)
    check_partition_properties(wl, got, out_idx, coff)
    check_all(wl, T, got, out_idx, coff, f"c1 T={T}")


def test_frontier_4096_nodes_random_width_bins(ctx):
    wl = W.config3("a")
    T, t = tuned_config3(ctx, wl)
    seed = 20260302
    say(f"[gpu] full frontier random-width bins nodes={wl.n_nodes} samples={wl.n_samples} T={T}")
    got, out_idx, coff = run_full(ctx, wl, T, bin_mode=1, bin_seed=seed, tune=t)
    check_partition_properties(wl, got, out_idx, coff)
    check_all(wl, T, got, out_idx, coff, "c3a random-width", bin_mode=1, bin_seed=seed)


def test_frontier_4096_nodes_entropy(ctx):
    wl = W.config3("a")
    _, t = tuned_config3(ctx, wl)
    say(f"[gpu] full frontier entropy criterion nodes={wl.n_nodes} samples={wl.n_samples} T=0")
    got, out_idx, coff = run_full(ctx, wl, 0, criterion=1, tune=t)
    check_partition_properties(wl, got, out_idx, coff)
    check_all(wl, 0, got, out_idx, coff, "c3a entropy", criterion=1)


@pytest.mark.parametrize("criterion", [0, 1])
def test_root_at_the_maximum_node_size(ctx, criterion):
    """One root of exactly 2^24 samples, the largest node the exact 128-bit
    comparisons admit (2^24 + 1 is rejected on the host), FP16 storage,
    random labels (near-ties everywhere), Gini and entropy (whose class
    counts here exceed the k ln k table and are computed directly)."""
    n = 1 << 24
    wl = W.random_frontier(71, n_rows=n, d=6, n_classes=2, sizes=[n], k=4, z=(1, 3), bins=256,
                           sort_threshold=0, layout="a", dtype=np.float16)
    say(f"[gpu] root n=2^24 FP16 criterion={criterion}")
    got, out_idx, coff = run_full(ctx, wl, 0, criterion=criterion)
    ref, _ = O.find_splits_w(wl, criterion=criterion)
    assert_splits_match(got, ref, f"n=2^24 criterion={criterion}")
    check_partition_properties(wl, got, out_idx, coff)
    want_idx, want_coff = O.partition(wl.X, wl.node_offsets, wl.sample_idx, wl.proj_offsets, wl.nz_offsets,
                                      wl.nz_feature, wl.nz_weight, ref, bins=wl.bins)
    assert np.array_equal(coff, want_coff) and np.array_equal(out_idx, want_idx)


def test_project_full_frontier_sampled_nodes(ctx):
    """sof_project over the whole 4096-node frontier (the launch the benchmark
    times, 2.6e8 values): the blocks of 64 nodes drawn from every size class,
    including the largest, equal the oracle's projection bit for bit."""
    import torch
    from paper_2603_00326_amd import sof as S
    wl = W.config3("a")
    say(f"[gpu] project full frontier nodes={wl.n_nodes} units={wl.units}")
    dev = S.to_device(wl)
    got = S.project(ctx, dev)
    torch.cuda.synchronize()
    n = np.diff(wl.node_offsets.astype(np.int64))
    k = np.diff(wl.proj_offsets.astype(np.int64))
    off = np.concatenate([[0], np.cumsum(n * k)])
    rng = np.random.default_rng(5)
    order = np.argsort(n)
    pick = sorted(set(rng.choice(wl.n_nodes, 56, replace=False).tolist()) | set(order[-8:].tolist()))
    sub = W.sub_frontier(wl, pick)
    want = O.project(sub.X, sub.node_offsets, sub.sample_idx, sub.proj_offsets, sub.nz_offsets, sub.nz_feature,
                     sub.nz_weight)
    g = got.cpu().numpy()
    pos = 0
    for v in pick:
        m = int(n[v] * k[v])
        assert np.array_equal(g[off[v]:off[v] + m].view(np.uint32), want[pos:pos + m].view(np.uint32)), f"node {v}"
        pos += m
