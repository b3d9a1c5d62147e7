"""GPU parity of level-wise forest growth (sof_grow_level) against the CPU
oracle: the device projection sampler, batched split search, partition, leaf
detection and node records of several trees grown to purity, with and without
per-level graph replay."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2603_00326_amd import sof as S
    return S.Context(0)


def grow_case(ctx, *, seed, d, n, C, trees, k, z, bins, T, max_depth=64, graph=True, dtype=np.float32,
              stats=False, sampler=0, weights=0, first_tree=0, criterion=0, bin_mode=0, bin_seed=0):
    import torch
    from paper_2603_00326_amd import sof as S
    say(f"[gpu] grow seed={seed} d={d} n={n} C={C} trees={trees} k={k} z={z} B={bins} T={T} "
        f"max_depth={max_depth} graph={graph} dtype={np.dtype(dtype).name} sampler={sampler} weights={weights} "
        f"first_tree={first_tree} criterion={criterion} bin_mode={bin_mode}")
    modes = dict(criterion=criterion, bin_mode=bin_mode, bin_seed=bin_seed)
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((d, n)).astype(np.float32)
    if dtype == np.float16:
        X = (np.clip(np.rint(X * 256.0), -2048, 2048) / 256.0).astype(np.float32)
    y = rng.integers(0, C, size=n).astype(np.int32)
    roots = [np.sort(np.random.default_rng(seed * 100 + t).integers(0, n, n)).astype(np.int32)
             for t in range(trees)]
    ro = np.arange(trees + 1, dtype=np.int64) * n
    ri = np.concatenate(roots)
    ref, ref_levels, ref_units = O.grow_forest(X, y, C, ro, ri, k=k, z=z, seed=seed + 7, bins=bins,
                                               sort_threshold=T, max_depth=max_depth, sampler=sampler,
                                               weights=weights, first_tree=first_tree, **modes)
    Xd = torch.from_numpy(X.astype(dtype)).to("cuda:0")
    f = S.Forest(ctx, Xd, torch.from_numpy(y).to("cuda:0"), C, ro, torch.from_numpy(ri).to("cuda:0"),
                 k=k, z=z, seed=seed + 7, bins=bins, sort_threshold=T, max_depth=max_depth, sampler=sampler,
                 weights=weights, first_tree=first_tree, **modes)
    if stats:
        sizes, units = [], []
        while True:
            nn, ns, depth = f.frontier_stats()
            if nn == 0:
                break
            assert depth == len(sizes), f"frontier depth {depth} at level {len(sizes)}"
            sizes.append(nn)
            units.append(ns * k)
            f.grow_level(graph)
        assert units == ref_units.tolist(), f"level units {units} vs {ref_units.tolist()}"
    else:
        sizes = f.grow(use_graph=graph)
    got = f.export()
    torch.cuda.synchronize()
    assert sizes == ref_levels.tolist(), f"frontier sizes {sizes} vs {ref_levels.tolist()}"
    assert len(got) == len(ref)
    for fld in ref.dtype.names:
        if fld == "gain":
            g, r = got["gain"], ref["gain"]
            assert np.all((r == 0) == (g == 0)), "gain zero pattern"
            assert np.all(np.abs(g - r) <= 1e-6 * np.abs(r)), "gain beyond 1e-6 relative"
        else:
            bad = np.nonzero(np.any((got[fld] != ref[fld]).reshape(len(ref), -1), axis=1))[0]
            assert bad.size == 0, f"field {fld} differs at node {bad[0]}: {got[bad[0]]} vs {ref[bad[0]]}"
    f.close()
    return got


def test_grow_three_trees_graph(ctx):
    grow_case(ctx, seed=51, d=10, n=400, C=3, trees=3, k=6, z=2, bins=64, T=50, graph=True)


def test_grow_three_trees_no_graph(ctx):
    grow_case(ctx, seed=51, d=10, n=400, C=3, trees=3, k=6, z=2, bins=64, T=50, graph=False)


def test_grow_frontier_stats_per_level(ctx):
    """Nodes, samples and depth of every frontier, read before each level,
    against the oracle's per-level node counts and projection units."""
    grow_case(ctx, seed=52, d=12, n=1500, C=4, trees=4, k=8, z=3, bins=128, T=64, stats=True)


def test_grow_histogram_only_depth_cap(ctx):
    got = grow_case(ctx, seed=3, d=12, n=3000, C=2, trees=2, k=8, z=3, bins=256, T=0, max_depth=5)
    assert got["depth"].max() <= 5


def test_grow_sort_only_four_classes(ctx):
    grow_case(ctx, seed=4, d=10, n=500, C=4, trees=2, k=4, z=3, bins=128, T=10**9)


def test_grow_fp16_storage_equals_oracle(ctx):
    grow_case(ctx, seed=6, d=16, n=2000, C=3, trees=2, k=8, z=4, bins=256, T=100, dtype=np.float16)


# The paper's sampler: each feature enters a projection with probability z/d
# (so some projections are empty), FP32 weights uniform on (-1, 1) or +/-1.
@pytest.mark.parametrize("weights", [1, 0])
def test_grow_density_sampler(ctx, weights):
    grow_case(ctx, seed=61, d=40, n=3000, C=3, trees=3, k=8, z=2, bins=128, T=300, graph=True,
              sampler=1, weights=weights)


def test_grow_density_sampler_fp16_no_graph(ctx):
    grow_case(ctx, seed=62, d=24, n=2500, C=2, trees=2, k=6, z=3, bins=256, T=0, graph=False,
              dtype=np.float16, sampler=1, weights=1)


def test_grow_tree_ids_from_first_tree(ctx):
    """Tree ids first_tree .. first_tree + n_trees - 1 key the sampler; the
    per-tree frontier bookkeeping is indexed by the local tree index."""
    grow_case(ctx, seed=53, d=12, n=600, C=3, trees=3, k=6, z=2, bins=64, T=40, first_tree=1000)


def test_grow_many_trees(ctx):
    """More trees than a block has threads (257+): every tree's start in the
    next frontier is written at every level."""
    grow_case(ctx, seed=54, d=8, n=60, C=2, trees=300, k=3, z=2, bins=32, T=20, first_tree=7)


# Roots above 8192 samples, so that the big-node passes (range, value cache,
# histogram, scan), the larger mid-node instance and the chunked partition all
# run under drawn projections.
@pytest.mark.parametrize("sampler,z,dtype", [(0, 3, np.float32), (1, 2, np.float32), (0, 5, np.float16)])
def test_grow_big_roots(ctx, sampler, z, dtype):
    grow_case(ctx, seed=55 + z, d=64, n=40000, C=3, trees=2, k=8, z=z, bins=256, T=200, max_depth=8,
              dtype=dtype, sampler=sampler, weights=sampler)


def tree_nodes(nodes, tree):
    """Nodes of one tree in the forest's order, with their parent/child ids
    renumbered to positions within that tree."""
    keep = np.nonzero(nodes["tree"] == tree)[0]
    pos = np.full(len(nodes), -1, np.int64)
    pos[keep] = np.arange(keep.size)
    t = nodes[keep].copy()
    for f in ("parent", "left", "right"):
        v = t[f].astype(np.int64)
        t[f] = np.where(v >= 0, pos[np.clip(v, 0, len(nodes) - 1)], -1)
    return t


def test_full_training_tree0_against_oracle(ctx):
    """The full-training workload (8 trees from 2M-row bootstrap roots of a
    2M x 1024 matrix, k = 128 drawn projections of 3 nonzeros, 256 bins,
    autotuned switch), grown to depth 20 on the GPU; tree 0 against the
    oracle's growth of that tree alone, record by record."""
    import torch
    from paper_2603_00326_amd import sof as S
    from paper_2603_00326_amd import workloads as W
    X, y, C, ro, ri = W.config4_data()
    k, z, bins, seed, depth = 128, 3, 256, 4, 20
    Xd = torch.from_numpy(X).to("cuda:0")
    yd = torch.from_numpy(y).to("cuda:0")
    T = int(S.autotune(ctx, C, k, z, bins, data=(Xd, yd, C))["sort_threshold"])
    say(f"[gpu] full training 8 trees x {X.shape[1]} rows, d={X.shape[0]}, k={k}, T={T}, depth {depth}")
    f = S.Forest(ctx, Xd, yd, C, ro, torch.from_numpy(ri).to("cuda:0"),
                 k=k, z=z, seed=seed, bins=bins, sort_threshold=T, max_depth=depth)
    f.grow(use_graph=True)
    got = tree_nodes(f.export(), 0)
    f.close()
    del Xd
    torch.cuda.empty_cache()
    ref, _, _ = O.grow_forest(X, y, C, ro[:2], ri[:int(ro[1])], k=k, z=z, seed=seed, bins=bins,
                              sort_threshold=T, max_depth=depth)
    say(f"[gpu] tree 0: {len(got)} GPU nodes, {len(ref)} oracle nodes")
    assert len(got) == len(ref)
    for fld in ref.dtype.names:
        if fld == "gain":
            g, r = got["gain"], ref["gain"]
            assert np.all((r == 0) == (g == 0)), "gain zero pattern"
            assert np.all(np.abs(g - r) <= 1e-6 * np.abs(r)), "gain beyond 1e-6 relative"
        else:
            bad = np.nonzero(np.any((got[fld] != ref[fld]).reshape(len(ref), -1), axis=1))[0]
            assert bad.size == 0, f"field {fld} differs at node {bad[0]}: {got[bad[0]]} vs {ref[bad[0]]}"


# ---------------------------------------------------------------------------
# growth under the entropy criterion and with random-width bins (keyed by
# tree position), on every path: sort below T, small/mid histograms, and
# roots above 8192 samples (big-node passes)

@pytest.mark.parametrize("criterion,bin_mode,T,graph", [(1, 0, 50, True), (1, 0, 0, False), (0, 1, 50, True),
                                                        (1, 1, 30, False), (1, 0, 2**31 - 1, True)])
def test_grow_entropy_and_random_width_bins(ctx, criterion, bin_mode, T, graph):
    grow_case(ctx, seed=57, d=10, n=600, C=3, trees=3, k=6, z=2, bins=64, T=T, graph=graph,
              criterion=criterion, bin_mode=bin_mode, bin_seed=1234)


@pytest.mark.parametrize("criterion,bin_mode,dtype", [(1, 0, np.float32), (0, 1, np.float16), (1, 1, np.float32)])
def test_grow_entropy_and_random_width_big_roots(ctx, criterion, bin_mode, dtype):
    grow_case(ctx, seed=58, d=16, n=20000, C=2, trees=2, k=8, z=3, bins=256, T=40, max_depth=4, graph=True,
              dtype=dtype, criterion=criterion, bin_mode=bin_mode, bin_seed=77)


def test_grow_density_sampler_entropy_random_width(ctx):
    grow_case(ctx, seed=59, d=24, n=800, C=4, trees=2, k=6, z=3, bins=128, T=60, graph=True, sampler=1,
              weights=1, criterion=1, bin_mode=1, bin_seed=5)


# Roots of 140000 samples (18 chunks): the XCD-local item order of the
# big-node passes under drawn projections, with entropy, random-width bins
# and FP16 storage.
@pytest.mark.parametrize("criterion,bin_mode,dtype", [(1, 0, np.float32), (0, 1, np.float32), (0, 0, np.float16)])
def test_grow_xcd_layout_roots(ctx, criterion, bin_mode, dtype):
    grow_case(ctx, seed=60, d=12, n=140000, C=3, trees=2, k=6, z=3, bins=256, T=40, max_depth=3, graph=True,
              dtype=dtype, criterion=criterion, bin_mode=bin_mode, bin_seed=9)
