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
              stats=False, sampler=0, weights=0):
    import torch
    from paper_2603_00326_amd import sof as S
    say(f"[gpu] grow seed={seed} d={d} n={n} C={C} trees={trees} k={k} z={z} B={bins} T={T} "
        f"max_depth={max_depth} graph={graph} dtype={np.dtype(dtype).name} sampler={sampler} weights={weights}")
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
                                               weights=weights)
    Xd = torch.from_numpy(X.astype(dtype)).to("cuda:0")
    f = S.Forest(ctx, Xd, torch.from_numpy(y).to("cuda:0"), C, ro, torch.from_numpy(ri).to("cuda:0"),
                 k=k, z=z, seed=seed + 7, bins=bins, sort_threshold=T, max_depth=max_depth, sampler=sampler,
                 weights=weights)
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
