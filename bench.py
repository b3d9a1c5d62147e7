#!/usr/bin/env python3
"""Split-search benchmark on one GPU.

One step is the whole hot path over one frontier: the batched split search
(projection, node range, histogram or sort, Gini scan and argmax; paper
section 4, steps 1-3) followed by the stable partition of every node's
samples.  Inputs are seeded and synthetic and are resident in device memory
before the timed region starts.

Prints one JSON line:
  value            node-sample x projection per second of the whole step
  roofline         the whole batched split search (one find_splits call):
                   algorithmic bytes per call over its mean duration (HIP
                   events recorded on the launch stream inside the timed
                   region), against 8 TB/s of HBM; the slowest data kernel's
                   figure sits beside it (dominant_kernel)
  cpu_baseline     the CPU oracle on the same frontier (or a bounded sample)
  plain_per_node   the same library called once per node from a host loop
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SORT_LIMIT = 8192
WAVE_SORT_MAX, SMALL_MAX, MID_SPLIT, MID_MAX = 64, 512, 4096, 8192

WORKLOADS = {
    "c3a": "batched frontier, 4096 log-normal nodes (median 300, 2..100000, ~4.0M samples) over a "
           "4.0M x 512 FP32 matrix, node rows contiguous, 3 classes, k=64, z=4, B=256",
    "c3b": "as c3a, each node's rows an ascending random subset of the matrix",
    "c3a_rw": "as c3a with random-width bins (boundaries at random-width intervals, two-level routing)",
    "c3a_ent": "as c3a with the entropy criterion (information gain, binary64), histogram path at every node",
    "c2": "single root node, n=1048576, d=256 FP32, 2 classes, k=256, z=3, B=256, histogram path",
    "c5": "single root node, n=10M, d=128 FP16 on the 1/256 grid, 2 classes, k=128, z=1..8, B=256",
    "c5f32": "as c5 with the same values stored FP32",
    "c1": "single root node, n=4096, d=64 FP32, 2 classes, k=64, z=3, B=256",
    "c4": "full training: 8 trees grown to purity level by level from bootstrap roots of a 2M x 1024 FP32 "
          "matrix (90% zeros), 4 classes, k=128, z=3 from the device sampler, B=256, max depth 64",
    "c4p": "as c4 with the paper's projection sampler: k = 1.5 sqrt(d) = 48 projections per node, each "
           "feature kept with probability 2/d (3 sqrt(d) nonzeros per node on average, Binomial counts, "
           "empty projections included), FP32 weights uniform on (-1, 1)",
    "accuracy": "held-out accuracy of 32-tree forests grown with exact splits, histograms and the dynamic "
                "switch on config 1's rule (4096 training rows, 100000 test rows, d=64, 10% label noise)",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name: str):
    from paper_2603_00326_amd import workloads as W
    if name == "c3a":
        return W.config3("a")
    if name == "c3b":
        return W.config3("b")
    if name == "c3a_rw":
        wl = W.config3("a")
        wl.meta.update(bin_mode=1, bin_seed=20260302)
        return wl
    if name == "c3a_ent":
        wl = W.config3("a")
        wl.meta.update(criterion=1)
        return wl
    if name == "c2":
        return W.config2()
    if name == "c5":
        return W.config5(fp16=True)
    if name == "c5f32":
        return W.config5(fp16=False)
    if name == "c1":
        return W.config1()
    raise SystemExit(f"unknown workload {name}; choose from {sorted(WORKLOADS)}")


# ---------------------------------------------------------------------------
# algorithmic bytes per kernel (each projection gathers its own z columns over
# the node's samples; sample indices and labels are read once per node)

def node_classes(wl, T: int):
    """Size class of every node as the library classifies it: 'none' (no
    projections), 'small', 'mid', 'mid2', 'sort', 'big'."""
    n = np.diff(wl.node_offsets.astype(np.int64))
    k = np.diff(wl.proj_offsets.astype(np.int64))
    Te = min(int(T), SORT_LIMIT + 1)
    sortp = n < Te
    cls = np.full(len(n), "big", dtype=object)
    cls[~sortp & (n <= MID_MAX)] = "mid2"
    cls[~sortp & (n <= MID_SPLIT)] = "mid"
    cls[~sortp & (n <= SMALL_MAX)] = "small"
    cls[sortp] = "sort"
    cls[sortp & (n <= WAVE_SORT_MAX)] = "small"
    cls[k == 0] = "none"
    return n, k, cls


def stage_bytes(wl, T: int):
    """Algorithmic bytes of each stage of one find-splits call."""
    n, k, cls = node_classes(wl, T)
    sx = wl.X.dtype.itemsize
    zsum = np.add.reduceat(np.diff(wl.nz_offsets.astype(np.int64)), wl.proj_offsets[:-1].astype(np.int64)) \
        if wl.n_proj else np.zeros(len(n), np.int64)
    zsum = np.where(k > 0, zsum, 0)
    cols = n * zsum * sx          # sum over the node's projections of n * z_p * s_x
    idx_lab = n * (4 + 4)
    out = {}
    for name, c in (("small", "small"), ("mid", "mid"), ("mid2", "mid2"), ("sort", "sort")):
        m = cls == c
        out[name] = float((idx_lab[m] + cols[m]).sum())
    m = cls == "big"
    out["big_range"] = float((n[m] * 4 + cols[m]).sum())
    out["big_hist"] = float((idx_lab[m] + cols[m]).sum())
    out["find"] = float((idx_lab[cls != "none"] + cols[cls != "none"]).sum())
    return out


def bmin_bytes(wl, T: int) -> float:
    """The floor of the split search's HBM bytes when every distinct (sample,
    feature) cell a node uses is read once, whatever number of its
    projections share the feature: n (s_i + s_y) + n |distinct features| s_x."""
    n, k, cls = node_classes(wl, T)
    sx = wl.X.dtype.itemsize
    po = wl.proj_offsets.astype(np.int64)
    zo = wl.nz_offsets.astype(np.int64)
    total = 0
    for v in np.nonzero(cls != "none")[0]:
        f = wl.nz_feature[zo[po[v]]:zo[po[v + 1]]]
        total += int(n[v]) * (8 + np.unique(f).size * sx)
    return float(total)


def partition_bytes(wl, splits):
    """Algorithmic bytes of the partition: n (z_{p*} s_x + 2 s_i) per split node."""
    n = np.diff(wl.node_offsets.astype(np.int64))
    po = wl.proj_offsets.astype(np.int64)
    zo = wl.nz_offsets.astype(np.int64)
    sx = wl.X.dtype.itemsize
    total = 0
    for v in np.nonzero(splits["proj"] >= 0)[0]:
        q = po[v] + splits["proj"][v]
        total += n[v] * ((zo[q + 1] - zo[q]) * sx + 8)
    return float(total)


# ---------------------------------------------------------------------------
# measured HBM traffic of a kernel (rocprofv3 FETCH_SIZE / WRITE_SIZE, per
# dispatch, scaled by a device-copy calibration), from the committed profile
# summary; None when the kernel source changed since the counters were taken

def measured_traffic(kernel: str, workload: str):
    import hashlib
    src = os.path.join(ROOT, "paper_2603_00326_amd", "csrc", "k_find.hip")
    prof = os.path.join(ROOT, "profiles", f"find_{workload}_profile.md")
    if not os.path.exists(prof) or not os.path.exists(src):
        return None
    md5 = hashlib.md5(open(src, "rb").read()).hexdigest()
    for line in open(prof):
        parts = line.split()
        if not parts or parts[0] != "traffic":
            continue
        kv = dict(p.split("=", 1) for p in parts[1:] if "=" in p)
        if kv.get("kernel") == kernel and kv.get("workload") == workload and kv.get("source_md5") == md5:
            return (float(kv["fetch_kib"]) * float(kv["fetch_scale"]) +
                    float(kv["write_kib"]) * float(kv["write_scale"])) * 1024.0
    return None


# ---------------------------------------------------------------------------
# the CPU oracle on a bounded sample of the same frontier

def cpu_baseline(wl, T, budget_units: float):
    from oracle import oracle as O
    from paper_2603_00326_amd import workloads as W
    O.lib()
    units_all = wl.units
    if units_all <= budget_units:
        sample, nodes = wl, None
        desc = "whole frontier, one oracle call (find splits + partition)"
    else:
        rng = np.random.default_rng(12345)
        order = rng.permutation(wl.n_nodes)
        n = np.diff(wl.node_offsets.astype(np.int64))
        k = np.diff(wl.proj_offsets.astype(np.int64))
        acc, nodes = 0, []
        for v in order:
            nodes.append(int(v))
            acc += int(n[v] * k[v])
            if acc >= budget_units:
                break
        nodes.sort()
        sample = W.sub_frontier(wl, nodes)
        desc = (f"{len(nodes)} of {wl.n_nodes} nodes drawn uniformly (seed 12345), "
                f"{sample.units} of {units_all} units, find splits + partition")
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()

    def once(nt):
        t0 = time.perf_counter()
        ref, _ = O.find_splits(sample.X, sample.y, sample.n_classes, sample.node_offsets, sample.sample_idx,
                               sample.proj_offsets, sample.nz_offsets, sample.nz_feature, sample.nz_weight,
                               bins=sample.bins, sort_threshold=T, node_bins=sample.node_bins, threads=nt,
                               bin_mode=int(wl.meta.get("bin_mode", 0)),
                               bin_seed=int(wl.meta.get("bin_seed", 0)),
                               criterion=int(wl.meta.get("criterion", 0)))
        O.partition(sample.X, sample.node_offsets, sample.sample_idx, sample.proj_offsets, sample.nz_offsets,
                    sample.nz_feature, sample.nz_weight, ref, bins=sample.bins, node_bins=sample.node_bins)
        return time.perf_counter() - t0

    runs = [once(threads)]
    while len(runs) < 5 and sum(runs) < 20.0:
        runs.append(once(threads))
    el = float(np.median(runs))
    out = {"value": sample.units / el, "unit": "node-sample*projection/s", "cores": threads,
           "kind": "oracle", "sample": desc, "seconds": round(el, 3), "runs": len(runs),
           "cpu_model": cpu_model()}
    if el * threads <= 40.0:
        one = once(1)
        out["single_thread"] = {"value": sample.units / one, "seconds": round(one, 3)}
    return out


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ---------------------------------------------------------------------------
# the plain form: one single-node call per node from a host loop

class PlainForm:
    """Per-node frontiers over views of the batched device arrays."""

    def __init__(self, ctx, dev, wl, T):
        import torch
        from paper_2603_00326_amd import sof as S
        self.S, self.ctx, self.T = S, ctx, T
        no = wl.node_offsets.astype(np.int64)
        po = wl.proj_offsets.astype(np.int64)
        zo = wl.nz_offsets.astype(np.int64)
        dv = dev.X.device
        self.items = []
        self.keep = []
        max_ws = 0
        for v in range(wl.n_nodes):
            n, k = int(no[v + 1] - no[v]), int(po[v + 1] - po[v])
            z0 = int(zo[po[v]])
            offs = torch.tensor([0, n], dtype=torch.int32, device=dv)
            pof = torch.tensor([0, k], dtype=torch.int32, device=dv)
            zof = torch.from_numpy((zo[po[v]:po[v + 1] + 1] - z0).astype(np.int32)).to(dv)
            nb = None if dev.node_bins is None else dev.node_bins[v:v + 1]
            f = S.DeviceFrontier(X=dev.X, y=dev.y, n_classes=dev.n_classes, node_offsets=offs,
                                 sample_idx=dev.sample_idx[no[v]:no[v + 1]], proj_offsets=pof,
                                 nz_offsets=zof, nz_feature=dev.nz_feature[z0:],
                                 nz_weight=dev.nz_weight[z0:], node_bins=nb, max_node_samples=n,
                                 max_proj_per_node=k)
            out = torch.empty((1, 10), dtype=torch.int32, device=dv)
            oidx = torch.empty(max(n, 1), dtype=torch.int32, device=dv)
            coff = torch.empty(3, dtype=torch.int32, device=dv)
            d, fr, p = f.structs()
            q = S.sof_params(S._ptr(nb), int(wl.bins), int(T), int(wl.meta.get("bin_mode", 0)),
                             int(wl.meta.get("criterion", 0)), int(wl.meta.get("bin_seed", 0)))
            sz = ctypes.c_size_t(0)
            S._check(S.lib().sof_workspace_size(ctx.handle, ctypes.byref(d), ctypes.byref(fr), ctypes.byref(p),
                                                ctypes.byref(q), ctypes.byref(sz)))
            max_ws = max(max_ws, sz.value)
            self.items.append((d, fr, p, q, out, oidx, coff))
            self.keep.append((f, out, oidx, coff, nb))
        self.ws, self.wsb = ctx.workspace(max_ws)

    def step(self, stream):
        S, L = self.S, self.S.lib()
        h = self.ctx.handle
        for d, fr, p, q, out, oidx, coff in self.items:
            S._check(L.sof_find_splits(h, ctypes.byref(d), ctypes.byref(fr), ctypes.byref(p), ctypes.byref(q),
                                       out.data_ptr(), None, self.ws, self.wsb, stream))
            S._check(L.sof_partition(h, ctypes.byref(d), ctypes.byref(fr), ctypes.byref(p), ctypes.byref(q),
                                     out.data_ptr(), oidx.data_ptr(), coff.data_ptr(), self.ws, self.wsb,
                                     stream))


# ---------------------------------------------------------------------------
# full training: level-wise growth of a forest

def run_growth(args, S, ctx):
    """One step grows every tree of the forest to purity (or the depth cap):
    per level, device projection sampling, batched split search, partition,
    leaf detection and node records, replayed from a captured HIP graph."""
    import torch
    from paper_2603_00326_amd import workloads as W
    t0 = time.perf_counter()
    X, y, C, ro, ri = W.config4_data()
    k, z, bins, max_depth, seed = 128, 3, 256, 64, 4
    sampler, weights = S.SOF_SAMPLER_FIXED, S.SOF_WEIGHTS_SIGN
    if args.workload == "c4p":
        k, z = 48, 2          # 1.5 sqrt(1024) projections, 3 sqrt(1024) / k nonzeros each on average
        sampler, weights = S.SOF_SAMPLER_DENSITY, S.SOF_WEIGHTS_UNIFORM
    log(f"[bench] c4 data {X.shape[1]} x {X.shape[0]}, {len(ro) - 1} trees, {ri.size} root samples "
        f"(generated in {time.perf_counter() - t0:.1f}s)")
    dev_name = "cuda:0"
    Xd = torch.from_numpy(X).to(dev_name)
    yd = torch.from_numpy(y).to(dev_name)
    rid = torch.from_numpy(ri).to(dev_name)
    torch.cuda.synchronize()
    T, tune = args.threshold, None
    if T is None:
        tune = S.autotune(ctx, C, k, z, bins, data=(Xd, yd, C))
        T = int(tune["sort_threshold"])
    log(f"[bench] sort threshold T={T}")
    stream = torch.cuda.current_stream()
    sx = 4

    def grow_once(timed):
        f = S.Forest(ctx, Xd, yd, C, ro, rid, k=k, z=z, seed=seed, bins=bins, sort_threshold=T,
                     max_depth=max_depth, sampler=sampler, weights=weights)
        torch.cuda.synchronize()
        levels, evs = [], []
        t_start = time.perf_counter()
        while True:
            nn, ns, depth = f.frontier_stats()
            if nn == 0:
                break
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            f.grow_level(True)
            e1.record(stream)
            levels.append((depth, nn, ns))
            evs.append((e0, e1))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        nodes = f.export() if timed else None
        pred = None
        if timed:
            nd = S.nodes_to_device(nodes, dev_name)
            rt = torch.arange(len(ro) - 1, dtype=torch.int32, device=dev_name)
            S.predict(ctx, Xd, nd, rt, C, votes=False)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            _, P = S.predict(ctx, Xd, nd, rt, C, votes=False)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            pred = {"rows": int(X.shape[1]), "trees": len(ro) - 1, "ms": round(ms, 3),
                    "row_trees_per_s": X.shape[1] * (len(ro) - 1) / (ms * 1e-3),
                    "training_accuracy": float((P.cpu().numpy() == y).mean())}
        f.close()
        return wall, levels, [a.elapsed_time(b) for a, b in evs], (nodes, pred)

    for _ in range(args.warmup):
        grow_once(False)
    walls, last = [], None
    for _ in range(args.steps):
        wall, levels, lms, nodes = grow_once(True)
        walls.append(wall)
        last = (levels, lms, nodes)
    levels, lms, (nodes, pred_info) = last
    units = sum(ns * k for _, _, ns in levels)
    ms_per_step = float(np.mean(walls)) * 1e3
    # algorithmic bytes per level: the split search reads each sample's index,
    # label and k*z feature values; the partition re-reads z values and moves
    # two indices per sample of every split node (z: the law's mean count for
    # the density sampler)
    internal = nodes[nodes["is_leaf"] == 0]
    rows, tot_b, tot_ms = [], 0.0, 0.0
    for (depth, nn, ns), ms in zip(levels, lms):
        split_n = int(internal["n_samples"][internal["depth"] == depth].astype(np.int64).sum())
        b = ns * (8 + k * z * sx) + split_n * (z * sx + 8)
        tot_b += b
        tot_ms += ms
        rows.append({"depth": depth, "nodes": nn, "samples": ns, "units": ns * k, "ms": round(ms, 4),
                     "GBs": round(b / (ms * 1e-3) / 1e9, 1) if ms > 0 else None})
    achieved = tot_b / (tot_ms * 1e-3) / 1e9 if tot_ms > 0 else 0.0
    result = {
        "metric": "split-search throughput: node-sample×projection/s + % of HBM roofline",
        "value": units / (ms_per_step * 1e-3),
        "unit": "node-sample*projection/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload], "trees": len(ro) - 1,
                   "root_samples": int(ri.size), "k": k, "z": z, "sampler": int(sampler), "weights": int(weights),
                   "bins": bins, "sort_threshold": T,
                   "max_depth": max_depth, "levels": len(levels), "nodes": int(len(nodes)),
                   "units": int(units), "step": "grow every tree to purity (one forest)"},
        "roofline": {"bound": "hbm", "kernel": "grow_level (every kernel of a level, summed over levels)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "bytes_per_launch": tot_b / max(len(levels), 1),
                     "ms_per_launch": round(tot_ms / max(len(levels), 1), 5)},
        "levels": rows,
        "level_ms_sum": round(tot_ms, 3),
        "predict": pred_info,
    }
    if tune:
        result["autotune"] = tune
    if not args.no_cpu:
        from oracle import oracle as O
        O.lib()
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
        D = min(args.cpu_depth, max_depth)
        log(f"[bench] CPU oracle baseline: tree 0 of the forest to depth {D}")
        t0 = time.perf_counter()
        _, _, lu = O.grow_forest(X, y, C, ro[:2], ri[:int(ro[1])], k=k, z=z, seed=seed, bins=bins,
                                 sort_threshold=T, max_depth=D, threads=threads, sampler=sampler, weights=weights)
        el = time.perf_counter() - t0
        top = [i for i, r in enumerate(rows) if r["depth"] < D]
        gpu_top = sum(rows[i]["units"] for i in top) / (sum(lms[i] for i in top) * 1e-3) if top else None
        result["cpu_baseline"] = {"value": float(lu.sum()) / el, "unit": "node-sample*projection/s",
                                  "cores": threads, "kind": "oracle",
                                  "sample": f"tree 0 of {len(ro) - 1}, levels 0..{D - 1} ({int(lu.sum())} units)",
                                  "seconds": round(el, 3),
                                  "gpu_same_levels": gpu_top}
    print(json.dumps(result), flush=True)


# ---------------------------------------------------------------------------
# accuracy of exact, histogram and dynamic forests (the paper finds the three
# statistically indistinguishable)

def run_accuracy(args, S, ctx):
    import torch
    from paper_2603_00326_amd import workloads as W
    X, y, Xt, yt = W.accuracy_data()
    C, trees, k, z, bins, n = 2, 32, 64, 3, 256, X.shape[1]
    dev_name = "cuda:0"
    Xd, yd, Xtd = (torch.from_numpy(a).to(dev_name) for a in (X, y, Xt))
    ri = np.concatenate([np.sort(np.random.default_rng(1000 + t).integers(0, n, n)) for t in range(trees)])
    rid = torch.from_numpy(ri.astype(np.int32)).to(dev_name)
    ro = np.arange(trees + 1, dtype=np.int64) * n
    tune = S.autotune(ctx, C, k, z, bins, data=(Xd, yd, C))
    out = {}
    # dynamic: the threshold this GPU's autotuner picks, and the paper's CPU breakeven (~1200 samples)
    for name, T in (("exact", 2**31 - 1), ("histogram", 0), ("dynamic", int(tune["sort_threshold"])),
                    ("dynamic_T1200", 1200)):
        f = S.Forest(ctx, Xd, yd, C, ro, rid, k=k, z=z, seed=11, bins=bins, sort_threshold=T, max_depth=64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f.grow()
        torch.cuda.synchronize()
        grow_ms = (time.perf_counter() - t0) * 1e3
        _, P = f.predict(Xtd, votes=False)
        nodes = len(f.export())
        f.close()
        acc = float((P.cpu().numpy() == yt).mean())
        out[name] = {"sort_threshold": T, "accuracy": round(acc, 5),
                     "stderr": round(float(np.sqrt(acc * (1 - acc) / len(yt))), 5),
                     "nodes": nodes, "grow_ms": round(grow_ms, 2)}
        log(f"[bench] {name}: T={T} accuracy {acc:.4f} ({nodes} nodes, {grow_ms:.1f} ms)")
    accs = [v["accuracy"] for v in out.values()]
    print(json.dumps({
        "metric": "held-out accuracy, exact vs histogram vs dynamic splits",
        "value": out["dynamic"]["accuracy"], "unit": "fraction correct", "n_gpus": 1,
        "higher_is_better": True, "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "accuracy", "description": WORKLOADS["accuracy"], "trees": trees, "k": k,
                   "z": z, "bins": bins, "train_rows": n, "test_rows": int(len(yt)),
                   "bayes_accuracy": 0.9},
        "forests": out, "max_difference": round(max(accs) - min(accs), 5)}), flush=True)


# ---------------------------------------------------------------------------

def graph_leg(step, out, steps):
    """The same step captured once into a HIP graph (the find's and the
    partition's forks onto the context's streams become graph branches) and
    replayed: every replay's split records and partition are checked against
    an eager step's, then `steps` replays are timed."""
    import torch
    idx_e, coff_e = step()
    torch.cuda.synchronize()
    ref = (out.clone(), idx_e.clone(), coff_e.clone())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        idx_g, coff_g = step()
    torch.cuda.synchronize()
    checked = 0
    for _ in range(3):
        out.fill_(-7)
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip((out, idx_g, coff_g), ref):
            if not torch.equal(a, b):
                raise RuntimeError("graph replay differs from the eager step")
        checked += 1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    del g
    return {"ms_per_step": round(ms, 4), "steps": steps, "replays_checked": checked,
            "note": "find_splits + partition captured once into one HIP graph and replayed"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3a", choices=sorted(WORKLOADS))
    ap.add_argument("--threshold", type=int, default=None,
                    help="sort/histogram switch T (default: the autotuner's choice)")
    ap.add_argument("--bins-switch", type=int, default=None,
                    help="config 3: nodes below this size take half the bins (default: the autotuner's "
                         "rule; 0 = full bins everywhere)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--small-max", type=int, default=None,
                    help="wave tile edge: nodes up to this size take a wave per projection (256..512; default tuned)")
    ap.add_argument("--mid-split", type=int, default=None,
                    help="wave tile edge: 16 samples per thread up to this size (2048..4096; default tuned)")
    ap.add_argument("--graph", type=int, default=1,
                    help="also time the step captured into one HIP graph and replayed")
    ap.add_argument("--project", type=int, default=1,
                    help="also time step 1 alone (sof_project) after the timed loop (0 skips it)")
    ap.add_argument("--plain", type=int, default=2,
                    help="steps of the per-node-launch form (0 skips it)")
    ap.add_argument("--cpu-units", type=float, default=3e9,
                    help="bound on the oracle sample, in node-sample*projection units")
    ap.add_argument("--cpu-depth", type=int, default=20,
                    help="c4: depth bound of the oracle's sample tree")
    ap.add_argument("--copy-only", type=float, default=0.0,
                    help="run only a plain device copy of this many GiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(the library has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2603_00326_amd import sof as S

    dev_name = "cuda:0"
    if args.copy_only > 0:
        n = int(args.copy_only * (1 << 30)) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev_name)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 3}))
        return

    if args.workload in ("c4", "c4p"):
        run_growth(args, S, S.Context(0))
        return
    if args.workload == "accuracy":
        run_accuracy(args, S, S.Context(0))
        return

    t0 = time.perf_counter()
    wl = make_workload(args.workload)
    log(f"[bench] workload {args.workload}: {wl.n_nodes} nodes, {wl.n_samples} samples, "
        f"{wl.n_proj} projections, units {wl.units} (generated in {time.perf_counter() - t0:.1f}s)")
    ctx = S.Context(0)
    dev = S.to_device(wl, dev_name)
    torch.cuda.synchronize()

    T = args.threshold
    tune = None
    per_node_bins = args.workload.startswith("c3")   # config 3: 128-256 bins per node
    if T is None or (per_node_bins and args.bins_switch is None):
        tune = S.autotune(ctx, wl.n_classes, int(wl.meta.get("k", 64)), int(wl.meta.get("z", 3)), wl.bins,
                          data=dev)
        if T is None:
            T = int(tune["sort_threshold"])
    if wl.meta.get("criterion", 0):
        T = 0   # the entropy criterion runs on the histogram path
    log(f"[bench] sort threshold T={T}" + (f" (autotuned in {tune['ms']:.1f} ms)" if tune else ""))
    bins_small, bins_switch = wl.bins, 0
    if per_node_bins:
        bins_small = tune["bins_small"] if tune else max(wl.bins // 2, 2)
        bins_switch = args.bins_switch if args.bins_switch is not None else tune["bins_switch"]
        if bins_switch > 0:
            n_v = np.diff(wl.node_offsets.astype(np.int64))
            wl.node_bins = np.where(n_v < bins_switch, bins_small, wl.bins).astype(np.int32)
            dev.node_bins = torch.from_numpy(wl.node_bins).to(dev_name)
        log(f"[bench] bins: {bins_small} below n={bins_switch}, else {wl.bins}")

    stream = torch.cuda.current_stream()
    out = torch.empty((max(wl.n_nodes, 1), 10), dtype=torch.int32, device=dev_name)

    # the wave tile edges the autotuner chose (0: the library's defaults)
    small_max = int(tune["small_max"]) if tune else 0
    mid_split = int(tune["mid_split"]) if tune else 0
    if args.small_max is not None:
        small_max = args.small_max
    if args.mid_split is not None:
        mid_split = args.mid_split
    bin_mode = int(wl.meta.get("bin_mode", 0))
    bin_seed = int(wl.meta.get("bin_seed", 0))
    criterion = int(wl.meta.get("criterion", 0))

    def step():
        S.find_splits(ctx, dev, bins=wl.bins, sort_threshold=T, out=out, bin_mode=bin_mode, bin_seed=bin_seed,
                      criterion=criterion, small_max=small_max, mid_split=mid_split)
        return S.partition(ctx, dev, out, bins=wl.bins)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # the timed calls record HIP events around each find_splits call only
    ctx.timing(True, whole=True)
    ctx.timing_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    whole_ms, calls = ctx.timing_read()
    ctx.timing(False)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = wl.units / (ms_per_step * 1e-3)
    # Stage figures, after the timed region (their 22 events per call cost
    # about 5% of a c3a step): a few calls with the events of every stage on
    # the streams that run it, then a few with the size classes serialised, so
    # that each stage's events bound its own kernels (with concurrent classes
    # a stage's events also span its wait for compute units).
    ctx.timing(True)
    ctx.timing_read()
    for _ in range(5):
        step()
    torch.cuda.synchronize()
    stage_ms, ccalls = ctx.timing_read()
    ctx.timing(False)
    ctx.timing(True, serial=True)
    ctx.timing_read()
    for _ in range(5):
        step()
    torch.cuda.synchronize()
    serial_ms, scalls = ctx.timing_read()
    ctx.timing(False)

    splits = S.splits_to_numpy(out)[:wl.n_nodes]
    sb = stage_bytes(wl, T)
    per = {k: v / max(ccalls, 1) for k, v in stage_ms.items()}
    per["total"] = whole_ms["total"] / max(calls, 1)   # the timed calls'
    sper = {k: v / max(scalls, 1) for k, v in serial_ms.items()}
    data_stages = ("big_range", "big_hist", "mid", "mid2", "small", "sort")
    dom = max(data_stages, key=lambda s: sper[s])
    kernel_name = {"big_range": "k_brange", "big_hist": "k_bhist", "mid": "k_mid", "mid2": "k_mid_large",
                   "small": "k_small", "sort": "k_sortblk"}[dom]
    achieved = sb[dom] / (sper[dom] * 1e-3) / 1e9 if sper[dom] > 0 else 0.0
    find_gbs = sb["find"] / (per["total"] * 1e-3) / 1e9 if per["total"] > 0 else 0.0
    # the headline is the whole batched split search (every kernel of one
    # find_splits call, between the events around it); the slowest data
    # kernel is reported beside it
    roof = {"bound": "hbm", "kernel": "find_splits (the whole batched launch sequence of one call)",
            "achieved": round(find_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(find_gbs / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic("find_splits", args.workload),
            "bytes_per_launch": sb["find"], "ms_per_launch": round(per["total"], 5),
            "dominant_kernel": {"kernel": kernel_name, "achieved": round(achieved, 1),
                                "frac": round(achieved / HBM_PEAK_GBS, 4),
                                "traffic": measured_traffic(kernel_name, args.workload),
                                "bytes_per_launch": sb[dom], "ms_per_launch": round(sper[dom], 5),
                                "timing": "5 calls after the timed region with the size classes serialised"}}
    bmin = bmin_bytes(wl, T)
    bmin_gbs = bmin / (per["total"] * 1e-3) / 1e9 if per["total"] > 0 else 0.0
    pb = partition_bytes(wl, splits)

    result = {
        "metric": "split-search throughput: node-sample×projection/s + % of HBM roofline",
        "value": value,
        "unit": "node-sample*projection/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16" if wl.X.dtype == np.float16 else "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload],
                   "nodes": wl.n_nodes, "samples": int(wl.n_samples), "units": int(wl.units),
                   "sort_threshold": T, "bins": wl.bins,
                   "bins_small": int(bins_small) if bins_switch > 0 else None,
                   "bins_switch": int(bins_switch),
                   "wave_tile": {"small_max": small_max or 512, "mid_split": mid_split or 4096},
                   "bin_layout": "random width" if bin_mode else "equal width",
                   "criterion": "entropy" if criterion else "gini",
                   "step": "find_splits + partition"},
        "roofline": roof,
        "find_splits": {"ms": round(per["total"], 4), "algorithmic_bytes": sb["find"],
                        "achieved_GBs": round(find_gbs, 1), "frac": round(find_gbs / HBM_PEAK_GBS, 4),
                        "bmin_bytes": bmin, "bmin_GBs": round(bmin_gbs, 1),
                        "bmin_frac": round(bmin_gbs / HBM_PEAK_GBS, 4),
                        "stage_ms": {k: round(v, 4) for k, v in per.items()},
                        "stage_ms_note": "stages: 5 calls after the timed region (concurrent classes); "
                                         "total: the timed calls",
                        "stage_ms_serialised": {k: round(v, 4) for k, v in sper.items()},
                        "stage_bytes": sb},
        "partition": {"algorithmic_bytes": pb},
    }
    if tune:
        result["autotune"] = tune

    if args.graph:
        result["graph_step"] = graph_leg(step, out, args.steps)

    if args.project:
        # step 1 alone through sof_project: every (node, projection, sample)
        # value written out, [projection][sample] per node
        n_v = np.diff(wl.node_offsets.astype(np.int64))
        k_v = np.diff(wl.proj_offsets.astype(np.int64))
        S.project(ctx, dev)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 5
        e0.record(stream)
        for _ in range(reps):
            S.project(ctx, dev)
        e1.record(stream)
        torch.cuda.synchronize()
        pms = e0.elapsed_time(e1) / reps
        sx = wl.X.dtype.itemsize
        zsum = np.add.reduceat(np.diff(wl.nz_offsets.astype(np.int64)), wl.proj_offsets[:-1].astype(np.int64)) \
            if wl.n_proj else np.zeros(len(n_v), np.int64)
        pbytes = float((n_v * (4 + np.where(k_v > 0, zsum, 0) * sx + 4 * k_v)).sum())
        result["project"] = {"ms": round(pms, 4), "units_per_s": wl.units / (pms * 1e-3),
                             "algorithmic_bytes": pbytes,
                             "achieved_GBs": round(pbytes / (pms * 1e-3) / 1e9, 1),
                             "frac": round(pbytes / (pms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                             "note": "sof_project alone: sample ids read once per node, z columns gathered and "
                                     "one FP32 value written per (node, projection, sample)"}

    if args.plain > 0:
        log(f"[bench] plain per-node form: {wl.n_nodes} single-node calls per step")
        pf = PlainForm(ctx, dev, wl, T)
        pf.step(stream.cuda_stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.plain):
            pf.step(stream.cuda_stream)
        torch.cuda.synchronize()
        pms = (time.perf_counter() - t0) * 1e3 / args.plain
        result["plain_per_node"] = {"value": wl.units / (pms * 1e-3), "ms_per_step": round(pms, 3),
                                    "steps": args.plain, "speedup_of_batched": round(pms / ms_per_step, 2)}

    if not args.no_cpu:
        log("[bench] CPU oracle baseline")
        result["cpu_baseline"] = cpu_baseline(wl, T, args.cpu_units)

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
