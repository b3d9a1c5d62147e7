"""Python binding of libsof (the C ABI in include/sof.h).

Argument marshalling only: every step of the split search runs in the HIP
kernels of libsof.so.  PyTorch supplies device memory (tensors) and streams.
The binding raises if the library is missing; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsof.so")

SOF_OK = 0
SOF_ERR_INVALID_ARG = -1
SOF_ERR_UNSUPPORTED = -2
SOF_ERR_WORKSPACE = -3
SOF_ERR_OVERFLOW = -4
SOF_ERR_HIP = -5
SOF_ERR_DEVICE = -6
SOF_F32, SOF_F16 = 0, 1
SOF_BINS_EQUAL, SOF_BINS_RANDOM = 0, 1
SOF_CRIT_GINI, SOF_CRIT_ENTROPY = 0, 1
SOF_SPLIT_HIST, SOF_SPLIT_SORT, SOF_SPLIT_RHIST = 0, 1, 2
SOF_SAMPLER_FIXED, SOF_SAMPLER_DENSITY = 0, 1
SOF_WEIGHTS_SIGN, SOF_WEIGHTS_UNIFORM = 0, 1
SORT_LIMIT = 8192
INT32_MAX = 2**31 - 1

EXPORTED = [
    "sof_version", "sof_last_error", "sof_create", "sof_destroy", "sof_workspace_size",
    "sof_project", "sof_find_splits", "sof_partition", "sof_forest_create", "sof_forest_destroy",
    "sof_grow_level", "sof_forest_frontier_size", "sof_forest_frontier_stats", "sof_forest_export",
    "sof_autotune", "sof_predict",
    "sof_timing_enable", "sof_timing_read", "sof_find_splits_noalloc", "sof_autotune_on",
]


class SofError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libsof error {code}: {msg}")
        self.code = code


P = ctypes.c_void_p
i32, i64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64


class sof_data(ctypes.Structure):
    _fields_ = [("x", P), ("y", P), ("ld", i64), ("n_rows", i32), ("n_features", i32),
                ("n_classes", i32), ("dtype", i32)]


class sof_frontier(ctypes.Structure):
    _fields_ = [("node_offsets", P), ("sample_idx", P), ("n_samples", i64), ("n_nodes", i32),
                ("max_node_samples", i32)]


class sof_proj(ctypes.Structure):
    _fields_ = [("proj_offsets", P), ("nz_offsets", P), ("nz_feature", P), ("nz_weight", P),
                ("n_nz", i64), ("n_proj", i32), ("max_proj_per_node", i32), ("nz_value", P)]


class sof_params(ctypes.Structure):
    _fields_ = [("node_bins", P), ("bins", i32), ("sort_threshold", i32), ("bin_mode", i32), ("criterion", i32),
                ("bin_seed", u64), ("small_max", i32), ("mid_split", i32)]


class sof_forest_desc(ctypes.Structure):
    _fields_ = [("root_offsets", P), ("root_idx", P), ("seed", u64), ("n_trees", i32),
                ("first_tree", i32), ("k", i32), ("z", i32), ("bins", i32), ("sort_threshold", i32),
                ("max_depth", i32), ("sampler", i32), ("weights", i32), ("criterion", i32), ("bin_mode", i32),
                ("pad", i32), ("bin_seed", u64)]


class sof_tune(ctypes.Structure):
    _fields_ = [("sort_threshold", i32), ("bins_small", i32), ("bins_switch", i32), ("n_points", i32),
                ("sort_us", ctypes.c_float * 32), ("hist_us", ctypes.c_float * 32),
                ("sizes", i32 * 32), ("elapsed_ms", ctypes.c_float), ("half_us", ctypes.c_float * 32),
                ("small_max", i32), ("mid_split", i32), ("tile_base_us", ctypes.c_float * 32),
                ("tile_us", ctypes.c_float * 32)]


SPLIT_DTYPE = np.dtype([
    ("proj", "<i4"), ("kind", "<i4"), ("bin", "<i4"), ("threshold", "<f4"), ("lo", "<f4"),
    ("scale", "<f4"), ("n_left", "<i4"), ("n_right", "<i4"), ("flags", "<i4"), ("gain", "<f4"),
])
assert SPLIT_DTYPE.itemsize == 40

TREE_NODE_DTYPE = np.dtype([
    ("tree", "<i4"), ("depth", "<i4"), ("parent", "<i4"), ("left", "<i4"), ("right", "<i4"),
    ("n_samples", "<i4"), ("label", "<i4"), ("is_leaf", "<i4"), ("kind", "<i4"), ("bin", "<i4"),
    ("threshold", "<f4"), ("lo", "<f4"), ("scale", "<f4"), ("n_bins", "<i4"), ("nnz", "<i4"),
    ("pad", "<i4"), ("feature", "<i4", (16,)), ("weight", "<f4", (16,)), ("gain", "<f8"),
])
assert TREE_NODE_DTYPE.itemsize == 200

_lib = None


def lib():
    """Load libsof.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2603_00326_amd.build.build()")
        # PyTorch first: its wheel ships its own HIP runtime under the same
        # soname as the system one libsof.so links, so whichever loads first
        # serves both; loaded the other way round, torch finds no GPU
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        L.sof_version.restype = ctypes.c_char_p
        L.sof_last_error.restype = ctypes.c_char_p
        L.sof_create.argtypes = [ctypes.c_int, ctypes.POINTER(P)]
        L.sof_destroy.argtypes = [P]
        L.sof_workspace_size.argtypes = [P, ctypes.POINTER(sof_data), ctypes.POINTER(sof_frontier),
                                         ctypes.POINTER(sof_proj), ctypes.POINTER(sof_params),
                                         ctypes.POINTER(ctypes.c_size_t)]
        L.sof_project.argtypes = [P, ctypes.POINTER(sof_data), ctypes.POINTER(sof_frontier),
                                  ctypes.POINTER(sof_proj), P, P, ctypes.c_size_t, P]
        L.sof_find_splits.argtypes = [P, ctypes.POINTER(sof_data), ctypes.POINTER(sof_frontier),
                                      ctypes.POINTER(sof_proj), ctypes.POINTER(sof_params), P, P, P,
                                      ctypes.c_size_t, P]
        L.sof_find_splits_noalloc.argtypes = [P, ctypes.POINTER(sof_data), ctypes.POINTER(sof_frontier),
                                              ctypes.POINTER(sof_proj), ctypes.POINTER(sof_params), P, P, P]
        L.sof_partition.argtypes = [P, ctypes.POINTER(sof_data), ctypes.POINTER(sof_frontier),
                                    ctypes.POINTER(sof_proj), ctypes.POINTER(sof_params), P, P, P, P,
                                    ctypes.c_size_t, P]
        if hasattr(L, "sof_forest_create"):
            L.sof_forest_create.argtypes = [P, ctypes.POINTER(sof_data), ctypes.POINTER(sof_forest_desc),
                                            ctypes.POINTER(P)]
            L.sof_forest_destroy.argtypes = [P]
            L.sof_grow_level.argtypes = [P, ctypes.c_int, P]
            L.sof_forest_frontier_size.argtypes = [P, ctypes.POINTER(i64), P]
            L.sof_forest_frontier_stats.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                                    ctypes.POINTER(ctypes.c_int32), P]
            L.sof_forest_export.argtypes = [P, P, i64, ctypes.POINTER(i64), P]
        L.sof_timing_enable.argtypes = [P, ctypes.c_int]
        L.sof_timing_read.argtypes = [P, P, ctypes.POINTER(i32)]
        L.sof_predict.argtypes = [P, ctypes.POINTER(sof_data), P, i64, P, i32, P, P, P]
        L.sof_autotune.argtypes = [P, i32, i32, i32, i32, i32, ctypes.POINTER(sof_tune), P]
        L.sof_autotune_on.argtypes = [P, ctypes.POINTER(sof_data), i32, i32, i32, ctypes.POINTER(sof_tune), P]
        _lib = L
    return _lib


def _check(rc: int):
    if rc != SOF_OK:
        raise SofError(rc, lib().sof_last_error().decode())


def version() -> str:
    return lib().sof_version().decode()


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(stream) -> int | None:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


class Context:
    """A libsof context on one HIP device."""

    def __init__(self, device: int = 0):
        h = P()
        _check(lib().sof_create(int(device), ctypes.byref(h)))
        self.handle = h
        self.device = device
        self._ws = None

    def close(self):
        if self.handle:
            lib().sof_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def timing(self, enable, serial: bool = False, whole: bool = False):
        """Benchmark instrumentation: HIP events around each find_splits call
        and its stages; serial runs the size classes one after another so that
        each stage's events bound its own kernels; whole records only the
        events around the call."""
        _check(lib().sof_timing_enable(self.handle, 0 if not enable else (2 if serial else (3 if whole else 1))))

    STAGES = ("plan", "big_range", "big_merge", "big_hist", "big_scan", "mid", "mid2", "small", "sort",
              "reduce")

    def timing_read(self):
        """({stage: ms, ..., "total": ms}, calls) summed since the last read."""
        n = len(self.STAGES)
        ms = (ctypes.c_float * (n + 1))()
        calls = i32(0)
        _check(lib().sof_timing_read(self.handle, ctypes.cast(ms, P), ctypes.byref(calls)))
        out = {name: float(ms[i]) for i, name in enumerate(self.STAGES)}
        out["total"] = float(ms[n])
        return out, int(calls.value)

    def workspace(self, nbytes: int):
        """A cached device workspace of at least nbytes (256-byte aligned)."""
        import torch
        if self._ws is None or self._ws.numel() < nbytes + 256:
            self._ws = torch.empty(max(nbytes + 256, 1 << 16), dtype=torch.uint8,
                                   device=f"cuda:{self.device}")
        base = self._ws.data_ptr()
        off = (-base) % 256
        return base + off, self._ws.numel() - off


@dataclass
class DeviceFrontier:
    """Device copies of one batch of split-search input (torch tensors)."""

    X: object
    y: object
    n_classes: int
    node_offsets: object
    sample_idx: object
    proj_offsets: object
    nz_offsets: object
    nz_feature: object
    nz_weight: object
    node_bins: object = None
    nz_value: object = None      # FP32 weights (then nz_weight is None)
    max_node_samples: int = 0
    max_proj_per_node: int = 0

    @property
    def n_nodes(self) -> int:
        return int(self.node_offsets.numel() - 1)

    def structs(self):
        X = self.X
        dtype = SOF_F16 if str(X.dtype) == "torch.float16" else SOF_F32
        d = sof_data(_ptr(X), _ptr(self.y), int(X.stride(0)), int(X.shape[1]), int(X.shape[0]),
                     int(self.n_classes), dtype)
        f = sof_frontier(_ptr(self.node_offsets), _ptr(self.sample_idx), int(self.sample_idx.numel()),
                         self.n_nodes, int(self.max_node_samples))
        p = sof_proj(_ptr(self.proj_offsets), _ptr(self.nz_offsets), _ptr(self.nz_feature),
                     _ptr(self.nz_weight), int(self.nz_feature.numel()), int(self.nz_offsets.numel() - 1),
                     int(self.max_proj_per_node), _ptr(self.nz_value))
        return d, f, p


def to_device(wl, device="cuda:0", X=None) -> DeviceFrontier:
    """Copy a workload's host arrays to the device (no computation)."""
    import torch

    def t(a, dt):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(device)

    n = np.diff(wl.node_offsets.astype(np.int64))
    k = np.diff(wl.proj_offsets.astype(np.int64))
    Xd = X if X is not None else torch.from_numpy(np.ascontiguousarray(wl.X)).to(device)
    fw = np.asarray(wl.nz_weight).dtype.kind == "f"
    return DeviceFrontier(
        X=Xd, y=t(wl.y, np.int32), n_classes=int(wl.n_classes),
        node_offsets=t(wl.node_offsets, np.int32), sample_idx=t(wl.sample_idx, np.int32),
        proj_offsets=t(wl.proj_offsets, np.int32), nz_offsets=t(wl.nz_offsets, np.int32),
        nz_feature=t(wl.nz_feature, np.int32), nz_weight=None if fw else t(wl.nz_weight, np.int8),
        nz_value=t(wl.nz_weight, np.float32) if fw else None,
        node_bins=None if wl.node_bins is None else t(wl.node_bins, np.int32),
        max_node_samples=int(n.max()) if n.size else 0, max_proj_per_node=int(k.max()) if k.size else 0)


def _params(dev: DeviceFrontier, bins: int, sort_threshold: int, bin_mode: int = SOF_BINS_EQUAL,
            bin_seed: int = 0, criterion: int = SOF_CRIT_GINI, small_max: int = 0, mid_split: int = 0) -> sof_params:
    return sof_params(_ptr(dev.node_bins), int(bins), int(sort_threshold), int(bin_mode), int(criterion),
                      int(bin_seed) & (2**64 - 1), int(small_max), int(mid_split))


def workspace_size(dev: DeviceFrontier, bins: int = 256, sort_threshold: int = 0, ctx=None,
                   criterion: int = SOF_CRIT_GINI) -> int:
    d, f, p = dev.structs()
    q = _params(dev, bins, sort_threshold, criterion=criterion)
    out = ctypes.c_size_t(0)
    _check(lib().sof_workspace_size(ctx.handle if ctx else None, ctypes.byref(d), ctypes.byref(f),
                                    ctypes.byref(p), ctypes.byref(q), ctypes.byref(out)))
    return int(out.value)


def find_splits(ctx: Context, dev: DeviceFrontier, *, bins=256, sort_threshold=0, hist=False,
                out=None, stream=None, bin_mode=SOF_BINS_EQUAL, bin_seed=0, criterion=SOF_CRIT_GINI,
                small_max=0, mid_split=0):
    """Best split per node.  Returns (splits int32 tensor (N, 10) in sof_split
    layout, hist int32 tensor (P, bins, C) or None).  small_max / mid_split:
    the wave tile edges (0: the library's defaults)."""
    import torch
    d, f, p = dev.structs()
    q = _params(dev, bins, sort_threshold, bin_mode, bin_seed, criterion, small_max, mid_split)
    ws, wsb = ctx.workspace(workspace_size(dev, bins, sort_threshold, ctx, criterion))
    N = dev.n_nodes
    if out is None:
        out = torch.empty((max(N, 1), 10), dtype=torch.int32, device=dev.node_offsets.device)
    H = None
    if hist:
        H = torch.empty((int(dev.nz_offsets.numel() - 1), bins, dev.n_classes), dtype=torch.int32,
                        device=dev.node_offsets.device)
    _check(lib().sof_find_splits(ctx.handle, ctypes.byref(d), ctypes.byref(f), ctypes.byref(p),
                                 ctypes.byref(q), _ptr(out), _ptr(H), ws, wsb, _stream(stream)))
    return out, H


def find_splits_noalloc(ctx: Context, dev: DeviceFrontier, *, bins=256, sort_threshold=0, hist=False,
                        out=None, stream=None, bin_mode=SOF_BINS_EQUAL, bin_seed=0, criterion=SOF_CRIT_GINI):
    """find_splits through sof_find_splits_noalloc: the library's static
    per-device scratch instead of a workspace.  Pass preallocated out (and
    hist) tensors to allocate nothing at all."""
    import torch
    d, f, p = dev.structs()
    q = _params(dev, bins, sort_threshold, bin_mode, bin_seed, criterion)
    N = dev.n_nodes
    if out is None:
        out = torch.empty((max(N, 1), 10), dtype=torch.int32, device=dev.node_offsets.device)
    H = hist if hist is not False and hist is not True else None
    if hist is True:
        H = torch.empty((int(dev.nz_offsets.numel() - 1), bins, dev.n_classes), dtype=torch.int32,
                        device=dev.node_offsets.device)
    _check(lib().sof_find_splits_noalloc(ctx.handle, ctypes.byref(d), ctypes.byref(f), ctypes.byref(p),
                                         ctypes.byref(q), _ptr(out), _ptr(H), _stream(stream)))
    return out, H


def partition(ctx: Context, dev: DeviceFrontier, splits, *, bins=256, stream=None):
    """Stable partition.  Returns (out_idx, child_offsets) int32 tensors."""
    import torch
    d, f, p = dev.structs()
    q = _params(dev, bins, 0)
    ws, wsb = ctx.workspace(workspace_size(dev, bins, 0, ctx))
    out_idx = torch.empty_like(dev.sample_idx)
    coff = torch.empty(2 * dev.n_nodes + 1, dtype=torch.int32, device=dev.sample_idx.device)
    _check(lib().sof_partition(ctx.handle, ctypes.byref(d), ctypes.byref(f), ctypes.byref(p),
                               ctypes.byref(q), _ptr(splits), _ptr(out_idx), _ptr(coff), ws, wsb,
                               _stream(stream)))
    return out_idx, coff


def project(ctx: Context, dev: DeviceFrontier, *, stream=None):
    """Projected values, node blocks [projection][sample] in node order."""
    import torch
    d, f, p = dev.structs()
    n = torch.diff(dev.node_offsets.long()).cpu().numpy()
    k = torch.diff(dev.proj_offsets.long()).cpu().numpy()
    total = int((n * k).sum())
    out = torch.empty(max(total, 1), dtype=torch.float32, device=dev.X.device)
    ws, wsb = ctx.workspace(workspace_size(dev, 256, 0, ctx))
    _check(lib().sof_project(ctx.handle, ctypes.byref(d), ctypes.byref(f), ctypes.byref(p), _ptr(out),
                             ws, wsb, _stream(stream)))
    return out[:total]


def splits_to_numpy(t) -> np.ndarray:
    """sof_split records (int32 tensor (N, 10)) as a numpy structured array."""
    a = t.detach().cpu().numpy().astype(np.int32, copy=False)
    return np.ascontiguousarray(a).view(SPLIT_DTYPE).reshape(-1)


def splits_from_numpy(rec: np.ndarray, device="cuda:0"):
    """Records with the sof_split fields (e.g. the oracle's) as an int32 device tensor."""
    import torch
    out = np.zeros(len(rec), SPLIT_DTYPE)
    for name in SPLIT_DTYPE.names:
        out[name] = rec[name]
    return torch.from_numpy(out.view(np.int32).reshape(-1, 10).copy()).to(device)


def data_struct(X, y, n_classes: int) -> sof_data:
    """sof_data over device tensors X ((d, n) FP32/FP16) and y (n int32)."""
    dtype = SOF_F16 if str(X.dtype) == "torch.float16" else SOF_F32
    return sof_data(_ptr(X), _ptr(y), int(X.stride(0)), int(X.shape[1]), int(X.shape[0]), int(n_classes), dtype)


def autotune(ctx: Context, n_classes: int, k: int, z: int, bins: int = 256, *, dtype=np.float32,
             stream=None, data=None) -> dict:
    """Run the library's crossover microbenchmark and return its choice: sort
    threshold, small-node bin rule and the measured curve.  With data (a
    DeviceFrontier, or a tuple (X, y, n_classes) of device tensors) it runs
    sof_autotune_on over that matrix and labels, else sof_autotune on
    synthetic rows of the given storage type."""
    t = sof_tune()
    if data is not None:
        d = data.structs()[0] if isinstance(data, DeviceFrontier) else data_struct(*data)
        _check(lib().sof_autotune_on(ctx.handle, ctypes.byref(d), int(k), int(z), int(bins), ctypes.byref(t),
                                     _stream(stream)))
    else:
        code = SOF_F16 if np.dtype(dtype) == np.float16 else SOF_F32
        _check(lib().sof_autotune(ctx.handle, code, int(n_classes), int(k), int(z), int(bins), ctypes.byref(t),
                                  _stream(stream)))
    n = int(t.n_points)
    return {"sort_threshold": int(t.sort_threshold), "bins_small": int(t.bins_small),
            "bins_switch": int(t.bins_switch), "small_max": int(t.small_max), "mid_split": int(t.mid_split),
            "ms": float(t.elapsed_ms),
            "sizes": [int(t.sizes[i]) for i in range(n)],
            "sort_us": [round(float(t.sort_us[i]), 5) for i in range(n)],
            "hist_us": [round(float(t.hist_us[i]), 5) for i in range(n)],
            "half_us": [round(float(t.half_us[i]), 5) for i in range(n)],
            "tile_base_us": [round(float(t.tile_base_us[i]), 5) for i in range(n)],
            "tile_us": [round(float(t.tile_us[i]), 5) for i in range(n)]}


def nodes_to_device(nodes: np.ndarray, device="cuda:0"):
    """Tree node records (TREE_NODE_DTYPE) as a device byte tensor."""
    import torch
    raw = np.ascontiguousarray(nodes, dtype=TREE_NODE_DTYPE).view(np.uint8).reshape(-1)
    return torch.from_numpy(raw.copy()).to(device)


def predict(ctx: Context, X, nodes, roots, n_classes: int, *, votes=True, stream=None):
    """Forest prediction for every row of X (torch (d, n) FP32/FP16 on the
    device).  nodes: device byte tensor of records (nodes_to_device), roots:
    device int32 tensor of root indices.  Returns (votes (n, C) or None, pred (n,))."""
    import torch
    dtype = SOF_F16 if str(X.dtype) == "torch.float16" else SOF_F32
    n = int(X.shape[1])
    d = sof_data(_ptr(X), None, int(X.stride(0)), n, int(X.shape[0]), int(n_classes), dtype)
    V = torch.empty((n, n_classes), dtype=torch.int32, device=X.device) if votes else None
    pred = torch.empty(max(n, 1), dtype=torch.int32, device=X.device)
    n_nodes = int(nodes.numel()) // TREE_NODE_DTYPE.itemsize
    _check(lib().sof_predict(ctx.handle, ctypes.byref(d), _ptr(nodes), n_nodes, _ptr(roots), int(roots.numel()),
                             _ptr(V), _ptr(pred), _stream(stream)))
    return V, pred[:n]


class Forest:
    """Level-wise growth of several trees to purity on the device."""

    def __init__(self, ctx: Context, X, y, n_classes: int, root_offsets, root_idx, *, k: int, z: int,
                 seed: int, bins: int = 256, sort_threshold: int = 0, max_depth: int = 64,
                 first_tree: int = 0, sampler: int = 0, weights: int = 0, criterion: int = SOF_CRIT_GINI,
                 bin_mode: int = SOF_BINS_EQUAL, bin_seed: int = 0):
        self.ctx = ctx
        self._keep = (X, y, root_idx)
        dtype = SOF_F16 if str(X.dtype) == "torch.float16" else SOF_F32
        self.data = sof_data(_ptr(X), _ptr(y), int(X.stride(0)), int(X.shape[1]), int(X.shape[0]),
                             int(n_classes), dtype)
        ro = np.ascontiguousarray(root_offsets, dtype=np.int64)
        self._ro = ro
        self.n_trees = len(ro) - 1
        self.desc = sof_forest_desc(ro.ctypes.data, _ptr(root_idx), int(seed) & (2**64 - 1), self.n_trees,
                                    int(first_tree), int(k), int(z), int(bins), int(sort_threshold),
                                    int(max_depth), int(sampler), int(weights), int(criterion), int(bin_mode), 0,
                                    int(bin_seed) & (2**64 - 1))
        h = P()
        _check(lib().sof_forest_create(ctx.handle, ctypes.byref(self.data), ctypes.byref(self.desc),
                                       ctypes.byref(h)))
        self.handle = h
        self.max_nodes = 2 * int(ro[-1]) + self.n_trees + 2

    def close(self):
        if getattr(self, "handle", None):
            lib().sof_forest_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def grow_level(self, use_graph: bool = True, stream=None):
        _check(lib().sof_grow_level(self.handle, int(bool(use_graph)), _stream(stream)))

    def frontier_size(self, stream=None) -> int:
        n = i64(0)
        _check(lib().sof_forest_frontier_size(self.handle, ctypes.byref(n), _stream(stream)))
        return int(n.value)

    def frontier_stats(self, stream=None):
        """(nodes, samples, depth) of the current frontier."""
        n, m, d = i64(0), i64(0), ctypes.c_int32(0)
        _check(lib().sof_forest_frontier_stats(self.handle, ctypes.byref(n), ctypes.byref(m), ctypes.byref(d),
                                               _stream(stream)))
        return int(n.value), int(m.value), int(d.value)

    def export(self, stream=None) -> np.ndarray:
        out = np.zeros(self.max_nodes, TREE_NODE_DTYPE)
        n = i64(0)
        _check(lib().sof_forest_export(self.handle, out.ctypes.data, int(self.max_nodes), ctypes.byref(n),
                                       _stream(stream)))
        return out[:n.value].copy()

    def predict(self, Xq, *, votes=True, stream=None):
        """Predict rows of Xq (device (d, n) tensor, the training layout) with this forest."""
        import torch
        nodes = nodes_to_device(self.export(stream), Xq.device)
        roots = torch.arange(self.n_trees, dtype=torch.int32, device=Xq.device)
        return predict(self.ctx, Xq, nodes, roots, self.data.n_classes, votes=votes, stream=stream)

    def grow(self, use_graph: bool = True, stream=None, max_levels: int = 65):
        """Grow until the frontier is empty; returns the frontier size before each level."""
        sizes = []
        for _ in range(max_levels):
            n = self.frontier_size(stream)
            if n == 0:
                break
            sizes.append(n)
            self.grow_level(use_graph, stream)
        return sizes
