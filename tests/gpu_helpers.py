"""Shared helpers of the GPU parity tests (comparison against the oracle)."""
from __future__ import annotations

import sys

import numpy as np

from oracle import oracle as O

GAIN_RTOL = 1e-6


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def assert_splits_match(gpu: np.ndarray, ref: np.ndarray, where: str = ""):
    """Bit-exact on every field but the gain; gain within 1e-6 relative of the
    FP64 oracle (and exactly 0 when the oracle's is 0)."""
    assert gpu.shape == ref.shape, where
    for f in ("proj", "kind", "bin", "n_left", "n_right", "flags"):
        bad = np.nonzero(gpu[f] != ref[f])[0]
        if bad.size:
            i = int(bad[0])
            raise AssertionError(f"{where}: field {f} differs at node {i} ({bad.size} nodes): "
                                 f"gpu {gpu[i]} oracle {ref[i]}")
    for f in ("threshold", "lo", "scale"):
        a = np.ascontiguousarray(gpu[f]).view(np.uint32)
        b = np.ascontiguousarray(ref[f].astype(np.float32)).view(np.uint32)
        bad = np.nonzero(a != b)[0]
        if bad.size:
            i = int(bad[0])
            raise AssertionError(f"{where}: field {f} bits differ at node {i}: gpu {gpu[i]} oracle {ref[i]}")
    g = gpu["gain"].astype(np.float64)
    r = ref["gain"]
    zero = r == 0
    assert np.all(g[zero] == 0), f"{where}: gain should be exactly 0"
    rel = np.abs(g[~zero] - r[~zero]) / r[~zero]
    if rel.size and rel.max() > GAIN_RTOL:
        i = int(np.nonzero(~zero)[0][int(np.argmax(rel))])
        raise AssertionError(f"{where}: gain rel err {rel.max():.3g} at node {i}: gpu {gpu[i]} oracle {ref[i]}")


def oracle_splits(wl, **kw):
    return O.find_splits_w(wl, **kw)
