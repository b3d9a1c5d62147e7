"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point the public header declares, and rejects bad arguments with
the documented status codes before any device work."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sof.h")

OK, INVALID, UNSUPPORTED, WORKSPACE, OVERFLOW, HIP = 0, -1, -2, -3, -4, -5
FAKE = 0x10000  # a non-NULL address; host-side validation never dereferences it


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\**\s*(sof_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def S():
    from paper_2603_00326_amd import sof
    if not os.path.exists(sof.LIB_PATH):
        pytest.fail(f"{sof.LIB_PATH} is not built; run __graft_entry__.build() first")
    return sof


@pytest.fixture(scope="module")
def L(S):
    return S.lib()


def test_header_declares_the_boundary():
    names = header_functions()
    for must in ("sof_create", "sof_destroy", "sof_workspace_size", "sof_project", "sof_find_splits",
                 "sof_partition", "sof_forest_create", "sof_grow_level", "sof_forest_frontier_size",
                 "sof_forest_export", "sof_autotune", "sof_predict", "sof_last_error"):
        assert must in names


def test_every_declared_symbol_is_exported(S, L):
    names = header_functions()
    raw = ctypes.CDLL(S.LIB_PATH)
    missing = [n for n in names if not hasattr(raw, n)]
    assert not missing, f"declared in sof.h but not exported: {missing}"
    assert sorted(S.EXPORTED) == names, "the Python binding's symbol list differs from the header"


def test_version_and_error_strings(L):
    assert L.sof_version().decode().startswith("sof")
    L.sof_last_error.restype = ctypes.c_char_p
    assert L.sof_create(0, None) == INVALID
    assert b"NULL" in L.sof_last_error()


def data(S, **kw):
    d = dict(x=FAKE, y=FAKE, ld=1000, n_rows=1000, n_features=16, n_classes=3, dtype=S.SOF_F32)
    d.update(kw)
    return S.sof_data(d["x"], d["y"], d["ld"], d["n_rows"], d["n_features"], d["n_classes"], d["dtype"])


def frontier(S, **kw):
    f = dict(node_offsets=FAKE, sample_idx=FAKE, n_samples=1000, n_nodes=4, max_node_samples=400)
    f.update(kw)
    return S.sof_frontier(f["node_offsets"], f["sample_idx"], f["n_samples"], f["n_nodes"],
                          f["max_node_samples"])


def proj(S, **kw):
    p = dict(proj_offsets=FAKE, nz_offsets=FAKE, nz_feature=FAKE, nz_weight=FAKE, n_nz=64, n_proj=32,
             max_proj_per_node=8, nz_value=None)
    p.update(kw)
    return S.sof_proj(p["proj_offsets"], p["nz_offsets"], p["nz_feature"], p["nz_weight"], p["n_nz"],
                      p["n_proj"], p["max_proj_per_node"], p["nz_value"])


def params(S, **kw):
    q = dict(node_bins=None, bins=256, sort_threshold=64, bin_mode=0, bin_seed=0, criterion=0, small_max=0,
             mid_split=0)
    q.update(kw)
    return S.sof_params(q["node_bins"], q["bins"], q["sort_threshold"], q["bin_mode"], q["criterion"],
                        q["bin_seed"], q["small_max"], q["mid_split"])


def ws_size(S, L, d=None, f=None, p=None, q=None):
    out = ctypes.c_size_t(0)
    rc = L.sof_workspace_size(None, ctypes.byref(d or data(S)), ctypes.byref(f or frontier(S)),
                              ctypes.byref(p or proj(S)), ctypes.byref(q or params(S)), ctypes.byref(out))
    return rc, out.value


def test_workspace_size_of_valid_arguments(S, L):
    rc, n = ws_size(S, L)
    assert rc == OK and n > 0
    # every wave tile in range is accepted and sized alike
    for sm, ms in ((256, 2048), (384, 3072), (512, 4096)):
        rc_t, n_t = ws_size(S, L, q=params(S, small_max=sm, mid_split=ms))
        assert rc_t == OK and n_t == n
    # larger frontiers never need less workspace
    rc2, n2 = ws_size(S, L, f=frontier(S, n_nodes=40, n_samples=100000, max_node_samples=4000),
                      d=data(S, n_rows=100000, ld=100000))
    assert rc2 == OK and n2 >= n
    rc3, n3 = ws_size(S, L, f=frontier(S, n_nodes=0, n_samples=0, max_node_samples=0, sample_idx=None))
    assert rc3 == OK and n3 <= n


@pytest.mark.parametrize("part,kw,code", [
    ("data", dict(dtype=7), UNSUPPORTED),
    ("data", dict(n_classes=1), UNSUPPORTED),
    ("data", dict(n_classes=17), UNSUPPORTED),
    ("data", dict(n_rows=0), INVALID),
    ("data", dict(n_features=0), INVALID),
    ("data", dict(ld=999), INVALID),
    ("data", dict(n_rows=(1 << 30) + 1, ld=(1 << 30) + 1), OVERFLOW),
    ("data", dict(x=None), INVALID),
    ("data", dict(y=None), INVALID),
    ("frontier", dict(n_nodes=-1), INVALID),
    ("frontier", dict(n_samples=-1), INVALID),
    ("frontier", dict(n_samples=1 << 31, max_node_samples=10), OVERFLOW),
    ("frontier", dict(n_samples=1 << 25, max_node_samples=(1 << 24) + 1), OVERFLOW),
    ("frontier", dict(max_node_samples=1001), INVALID),
    ("frontier", dict(node_offsets=None), INVALID),
    ("frontier", dict(sample_idx=None), INVALID),
    ("proj", dict(n_proj=-1), INVALID),
    ("proj", dict(max_proj_per_node=1025, n_proj=2000), INVALID),
    ("proj", dict(max_proj_per_node=33), INVALID),
    ("proj", dict(proj_offsets=None), INVALID),
    ("proj", dict(nz_feature=None), INVALID),
    ("proj", dict(nz_weight=None), INVALID),
    ("proj", dict(n_nz=1 << 31), OVERFLOW),
    ("params", dict(bins=1), UNSUPPORTED),
    ("params", dict(bins=257), UNSUPPORTED),
    ("params", dict(sort_threshold=-1), INVALID),
    ("params", dict(bin_mode=2), UNSUPPORTED),
    ("params", dict(bin_mode=-1), UNSUPPORTED),
    ("params", dict(criterion=2), UNSUPPORTED),
    ("params", dict(small_max=255), INVALID),
    ("params", dict(small_max=513), INVALID),
    ("params", dict(mid_split=2047), INVALID),
    ("params", dict(mid_split=4097), INVALID),
])
def test_workspace_size_rejects(S, L, part, kw, code):
    args = {"d": None, "f": None, "p": None, "q": None}
    key = {"data": "d", "frontier": "f", "proj": "p", "params": "q"}[part]
    args[key] = {"data": data, "frontier": frontier, "proj": proj, "params": params}[part](S, **kw)
    rc, _ = ws_size(S, L, **args)
    assert rc == code
    L.sof_last_error.restype = ctypes.c_char_p
    assert L.sof_last_error(), "a failing call leaves a message"


def test_null_context_rejected_everywhere(S, L):
    d, f, p, q = data(S), frontier(S), proj(S), params(S)
    by = ctypes.byref
    assert L.sof_find_splits(None, by(d), by(f), by(p), by(q), FAKE, None, FAKE, 1 << 20, None) == INVALID
    assert L.sof_partition(None, by(d), by(f), by(p), by(q), FAKE, FAKE, FAKE, FAKE, 1 << 20, None) == INVALID
    assert L.sof_project(None, by(d), by(f), by(p), FAKE, FAKE, 1 << 20, None) == INVALID
    desc = S.sof_forest_desc(FAKE, FAKE, 1, 1, 0, 8, 3, 256, 0, 64, 0)
    h = ctypes.c_void_p()
    assert L.sof_forest_create(None, by(d), by(desc), by(h)) == INVALID
    assert L.sof_grow_level(None, 1, None) == INVALID
    n, m, dep = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
    assert L.sof_forest_frontier_size(None, by(n), None) == INVALID
    assert L.sof_forest_frontier_stats(None, by(n), by(m), by(dep), None) == INVALID
    assert L.sof_forest_export(None, None, 0, by(n), None) == INVALID
    t = S.sof_tune()
    assert L.sof_autotune(None, S.SOF_F32, 2, 64, 3, 256, by(t), None) == INVALID
    assert L.sof_predict(None, by(d), FAKE, 10, FAKE, 1, None, FAKE, None) == INVALID
    assert L.sof_timing_enable(None, 1) == INVALID
    assert L.sof_destroy(None) == OK


def test_create_without_a_gpu_reports_an_error(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    rc = L.sof_create(0, ctypes.byref(h))
    assert rc in (HIP, INVALID) and not h.value


def test_binding_fails_loudly_without_the_library(S, monkeypatch):
    monkeypatch.setattr(S, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libsof.so"))
    monkeypatch.setattr(S, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        S.lib()


def test_entropy_on_the_histogram_path_is_accepted(S, L):
    rc, n = ws_size(S, L, q=params(S, criterion=1, sort_threshold=0))
    assert rc == OK and n > 0
    # the entropy workspace holds k ln k for k = 0 .. max_node_samples
    f = frontier(S, n_nodes=40, n_samples=100000, max_node_samples=60000)
    d = data(S, n_rows=100000, ld=100000)
    rc0, g = ws_size(S, L, d=d, f=f, q=params(S, sort_threshold=0))
    rc1, e = ws_size(S, L, d=d, f=f, q=params(S, criterion=1, sort_threshold=0))
    assert rc0 == rc1 == OK and e >= g + 60001 * 8


def test_fp32_weights_replace_integer_weights(S, L):
    rc, n = ws_size(S, L, p=proj(S, nz_weight=None, nz_value=FAKE))
    assert rc == OK and n > 0


def test_struct_layouts_match_the_header(tmp_path):
    """Sizes and field offsets of every ABI struct as the C compiler lays them
    out from sof.h equal the Python binding's."""
    import subprocess
    from paper_2603_00326_amd import sof
    structs = {"sof_data": sof.sof_data, "sof_frontier": sof.sof_frontier, "sof_proj": sof.sof_proj,
               "sof_params": sof.sof_params, "sof_forest_desc": sof.sof_forest_desc, "sof_tune": sof.sof_tune}
    lines = []
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for fname, *_ in cls._fields_:
            lines.append(f'printf("{name} {fname} %zu\\n", offsetof({name}, {fname}));')
    for fname in sof.TREE_NODE_DTYPE.names:
        lines.append(f'printf("sof_tree_node {fname} %zu\\n", offsetof(sof_tree_node, {fname}));')
    lines.append('printf("sof_tree_node size %zu\\n", sizeof(sof_tree_node));')
    lines.append('printf("sof_split size %zu\\n", sizeof(sof_split));')
    src = tmp_path / "lay.c"
    src.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"sof.h\"\nint main(void) {\n" +
                   "\n".join(lines) + "\nreturn 0;\n}\n")
    exe = tmp_path / "lay"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for ln in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        a, b, c = ln.split()
        got[(a, b)] = int(c)
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for fname, *_ in cls._fields_:
            assert got[(name, fname)] == getattr(cls, fname).offset, (name, fname)
    for fname in sof.TREE_NODE_DTYPE.names:
        assert got[("sof_tree_node", fname)] == sof.TREE_NODE_DTYPE.fields[fname][1], fname
    assert got[("sof_tree_node", "size")] == sof.TREE_NODE_DTYPE.itemsize == 200
    assert got[("sof_split", "size")] == sof.SPLIT_DTYPE.itemsize
