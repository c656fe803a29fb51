"""Host-only checks of the C ABI (no GPU needed): the library loads, exports
every function include/gfd.h declares, its struct layouts match the binding,
and malformed inputs are rejected with the documented codes before any
device call."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2608_02321_amd as P
from paper_2608_02321_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gfd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gfd_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_function():
    names = declared_functions()
    assert set(names) == set(B.EXPORTS), names
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (gfd_\w+)", out))
    for nm in names:
        assert nm in exported, nm
        assert hasattr(B.lib, nm)


STRUCTS = {
    "gfd_literal": B.gfd_literal, "gfd_edge": B.gfd_edge, "gfd_spec": B.gfd_spec,
    "gfd_result": B.gfd_result, "gfd_load_opts": B.gfd_load_opts,
    "gfd_validate_opts": B.gfd_validate_opts, "gfd_stats": B.gfd_stats, "gfd_allocator": B.gfd_allocator,
    "gfd_tuning": B.gfd_tuning,
    "gfd_graph_info": B.gfd_graph_info, "gfd_server_opts": B.gfd_server_opts,
    "gfd_request_info": B.gfd_request_info,
}


def test_struct_layouts_match_header(tmp_path):
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gfd.h"', "int main(void){"]
    for nm, cls in STRUCTS.items():
        lines.append(f'printf("{nm} %zu\\n", sizeof({nm}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{nm}.{f} %zu\\n", offsetof({nm}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                 check=True).stdout.splitlines())
    for nm, cls in STRUCTS.items():
        assert int(got[nm]) == C.sizeof(cls), nm
        for f, _ in cls._fields_:
            assert int(got[f"{nm}.{f}"]) == getattr(cls, f).offset, f"{nm}.{f}"


def test_constants_match_header():
    text = open(HEADER).read()
    defs = dict(re.findall(r"#define (GFD_\w+) \(?(-?\d+)\)?", text))
    for k, v in defs.items():
        if hasattr(B, k):
            assert getattr(B, k) == int(v), k


def _graph_arrays():
    n = 4
    row_ptr = np.array([0, 2, 3, 3, 4], dtype=np.int64)
    col = np.array([1, 2, 0, 1], dtype=np.int32)
    vl = np.zeros(n, dtype=np.int32)
    el = np.zeros(4, dtype=np.int32)
    attrs = np.zeros((1, n), dtype=np.int32)
    return n, row_ptr, col, vl, el, attrs


@pytest.mark.parametrize("mutate,code", [
    (lambda a: a[1].__setitem__(2, 1), -1),          # row_ptr decreases
    (lambda a: a[1].__setitem__(4, 3), -1),          # row_ptr does not end at m
    (lambda a: a[2].__setitem__(0, 9), -1),          # col out of range
    (lambda a: a[2].__setitem__(2, 1), -1),          # self-loop (row 1 -> 1)
    (lambda a: a[2].__setitem__(1, 1), -1),          # duplicate pair 0 -> 1
    (lambda a: a[3].__setitem__(0, -1), -1),         # negative vertex label
    (lambda a: a[4].__setitem__(0, -3), -1),         # negative edge label
    (lambda a: a[5].__setitem__((0, 0), -2), -1),    # attribute below the missing marker
])
def test_load_graph_rejects(mutate, code):
    a = list(_graph_arrays())
    mutate(a)
    n, rp, col, vl, el, at = a
    with pytest.raises(P.GfdError) as ei:
        P.load_graph(n, len(col), rp, col, vl, el, at)
    assert ei.value.code == code
    assert P.last_error()


def test_load_graph_size_limits():
    out = C.c_void_p()
    rc = B.lib.gfd_load_graph(1 << 31, 0, None, None, None, None, 0, None, None, C.byref(out))
    assert rc == B.GFD_EUNSUPPORTED
    rc = B.lib.gfd_load_graph(-1, 0, None, None, None, None, 0, None, None, C.byref(out))
    assert rc == B.GFD_EINVAL
    rc = B.lib.gfd_load_graph(0, 0, None, None, None, None, 0, None, None, None)
    assert rc == B.GFD_EINVAL


def test_validate_null_graph():
    rc = B.lib.gfd_validate(None, None, 0, None, None)
    assert rc == B.GFD_EINVAL
    assert "graph" in P.last_error()


def test_version():
    assert P.version() >= 100


def test_server_rejects_bad_arguments():
    h = C.c_void_p()
    assert B.lib.gfd_server_create(None, None, C.byref(h)) == B.GFD_EINVAL
    assert B.lib.gfd_server_create(None, None, None) == B.GFD_EINVAL
    rid = C.c_uint64()
    spec = B.make_spec({"k": 1, "vlabels": [0], "edges": [], "x": [], "y": []})
    assert B.lib.gfd_server_submit(None, C.byref(spec), 1, C.byref(rid)) == B.GFD_EINVAL
    assert B.lib.gfd_server_wait(None, 1, 0, None, None) == B.GFD_EINVAL
    B.lib.gfd_server_destroy(None)  # ignored


def test_load_graph_rejects_malformed_options():
    """An allocator with alloc but no free, or an unknown mem_kind, is refused
    before anything touches a device."""
    n, rp, col, vl, el, at = _graph_arrays()
    out = C.c_void_p()
    ptrs = (C.c_void_p * 1)(at[0].ctypes.data)
    args = (n, len(col), rp.ctypes.data, col.ctypes.data, vl.ctypes.data, el.ctypes.data, 1, ptrs)
    half = B.gfd_allocator(B.ALLOC_FN(lambda ctx, nb, st: None), B.FREE_FN(), None)
    opts = B.gfd_load_opts(None, B.GFD_MEM_HOST, half)
    assert B.lib.gfd_load_graph(*args, C.byref(opts), C.byref(out)) == B.GFD_EINVAL
    assert "free" in P.last_error()
    opts = B.gfd_load_opts(None, 7, B.gfd_allocator())
    assert B.lib.gfd_load_graph(*args, C.byref(opts), C.byref(out)) == B.GFD_EINVAL
    assert "mem_kind" in P.last_error()


@pytest.mark.parametrize("which,value,code", [
    ("vlabel", (1 << 24), B.GFD_EUNSUPPORTED),   # above GFD_MAX_LABEL
    ("elabel", (1 << 24), B.GFD_EUNSUPPORTED),
    ("vlabel", (1 << 31) - 1, B.GFD_EUNSUPPORTED),  # INT32_MAX: no signed overflow
    ("both", 5000, B.GFD_EUNSUPPORTED),          # 5001 * 5001 label pairs > 2^24
    ("vlabel", 4095, None),                      # 4096 * 1 pairs: accepted (no device here)
])
def test_label_id_limits(which, value, code):
    """Host tables are sized by the largest label ids: ids above GFD_MAX_LABEL
    and key spaces above GFD_MAX_LABEL_PAIRS are refused with a status code
    (not an allocation failure or a crash) before any device work."""
    n, rp, col, vl, el, at = _graph_arrays()
    if which in ("vlabel", "both"):
        vl[0] = value
    if which in ("elabel", "both"):
        el[0] = value
    if code is None:
        try:
            P.load_graph(n, len(col), rp, col, vl, el, at)
        except P.GfdError as e:  # no GPU in this container: the device step fails
            assert e.code in (B.GFD_EDEVICE, B.GFD_ENOMEM), e
        return
    with pytest.raises(P.GfdError) as ei:
        P.load_graph(n, len(col), rp, col, vl, el, at)
    assert ei.value.code == code
    assert "label" in P.last_error()
