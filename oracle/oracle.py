"""Python driver for the C oracle -- TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this module.  It compiles ``oracle.c`` with gcc into ``liboracle.so`` next to
it and calls it through ctypes.  It shares no code with the GPU library.

Semantics of a result dict (Section II definitions; see oracle.c):
    match_count, violation_count, match_fp, violation_fp  (ints, fp mod 2^64)
    satisfied = violation_count == 0
    violations = first min(K, violation_count) violating tuples, ascending
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

INDUCED, MONO = "induced", "mono"


class _Lit(C.Structure):
    _fields_ = [("kind", C.c_int32), ("var", C.c_int32), ("attr", C.c_int32),
                ("var2", C.c_int32), ("attr2", C.c_int32), ("value", C.c_int32)]


def compile_c(src: str, out: str) -> str:
    tmp = out + ".tmp"
    subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
                    "-pthread", src, "-o", tmp], check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = False) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        compile_c(SRC, LIB)
    return LIB


_lib = None


def load(path: str):
    """Open an oracle shared library (the built one, or a test's variant)."""
    L = C.CDLL(path)
    L.orc_graph_new.restype = C.c_void_p
    L.orc_graph_new.argtypes = [C.c_int64, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_void_p, C.c_int32, C.c_void_p]
    L.orc_graph_free.argtypes = [C.c_void_p]
    L.orc_validate.restype = C.c_int
    L.orc_validate.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p,
                               C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32,
                               C.c_int32, C.c_int32, C.c_int64, C.c_int64, C.c_int32,
                               C.c_void_p, C.c_void_p, C.c_void_p]
    return L


def lib():
    """The oracle library: the built one, or the build named by GFD_ORACLE_LIB
    (a sanitizer build of the same source, for the tests)."""
    global _lib
    if _lib is None:
        other = os.environ.get("GFD_ORACLE_LIB")
        if other:
            _lib = load(other)
        else:
            build()
            _lib = load(LIB)
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class OracleGraph:
    """The oracle's private copy of a graph (rows re-sorted, in-rows built)."""

    def __init__(self, g, L=None):
        L = L or lib()
        self.L = L
        self._keep = [np.ascontiguousarray(g.row_ptr, dtype=np.int64),
                      np.ascontiguousarray(g.col, dtype=np.int32),
                      np.ascontiguousarray(g.vlabel, dtype=np.int32),
                      np.ascontiguousarray(g.elabel, dtype=np.int32),
                      np.ascontiguousarray(g.attrs, dtype=np.int32).reshape(-1)]
        rp, col, vl, el, at = self._keep
        self.n, self.num_attrs = int(g.n), int(g.attrs.shape[0])
        self.h = L.orc_graph_new(g.n, g.m, _ptr(rp), _ptr(col), _ptr(vl), _ptr(el),
                                 self.num_attrs, _ptr(at))
        if not self.h:
            raise ValueError("oracle: malformed graph")
        self._keep = None

    def __del__(self):
        if getattr(self, "h", None):
            self.L.orc_graph_free(self.h)
            self.h = None


def _lits(lst):
    arr = (_Lit * max(1, len(lst)))()
    for i, l in enumerate(lst):
        if l["kind"] == "const":
            arr[i] = _Lit(0, l["var"], l["attr"], 0, 0, l["value"])
        else:
            arr[i] = _Lit(1, l["var"], l["attr"], l["var2"], l["attr2"], 0)
    return arr


def validate(og: OracleGraph, gfd: dict, semantics: str = INDUCED, K: int = 1024,
             root_range=None, threads: int = 1) -> dict:
    """Validate one GFD by the plain definition; root_range restricts t_0."""
    k = int(gfd["k"])
    qlab = np.asarray(gfd["vlabels"], dtype=np.int32)
    qe = np.asarray(gfd["edges"], dtype=np.int32).reshape(-1, 3)
    xs, ys = _lits(gfd.get("x", [])), _lits(gfd.get("y", []))
    out = np.zeros(4, dtype=np.uint64)
    viol = np.zeros(max(1, K * k), dtype=np.int32)
    nrep = C.c_int32(0)
    lo, hi = (0, og.n) if root_range is None else root_range
    rc = og.L.orc_validate(og.h, k, _ptr(qlab), len(qe), _ptr(qe), len(gfd.get("x", [])), xs,
                            len(gfd.get("y", [])), ys, int(bool(gfd.get("y_false", False))),
                            int(semantics == INDUCED), K, lo, hi, threads, _ptr(out),
                            _ptr(viol), C.byref(nrep))
    if rc != 0:
        raise ValueError("oracle: malformed GFD")
    r = nrep.value
    return {"match_count": int(out[0]), "violation_count": int(out[1]),
            "match_fp": int(out[2]), "violation_fp": int(out[3]),
            "satisfied": int(out[1]) == 0,
            "violations": viol[:r * k].reshape(r, k).tolist()}
