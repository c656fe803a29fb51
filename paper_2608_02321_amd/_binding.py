"""ctypes binding of include/gfd.h (argument marshalling only).

Every step of validation runs in libgfd.so's HIP kernels; this module only
converts Python/numpy inputs into the C structs and back.  It raises at import
time if the library is missing -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
# GFD_LIBRARY names another build of the same library (the unit-counting one,
# libgfd_count.so, for measurement runs)
LIB_PATH = os.environ.get("GFD_LIBRARY") or os.path.join(PKG, "libgfd.so")
UNIT_NAMES = ("attempts", "sources", "injective", "checks_both", "table_free", "table_hit",
              "short_row", "both_steps", "both_log2d", "checks_one", "one_steps", "one_log2d",
              "matches", "literal_reads", "violations", "inner_attempts")

GFD_OK, GFD_EINVAL, GFD_ENOMEM, GFD_EDEVICE, GFD_EUNSUPPORTED, GFD_EOVERFLOW = 0, -1, -2, -3, -4, -5
GFD_EAGAIN = -6
GFD_WILDCARD = GFD_ABSENT = -1
GFD_MAX_K = 8
GFD_MAX_LITERALS = 8
GFD_MAX_PATTERN_EDGES = GFD_MAX_K * (GFD_MAX_K - 1)
GFD_LIT_CONST, GFD_LIT_VAR = 0, 1
GFD_SEM_INDUCED, GFD_SEM_MONO = 0, 1
GFD_FLAG_FORCE_CHUNKED, GFD_FLAG_TIMING, GFD_FLAG_COUNT_ONLY, GFD_FLAG_NO_GRAPH = 1, 2, 4, 8
STATUS_NAMES = {0: "GFD_OK", -1: "GFD_EINVAL", -2: "GFD_ENOMEM", -3: "GFD_EDEVICE",
                -4: "GFD_EUNSUPPORTED", -5: "GFD_EOVERFLOW", -6: "GFD_EAGAIN"}
KERNEL_CLASSES = ("filter", "pull", "cpi", "extend", "extend_last", "scan", "topk", "other")


class GfdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class gfd_literal(C.Structure):
    _fields_ = [("kind", C.c_int32), ("var", C.c_int32), ("attr", C.c_int32),
                ("var2", C.c_int32), ("attr2", C.c_int32), ("constant", C.c_int32)]


class gfd_edge(C.Structure):
    _fields_ = [("src", C.c_int32), ("dst", C.c_int32), ("label", C.c_int32)]


class gfd_spec(C.Structure):
    _fields_ = [("num_vertices", C.c_int32), ("vertex_labels", C.c_int32 * GFD_MAX_K),
                ("num_edges", C.c_int32), ("edges", gfd_edge * GFD_MAX_PATTERN_EDGES),
                ("num_x", C.c_int32), ("x", gfd_literal * GFD_MAX_LITERALS),
                ("num_y", C.c_int32), ("y", gfd_literal * GFD_MAX_LITERALS),
                ("y_is_false", C.c_int32)]


class gfd_result(C.Structure):
    _fields_ = [("satisfied", C.c_int32), ("num_reported", C.c_int32),
                ("match_count", C.c_uint64), ("violation_count", C.c_uint64),
                ("match_fp", C.c_uint64), ("violation_fp", C.c_uint64),
                ("violations", C.POINTER(C.c_int32))]


GFD_MEM_HOST, GFD_MEM_DEVICE = 0, 1
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_int64)


class gfd_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class gfd_load_opts(C.Structure):
    _fields_ = [("hip_stream", C.c_void_p), ("mem_kind", C.c_int32), ("allocator", gfd_allocator)]


class gfd_tuning(C.Structure):
    _fields_ = [("flat_grid", C.c_int32), ("scan_grid", C.c_int32), ("probe_ahead", C.c_int32),
                ("staging_log2", C.c_int32), ("ext_occupancy", C.c_int32)]


def make_tuning(t) -> gfd_tuning:
    """gfd_tuning from a dict (missing keys: the library's defaults)."""
    t = t or {}
    return gfd_tuning(int(t.get("flat_grid", 0)), int(t.get("scan_grid", 0)),
                      int(t.get("probe_ahead", 0)), int(t.get("staging_log2", 0)),
                      int(t.get("ext_occupancy", 0)))


class gfd_validate_opts(C.Structure):
    _fields_ = [("k_max", C.c_int32), ("semantics", C.c_int32),
                ("mem_budget_bytes", C.c_int64), ("hip_stream", C.c_void_p),
                ("batched", C.c_int32), ("flags", C.c_int32),
                ("frontier_cap", C.c_int64), ("violation_cap", C.c_int64),
                ("allocator", gfd_allocator), ("tuning", gfd_tuning)]


class gfd_stats(C.Structure):
    _fields_ = [("wall_ms", C.c_double), ("launches", C.c_int32), ("chunked_gfds", C.c_int32),
                ("attempts", C.c_uint64), ("partials", C.c_uint64),
                ("cpi_candidates", C.c_uint64), ("cpi_entries", C.c_uint64),
                ("class_launches", C.c_int32 * 8), ("class_ms", C.c_double * 8),
                ("class_bytes", C.c_uint64 * 8), ("threshold_gfds", C.c_int32),
                ("threshold_passes", C.c_int32), ("leaf_gfds", C.c_int32),
                ("regrown_gfds", C.c_int32), ("front_pool_bytes", C.c_int64),
                ("cpi_arena_bytes", C.c_int64), ("graph_captures", C.c_int32),
                ("graph_replays", C.c_int32), ("units_counted", C.c_int32),
                ("units", C.c_uint64 * 16), ("leaf_split_gfds", C.c_int32),
                ("batches", C.c_int32)]


class gfd_graph_info(C.Structure):
    _fields_ = [("n", C.c_int64), ("m", C.c_int64), ("num_attrs", C.c_int32),
                ("num_vertex_labels", C.c_int32), ("num_edge_labels", C.c_int32),
                ("device_bytes", C.c_int64)]


class gfd_server_opts(C.Structure):
    _fields_ = [("workers", C.c_int32), ("max_batch_gfds", C.c_int32),
                ("mem_budget_bytes", C.c_int64), ("k_max", C.c_int32), ("semantics", C.c_int32),
                ("allocator", gfd_allocator)]


class gfd_request_info(C.Structure):
    _fields_ = [("submit_ns", C.c_int64), ("start_ns", C.c_int64), ("done_ns", C.c_int64),
                ("batch_id", C.c_uint64), ("batch_gfds", C.c_int32),
                ("batch_requests", C.c_int32), ("worker", C.c_int32)]


EXPORTS = ("gfd_load_graph", "gfd_free_graph", "gfd_trim", "gfd_validate", "gfd_validate_ex",
           "gfd_validate_noalloc",
           "gfd_get_graph_info", "gfd_server_create", "gfd_server_submit", "gfd_server_wait",
           "gfd_server_destroy", "gfd_last_error", "gfd_version")


def _load():
    # One HIP runtime per process: torch ships its own libamdhip64 (soname
    # libamdhip64.so.7, loaded as libamdhip64.so).  Loading torch first lets
    # libgfd.so bind to that same runtime; loading libgfd.so first would bring in
    # a second HIP/HSA runtime that cannot see the device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(python paper_2608_02321_amd/build.py); there is no CPU fallback")
    L = C.CDLL(LIB_PATH)
    L.gfd_load_graph.restype = C.c_int32
    L.gfd_load_graph.argtypes = [C.c_int64, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_int32, C.POINTER(C.c_void_p),
                                 C.POINTER(gfd_load_opts), C.POINTER(C.c_void_p)]
    L.gfd_free_graph.restype = None
    L.gfd_free_graph.argtypes = [C.c_void_p]
    L.gfd_trim.restype = C.c_int32
    L.gfd_trim.argtypes = [C.c_void_p]
    L.gfd_validate.restype = C.c_int32
    L.gfd_validate.argtypes = [C.c_void_p, C.POINTER(gfd_spec), C.c_int32,
                               C.POINTER(gfd_validate_opts), C.POINTER(gfd_result)]
    L.gfd_validate_noalloc.restype = C.c_int32
    L.gfd_validate_noalloc.argtypes = [C.c_void_p, C.POINTER(gfd_spec), C.c_int32,
                                       C.POINTER(gfd_validate_opts), C.POINTER(gfd_result)]
    L.gfd_validate_ex.restype = C.c_int32
    L.gfd_validate_ex.argtypes = [C.c_void_p, C.POINTER(gfd_spec), C.c_int32,
                                  C.POINTER(gfd_validate_opts), C.POINTER(gfd_result),
                                  C.POINTER(gfd_stats)]
    L.gfd_get_graph_info.restype = C.c_int32
    L.gfd_get_graph_info.argtypes = [C.c_void_p, C.POINTER(gfd_graph_info)]
    L.gfd_last_error.restype = C.c_char_p
    L.gfd_last_error.argtypes = []
    L.gfd_version.restype = C.c_int32
    L.gfd_version.argtypes = []
    L.gfd_server_create.restype = C.c_int32
    L.gfd_server_create.argtypes = [C.c_void_p, C.POINTER(gfd_server_opts), C.POINTER(C.c_void_p)]
    L.gfd_server_submit.restype = C.c_int32
    L.gfd_server_submit.argtypes = [C.c_void_p, C.POINTER(gfd_spec), C.c_int32,
                                    C.POINTER(C.c_uint64)]
    L.gfd_server_wait.restype = C.c_int32
    L.gfd_server_wait.argtypes = [C.c_void_p, C.c_uint64, C.c_int32, C.POINTER(gfd_result),
                                  C.POINTER(gfd_request_info)]
    L.gfd_server_destroy.restype = None
    L.gfd_server_destroy.argtypes = [C.c_void_p]
    return L


lib = _load()


def last_error() -> str:
    return lib.gfd_last_error().decode()


def version() -> int:
    return int(lib.gfd_version())


def _check(rc):
    if rc != GFD_OK:
        raise GfdError(rc, last_error())


def _stream_handle(stream):
    """hipStream_t of a torch stream (or an int handle); None = null stream."""
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def current_torch_stream():
    import torch
    if torch.cuda.is_available():
        return torch.cuda.current_stream()
    return None


class TorchAllocator:
    """gfd_allocator callbacks backed by torch's caching allocator, so the
    library's device memory is torch's: it shows in torch.cuda.memory_allocated
    and returns to torch's cache when freed.  Counts its calls (tests)."""

    def __init__(self, device=None):
        import torch
        self.torch = torch
        self.device = torch.cuda.current_device() if device is None else int(device)
        self.allocs = self.frees = 0
        self.live_bytes = self.peak_bytes = 0
        self._sizes = {}
        self._alloc = ALLOC_FN(self._on_alloc)
        self._free = FREE_FN(self._on_free)
        self.c = gfd_allocator(self._alloc, self._free, None)

    def _on_alloc(self, ctx, nbytes, stream):
        try:
            p = self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device, int(stream or 0))
        except Exception:  # out of memory: the library reports GFD_ENOMEM
            return None
        self.allocs += 1
        self._sizes[p] = int(nbytes)
        self.live_bytes += int(nbytes)
        self.peak_bytes = max(self.peak_bytes, self.live_bytes)
        return p

    def _on_free(self, ctx, ptr, nbytes):
        if not ptr:
            return
        self.frees += 1
        self.live_bytes -= self._sizes.pop(ptr, int(nbytes))
        self.torch.cuda.caching_allocator_delete(ptr)


_default_alloc = None


def torch_allocator():
    """The process-wide TorchAllocator (made on first use)."""
    global _default_alloc
    if _default_alloc is None:
        _default_alloc = TorchAllocator()
    return _default_alloc


def _torch_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except ImportError:
        return False


def _allocator(alloc):
    """gfd_allocator for an `allocator=` argument: "torch" (default) = the
    process-wide TorchAllocator (the library's own hipMalloc where torch sees
    no GPU), None = the library's own hipMalloc, or a TorchAllocator."""
    if isinstance(alloc, str) and alloc == "torch":
        alloc = torch_allocator() if _torch_gpu() else None
    if alloc is None:
        return gfd_allocator(), None
    return alloc.c, alloc


class GraphHandle:
    """A graph resident on the device (gfd_load_graph / gfd_free_graph).
    Holds the allocators its memory and workspaces came from, so their
    callbacks outlive the graph."""

    def __init__(self, h, info, allocators=()):
        self._h = h
        self.info = info
        self._allocators = list(allocators)

    @property
    def handle(self):
        if not self._h:
            raise ValueError("graph already freed")
        return self._h

    def keep(self, alloc):
        if alloc is not None and all(a is not alloc for a in self._allocators):
            self._allocators.append(alloc)

    def trim(self):
        """gfd_trim: return the workspaces kept between calls."""
        _check(lib.gfd_trim(self.handle))

    def free(self):
        h = getattr(self, "_h", None)
        if h and lib is not None:
            lib.gfd_free_graph(h)
        self._h = None

    def __del__(self):
        try:  # at interpreter exit the module globals may already be gone
            self.free()
        except Exception:
            pass


def _device_ptr(x):
    return int(x.data_ptr())


def load_graph(n, m, row_ptr, col, vlabel, elabel, attrs=None, stream=None,
               allocator="torch") -> GraphHandle:
    """gfd_load_graph: out-CSR as host arrays, or as torch tensors on the
    current GPU (mem_kind GFD_MEM_DEVICE: the library reads them there)."""
    try:
        import torch
        on_dev = isinstance(row_ptr, torch.Tensor) and row_ptr.is_cuda
    except ImportError:
        torch, on_dev = None, False
    if on_dev:
        keep = [row_ptr.to(torch.int64).contiguous(), col.to(torch.int32).contiguous(),
                vlabel.to(torch.int32).contiguous(), elabel.to(torch.int32).contiguous()]
        A = 0 if attrs is None else int(attrs.shape[0])
        cols = [attrs[a].to(torch.int32).contiguous() for a in range(A)]
        ptrs = (C.c_void_p * max(A, 1))(*[_device_ptr(c) for c in cols])
        args = [_device_ptr(x) for x in keep]
        kind = GFD_MEM_DEVICE
    else:
        keep = [np.ascontiguousarray(row_ptr, dtype=np.int64),
                np.ascontiguousarray(col, dtype=np.int32),
                np.ascontiguousarray(vlabel, dtype=np.int32),
                np.ascontiguousarray(elabel, dtype=np.int32)]
        A = 0 if attrs is None else int(np.asarray(attrs).shape[0])
        cols = [np.ascontiguousarray(np.asarray(attrs)[a], dtype=np.int32) for a in range(A)]
        ptrs = (C.c_void_p * max(A, 1))(*[c.ctypes.data for c in cols])
        args = [x.ctypes.data for x in keep]
        kind = GFD_MEM_HOST
    ca, alloc = _allocator(allocator)
    opts = gfd_load_opts(_stream_handle(stream), kind, ca)
    out = C.c_void_p()
    rc = lib.gfd_load_graph(int(n), int(m), *args, A, ptrs, C.byref(opts), C.byref(out))
    _check(rc)
    info = gfd_graph_info()
    _check(lib.gfd_get_graph_info(out, C.byref(info)))
    return GraphHandle(out.value, {f: getattr(info, f) for f, _ in gfd_graph_info._fields_},
                       [alloc] if alloc is not None else [])


def load(g, stream=None, allocator="torch") -> GraphHandle:
    """Load an object with n, m, row_ptr, col, vlabel, elabel, attrs attributes."""
    return load_graph(g.n, g.m, g.row_ptr, g.col, g.vlabel, g.elabel, g.attrs, stream=stream,
                      allocator=allocator)


def free_graph(gh: GraphHandle):
    gh.free()


def _lit(d) -> gfd_literal:
    if d["kind"] in ("const", GFD_LIT_CONST):
        return gfd_literal(GFD_LIT_CONST, d["var"], d["attr"], 0, 0, d["value"])
    return gfd_literal(GFD_LIT_VAR, d["var"], d["attr"], d["var2"], d["attr2"], 0)


def make_spec(gfd: dict) -> gfd_spec:
    """GFD dict (k, vlabels, edges, x, y, y_false) -> gfd_spec."""
    s = gfd_spec()
    k = int(gfd["k"])
    if len(gfd["vlabels"]) > GFD_MAX_K or len(gfd["edges"]) > GFD_MAX_PATTERN_EDGES or \
            len(gfd.get("x", [])) > GFD_MAX_LITERALS or len(gfd.get("y", [])) > GFD_MAX_LITERALS:
        raise GfdError(GFD_EUNSUPPORTED, "GFD exceeds the fixed spec capacity")
    s.num_vertices = k
    for i, l in enumerate(gfd["vlabels"]):
        s.vertex_labels[i] = int(l)
    s.num_edges = len(gfd["edges"])
    for i, (a, b, l) in enumerate(gfd["edges"]):
        s.edges[i] = gfd_edge(int(a), int(b), int(l))
    xs, ys = gfd.get("x", []), gfd.get("y", [])
    s.num_x, s.num_y = len(xs), len(ys)
    for i, l in enumerate(xs):
        s.x[i] = _lit(l)
    for i, l in enumerate(ys):
        s.y[i] = _lit(l)
    s.y_is_false = int(bool(gfd.get("y_false", False)))
    return s


class PreparedCall:
    """One gfd_validate_ex call with its specs, options and result buffers
    marshalled once, for repeated calls (serving loops, timing): run() only
    calls the C ABI and returns the stats; results() converts the last
    call's outputs to the dicts validate() returns."""

    def __init__(self, graph: GraphHandle, gfds, K: int = 1024, semantics: str = "induced",
                 mem_budget_bytes: int = 0, stream=None, flags: int = 0, batched: bool = False,
                 allocator="torch", tuning=None):
        self.graph, self.gfds, self.K = graph, list(gfds), int(K)
        n = len(self.gfds)
        self.n = n
        self.specs = (gfd_spec * max(n, 1))(*[make_spec(d) for d in self.gfds])
        self.res = (gfd_result * max(n, 1))()
        self.ks = [int(d["k"]) for d in self.gfds]
        self.buf = np.zeros((max(n, 1), max(1, self.K * GFD_MAX_K)), dtype=np.int32)
        for i in range(n):
            self.res[i].violations = self.buf[i].ctypes.data_as(C.POINTER(C.c_int32))
        ca, alloc = _allocator(allocator)
        graph.keep(alloc)
        self.opts = gfd_validate_opts(self.K, GFD_SEM_INDUCED if semantics == "induced"
                                      else GFD_SEM_MONO, int(mem_budget_bytes),
                                      _stream_handle(stream), int(bool(batched)), int(flags), 0, 0, ca,
                                      make_tuning(tuning))
        self.st = gfd_stats()

    def run(self, flags=None, stats=True):
        if flags is not None:
            self.opts.flags = int(flags)
        rc = lib.gfd_validate_ex(self.graph.handle, self.specs, self.n, C.byref(self.opts),
                                 self.res, C.byref(self.st) if stats else None)
        _check(rc)
        if not stats:
            return None
        return _stats_dict(self.st)

    def match_count(self):
        return sum(int(self.res[i].match_count) for i in range(self.n))

    def results(self):
        out = []
        for i in range(self.n):
            r, k = self.res[i], self.ks[i]
            out.append({"match_count": int(r.match_count),
                        "violation_count": int(r.violation_count),
                        "match_fp": int(r.match_fp), "violation_fp": int(r.violation_fp),
                        "satisfied": bool(r.satisfied),
                        "violations": self.buf[i][:r.num_reported * k].reshape(-1, k).tolist()})
        return out


def validate(graph: GraphHandle, gfds, K: int = 1024, semantics: str = "induced",
             mem_budget_bytes: int = 0, stream=None, flags: int = 0, frontier_cap: int = 0,
             violation_cap: int = 0, stats: bool = False, batched: bool = False,
             allocator="torch", noalloc: bool = False, tuning=None):
    """gfd_validate(_ex): one result dict per GFD (plus a stats dict if asked).
    noalloc: gfd_validate_noalloc instead (no allocator, no statistics)."""
    if noalloc:
        allocator = None
    n = len(gfds)
    specs = (gfd_spec * max(n, 1))(*[make_spec(d) for d in gfds])
    results = (gfd_result * max(n, 1))()
    bufs = []
    for i, d in enumerate(gfds):
        b = np.zeros(max(1, K * int(d["k"])), dtype=np.int32)
        bufs.append(b)
        results[i].violations = b.ctypes.data_as(C.POINTER(C.c_int32))
    ca, alloc = _allocator(allocator)
    graph.keep(alloc)
    opts = gfd_validate_opts(K, GFD_SEM_INDUCED if semantics == "induced" else GFD_SEM_MONO,
                             int(mem_budget_bytes), _stream_handle(stream), int(bool(batched)),
                             int(flags),
                             int(frontier_cap), int(violation_cap), ca, make_tuning(tuning))
    st = gfd_stats()
    if noalloc:
        if stats:
            raise ValueError("gfd_validate_noalloc keeps no statistics")
        rc = lib.gfd_validate_noalloc(graph.handle, specs, n, C.byref(opts), results)
    else:
        rc = lib.gfd_validate_ex(graph.handle, specs, n, C.byref(opts), results,
                                 C.byref(st) if stats else None)
    _check(rc)
    out = []
    for i, d in enumerate(gfds):
        r = results[i]
        k = int(d["k"])
        out.append({"match_count": int(r.match_count), "violation_count": int(r.violation_count),
                    "match_fp": int(r.match_fp), "violation_fp": int(r.violation_fp),
                    "satisfied": bool(r.satisfied),
                    "violations": bufs[i][:r.num_reported * k].reshape(-1, k).tolist()})
    if stats:
        return out, _stats_dict(st)
    return out


def _stats_dict(st):
    sd = {f: getattr(st, f) for f, _ in gfd_stats._fields_}
    for f in ("class_launches", "class_ms", "class_bytes"):
        sd[f] = dict(zip(KERNEL_CLASSES, list(sd[f])))
    sd["units"] = dict(zip(UNIT_NAMES, list(sd["units"])))
    return sd


class Server:
    """gfd_server_*: a resident graph serving validation requests with
    continuous batching.  submit() returns a request id; wait() returns the
    request's result dicts (as validate() gives them) and its timing info."""

    def __init__(self, graph: GraphHandle, K: int = 1024, semantics: str = "induced",
                 workers: int = 2, max_batch_gfds: int = 256, mem_budget_bytes: int = 0,
                 allocator="torch"):
        self.graph, self.K = graph, int(K)
        self.handle = None
        ca, alloc = _allocator(allocator)
        graph.keep(alloc)
        opts = gfd_server_opts(int(workers), int(max_batch_gfds), int(mem_budget_bytes), self.K,
                               GFD_SEM_INDUCED if semantics == "induced" else GFD_SEM_MONO, ca)
        h = C.c_void_p()
        _check(lib.gfd_server_create(graph.handle, C.byref(opts), C.byref(h)))
        self.handle = h
        self.pending = {}

    def submit(self, gfds) -> int:
        n = len(gfds)
        specs = (gfd_spec * max(n, 1))(*[make_spec(d) for d in gfds])
        rid = C.c_uint64()
        _check(lib.gfd_server_submit(self.handle, specs, n, C.byref(rid)))
        self.pending[rid.value] = [int(d["k"]) for d in gfds]
        return rid.value

    def wait(self, rid: int, timeout_ms: int = -1):
        """(results, info) once the request is done; None if not done within
        timeout_ms (timeout_ms < 0: wait as long as it takes)."""
        ks = self.pending.get(rid)
        if ks is None:  # not submitted here: the library reports it
            _check(lib.gfd_server_wait(self.handle, rid, int(timeout_ms), None, None))
            raise GfdError(GFD_EINVAL, f"request {rid} unknown")
        n = len(ks)
        res = (gfd_result * n)()
        bufs = []
        for i, k in enumerate(ks):
            b = np.zeros(max(1, self.K * k), dtype=np.int32)
            bufs.append(b)
            res[i].violations = b.ctypes.data_as(C.POINTER(C.c_int32))
        info = gfd_request_info()
        rc = lib.gfd_server_wait(self.handle, rid, int(timeout_ms), res, C.byref(info))
        if rc == GFD_EAGAIN:
            return None
        del self.pending[rid]
        _check(rc)
        out = []
        for i, k in enumerate(ks):
            r = res[i]
            out.append({"match_count": int(r.match_count), "violation_count": int(r.violation_count),
                        "match_fp": int(r.match_fp), "violation_fp": int(r.violation_fp),
                        "satisfied": bool(r.satisfied),
                        "violations": bufs[i][:r.num_reported * k].reshape(-1, k).tolist()})
        return out, {f: getattr(info, f) for f, _ in gfd_request_info._fields_}

    def close(self):
        h = getattr(self, "handle", None)
        if h and lib is not None:
            lib.gfd_server_destroy(h)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
