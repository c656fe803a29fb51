"""MI355X (gfx950) GFD validation: Compact Path Index construction, core-first
embedding enumeration and the fused X -> Y literal check, as HIP kernels
behind the C ABI in include/gfd.h.  This package is the thin Python binding.
"""
from ._binding import (GFD_ABSENT, GFD_FLAG_COUNT_ONLY, GFD_FLAG_FORCE_CHUNKED, GFD_FLAG_NO_GRAPH,
                       GFD_FLAG_TIMING, GFD_MAX_K,
                       GFD_MEM_DEVICE, GFD_MEM_HOST, GFD_SEM_INDUCED, GFD_SEM_MONO, GFD_WILDCARD, GfdError,
                       GraphHandle, PreparedCall, Server, TorchAllocator, free_graph, last_error, load,
                       load_graph, make_spec, torch_allocator, validate, version)

__all__ = ["GFD_ABSENT", "GFD_FLAG_COUNT_ONLY", "GFD_FLAG_FORCE_CHUNKED", "GFD_FLAG_NO_GRAPH", "GFD_FLAG_TIMING", "GFD_MAX_K",
           "GFD_MEM_DEVICE", "GFD_MEM_HOST", "GFD_SEM_INDUCED", "GFD_SEM_MONO", "GFD_WILDCARD", "GfdError",
           "GraphHandle", "PreparedCall", "Server", "TorchAllocator", "free_graph", "last_error", "load",
           "load_graph", "make_spec", "torch_allocator", "validate", "version"]
