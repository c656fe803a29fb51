"""gfd_validate_noalloc: the entry point that allocates nothing (its device
memory is the library's fixed scratch area).  Through the C ABI, its results
equal gfd_validate's on the same inputs, element by element, over two calls
in a row (the second smaller), on the 1M-vertex power-law workload and on
random graphs; a call that does not fit the area fails with GFD_ENOMEM and
the next call still works."""
import numpy as np
import pytest

from synth import configs
from synth.graphs import Graph
from synth.small import random_graph, random_gfd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2608_02321_amd as P
    return P


def _gfds(seed, count, n_vlabels=2):
    rng = np.random.default_rng(seed)
    return [random_gfd(seed * 100 + j, int(rng.integers(1, 7)), n_vlabels=n_vlabels, n_elabels=2,
                       n_attrs=2, attr_values=4, wildcard_frac=0.15, extra_edge_frac=0.3)
            for j in range(count)]


def _same(P, gh, gfds, **kw):
    ref = P.validate(gh, gfds, allocator=None, **kw)
    got = P.validate(gh, gfds, noalloc=True, **kw)
    assert got == ref, kw
    return got


def test_noalloc_matches_validate_twice(P):
    big = random_graph(31, 3000, 40000, n_vlabels=2, n_elabels=2, n_attrs=2, attr_values=4,
                       absent_frac=0.1)
    small = random_graph(32, 400, 3000, n_vlabels=2, n_elabels=2, n_attrs=2, attr_values=4,
                         absent_frac=0.1)
    gb, gs = P.load(big, allocator=None), P.load(small, allocator=None)
    for sem in ("induced", "mono"):
        # first call: 24 GFDs in one batch; second: 3 GFDs on the small graph
        _same(P, gb, _gfds(31, 24), K=64, semantics=sem, batched=True)
        _same(P, gs, _gfds(32, 3), K=16, semantics=sem)
        # and back, one GFD at a time, then the bounded path and staging overflow
        _same(P, gb, _gfds(33, 6), K=32, semantics=sem, batched=False)
        _same(P, gs, _gfds(34, 4), K=8, semantics=sem, flags=P.GFD_FLAG_FORCE_CHUNKED)
        _same(P, gb, _gfds(35, 5), K=16, semantics=sem, violation_cap=40, batched=True)
        # count-only: postponed leaves, and (K > 0) their first-K windows
        _same(P, gb, _gfds(36, 12), K=0, semantics=sem, flags=P.GFD_FLAG_COUNT_ONLY,
              batched=True)
        _same(P, gb, _gfds(36, 12), K=24, semantics=sem, flags=P.GFD_FLAG_COUNT_ONLY,
              batched=True)
    gb.free()
    gs.free()


def test_noalloc_full_size_powerlaw(P):
    """The 1M-vertex / 5M-edge workload's 8 GFDs, batched then one GFD."""
    g = configs.graph("powerlaw_1m")
    gfds = [{k: v for k, v in d.items() if k != "meta"} for d in configs.gfds("powerlaw_1m", g)]
    gh = P.load(g, allocator=None)
    _same(P, gh, gfds, K=1024, semantics="induced", batched=True)
    _same(P, gh, gfds[:1], K=1024, semantics="induced")
    gh.free()


def test_noalloc_area_exhausted_then_recovers(P):
    """Eight wildcard vertices over 4M vertices need candidate lists of 16 MB
    each, beyond the area: GFD_ENOMEM, and the next, smaller call is exact."""
    n, m = 4_000_000, 2_000_000
    rng = np.random.default_rng(36)
    src = np.sort(rng.integers(0, n, size=m))
    dst = (src + 1 + rng.integers(0, n - 1, size=m)) % n
    pairs = np.unique(np.stack([src, dst], 1), axis=0)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(pairs[:, 0], minlength=n), out=row_ptr[1:])
    g = Graph(n=n, m=len(pairs), row_ptr=row_ptr, col=pairs[:, 1].astype(np.int32),
              vlabel=np.zeros(n, dtype=np.int32), elabel=np.zeros(len(pairs), dtype=np.int32),
              attrs=np.zeros((1, n), dtype=np.int32), meta={"model": "hand"})
    gh = P.load(g, allocator=None)
    path8 = {"k": 8, "vlabels": [-1] * 8, "edges": [[i, i + 1, -1] for i in range(7)],
             "x": [], "y": [], "y_false": True}
    with pytest.raises(P.GfdError) as ei:
        P.validate(gh, [path8], K=4, noalloc=True)
    assert ei.value.code == -2 and "scratch" in P.last_error()
    edge = {"k": 2, "vlabels": [0, 0], "edges": [[0, 1, 0]], "x": [], "y": [], "y_false": True}
    r = _same(P, gh, [edge], K=4)
    assert r[0]["match_count"] == len(pairs) - int(np.isin(
        pairs[:, 0] * n + pairs[:, 1], pairs[:, 1] * n + pairs[:, 0]).sum())
    gh.free()
