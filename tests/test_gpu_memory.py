"""Device memory at the C ABI, on the GPU: inputs that are already device
tensors (mem_kind GFD_MEM_DEVICE), device memory from caller callbacks
(torch's caching allocator), allocation failure reported as GFD_ENOMEM, the
frontier pool and CPI arena growing to what a batch asks for, and gfd_trim.
Every result is checked against the CPU oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from synth.small import random_graph, random_gfd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2608_02321_amd as P
    return P


def _case(seed=21):
    rng = np.random.default_rng(seed)
    g = random_graph(seed, 1500, 15000, n_vlabels=2, n_elabels=2, n_attrs=2, attr_values=4,
                     absent_frac=0.1)
    gfds = [random_gfd(seed * 100 + j, int(rng.integers(1, 7)), n_vlabels=2, n_elabels=2,
                       n_attrs=2, attr_values=4, wildcard_frac=0.15, extra_edge_frac=0.3)
            for j in range(12)]
    return g, gfds


def _oracle(g, gfds, sem, K):
    og = O.OracleGraph(g)
    return [O.validate(og, d, sem, K=K, threads=4) for d in gfds]


def test_device_inputs_through_torch_allocator(P):
    """The graph comes from torch device tensors and every device byte of the
    graph and of the workspaces from a torch allocator: results equal the
    oracle's and the host-input load's; trim returns the workspaces and free
    the graph, so the allocator ends with every block returned."""
    import torch
    g, gfds = _case()
    dev = torch.device("cuda")
    ta = P.TorchAllocator()
    gh = P.load_graph(g.n, g.m, torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev),
                      torch.from_numpy(g.vlabel).to(dev), torch.from_numpy(g.elabel).to(dev),
                      torch.from_numpy(np.ascontiguousarray(g.attrs)).to(dev), allocator=ta)
    graph_bytes = gh.info["device_bytes"]
    assert ta.allocs > 0 and ta.live_bytes == graph_bytes
    host = P.load(g, allocator=None)  # the same graph from host arrays, hipMalloc
    for sem in ("induced", "mono"):
        exp = _oracle(g, gfds, sem, 40)
        for batched in (False, True):
            assert P.validate(gh, gfds, K=40, semantics=sem, batched=batched, allocator=ta) == exp
            assert P.validate(host, gfds, K=40, semantics=sem, batched=batched, allocator=None) == exp
    assert ta.live_bytes > graph_bytes  # a workspace is kept between calls
    assert torch.cuda.memory_allocated() >= ta.live_bytes
    gh.trim()
    assert ta.live_bytes == graph_bytes
    gh.free()
    host.free()
    assert ta.live_bytes == 0 and ta.allocs == ta.frees


class _FailingAllocator:
    """Torch-backed callbacks that refuse every allocation after `ok` of them."""

    def __init__(self, P, ok):
        self.inner, self.ok, self.refused = P.TorchAllocator(), ok, 0
        self._alloc = P._binding.ALLOC_FN(self._on_alloc)
        self.c = P._binding.gfd_allocator(self._alloc, self.inner._free, None)

    def _on_alloc(self, ctx, nbytes, stream):
        if self.inner.allocs >= self.ok:
            self.refused += 1
            return None
        return self.inner._on_alloc(ctx, nbytes, stream)


def test_allocation_failure_is_enomem(P):
    g, gfds = _case(22)
    for ok in (0, 3):  # refused at the first and at the fourth block of the load
        fa = _FailingAllocator(P, ok)
        with pytest.raises(P.GfdError) as ei:
            P.load(g, allocator=fa)
        assert ei.value.code == -2 and fa.refused == 1
        assert fa.inner.live_bytes == 0  # what the load got was returned
    gh = P.load(g, allocator=None)
    fa = _FailingAllocator(P, 2)  # a workspace needs more than two blocks
    with pytest.raises(P.GfdError) as ei:
        P.validate(gh, gfds, K=8, allocator=fa)
    assert ei.value.code == -2
    gh.keep(fa)
    # the graph still works, with other memory
    assert P.validate(gh, gfds, K=8, allocator=None) == _oracle(g, gfds, "induced", 8)
    gh.free()
    assert fa.inner.live_bytes == 0


def _hub_graph(seed=23, n=2000, hubs=20, hub_deg=200, low_deg=3):
    """Hubs with hub_deg out- and hub_deg in-neighbours among mostly low-degree
    vertices: paths through a hub are many more than the mean degree
    predicts."""
    from synth import from_edge_list
    rng = np.random.default_rng(seed)
    es = set()
    for h in range(hubs):
        for v in rng.choice(n, size=hub_deg, replace=False):
            if v != h:
                es.add((h, int(v)))
        for v in rng.choice(n, size=hub_deg, replace=False):
            if v != h:
                es.add((int(v), h))
    for u in range(hubs, n):
        for v in rng.choice(n, size=low_deg, replace=False):
            if v != u:
                es.add((u, int(v)))
    attrs = rng.integers(0, 20, size=(1, n))
    return from_edge_list(n, [(a, b, 0) for a, b in es], np.zeros(n, dtype=np.int32), attrs)


def test_frontier_pool_grows_to_the_batch(P):
    """A fresh workspace's frontier pool is sized by a mean-fan-out estimate,
    which degree skew defeats: a call whose frontiers need more runs those
    GFDs again in the fast path once the pool has grown, and the next call
    needs no regrowth.  Results never change."""
    g = _hub_graph()
    path4 = {"k": 4, "vlabels": [-1] * 4, "edges": [[0, 1, -1], [1, 2, -1], [2, 3, -1]],
             "x": [], "y": [{"kind": "var", "var": 0, "attr": 0, "var2": 3, "attr2": 0}],
             "y_false": False}
    gfds = [path4, random_gfd(2301, 3, n_vlabels=1, n_elabels=1, n_attrs=1, attr_values=20)]
    gh = P.load(g)
    ta = P.TorchAllocator()
    exp = _oracle(g, gfds, "mono", 16)
    # the pool starts at a sixteenth of the budget (16 MiB; the estimate is
    # about 3 MB) and may grow to a quarter (64 MiB); the path's second
    # frontier takes about 20 MB
    budget = 256 << 20
    got, st = P.validate(gh, gfds, K=16, semantics="mono", batched=True, stats=True,
                         mem_budget_bytes=budget, allocator=ta)
    assert got == exp
    assert st["regrown_gfds"] >= 1 and st["chunked_gfds"] == 0
    assert (16 << 20) < st["front_pool_bytes"] <= (64 << 20)
    got, st2 = P.validate(gh, gfds, K=16, semantics="mono", batched=True, stats=True,
                          mem_budget_bytes=budget, allocator=ta)
    assert got == exp and st2["regrown_gfds"] == 0
    assert st2["front_pool_bytes"] == st["front_pool_bytes"]
    gh.free()
    assert ta.live_bytes == 0


def test_budget_below_the_minimum_is_enomem(P):
    """A memory budget below 64 MiB is refused with GFD_ENOMEM before any
    launch, and the graph serves the next call exactly."""
    g, gfds = _case(23)
    gh = P.load(g)
    with pytest.raises(P.GfdError) as ei:
        P.validate(gh, gfds, K=16, batched=True, mem_budget_bytes=32 << 20)
    assert ei.value.code == -2 and "64 MiB" in P.last_error()  # GFD_ENOMEM
    got = P.validate(gh, gfds, K=16, batched=True, mem_budget_bytes=64 << 20)
    assert got == _oracle(g, gfds, "induced", 16)
    gh.free()
