"""Seeded GFD samplers (patterns plus X -> Y literals) over a synthetic graph.

A GFD (Section II) is a pattern Q[x] -- vertex labels in variable order x, and
directed labelled edges -- plus a dependency X -> Y (or X -> false) made of
constant literals x_i.A = c and variable literals x_i.A = x_j.B.

Representation (plain JSON-able dicts, read by both the oracle and the GPU
binding):

    {"k": 3, "vlabels": [0, 1, 1],            # -1 = wildcard
     "edges": [[0, 1, 0], [0, 2, 0]],         # [src, dst, label]; label -1 = any
     "x": [...], "y": [...], "y_false": False}
    literal: {"kind": "const", "var": i, "attr": a, "value": c}
          or {"kind": "var", "var": i, "attr": a, "var2": j, "attr2": b}

Patterns are cut from the graph itself: a seeded search or random walk picks a
vertex set S, and the pattern is the subgraph S induces, with its labels and
edge directions.  That occurrence is then a match under both the induced and
the non-induced reading, so results are non-empty.

The only arithmetic here is the sampler's own size cap: an upper bound on the
number of homomorphisms of a spanning tree of the pattern (a tree dynamic
program over label-restricted sparse adjacency), used to reject patterns whose
exhaustive enumeration would take too long on a CPU.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .graphs import Graph, in_csr, draw_codes

U_MAX_DEFAULT = 1e8


class GraphView:
    """Out/in adjacency plus per-edge-label sparse matrices for sampling."""

    def __init__(self, g: Graph):
        self.g = g
        self.in_ptr, self.in_src, self.in_lab = in_csr(g)
        self._mats = None

    def out_row(self, v):
        a, b = self.g.row_ptr[v], self.g.row_ptr[v + 1]
        return self.g.col[a:b]

    def in_row(self, v):
        a, b = self.in_ptr[v], self.in_ptr[v + 1]
        return self.in_src[a:b]

    def skel(self, v):
        return np.union1d(self.out_row(v), self.in_row(v))

    def edge_label(self, a, b):
        """Label of edge a->b, or None if absent."""
        lo, hi = self.g.row_ptr[a], self.g.row_ptr[a + 1]
        i = lo + np.searchsorted(self.g.col[lo:hi], b)
        if i < hi and self.g.col[i] == b:
            return int(self.g.elabel[i])
        return None

    def adjacent(self, a, b):
        return self.edge_label(a, b) is not None or self.edge_label(b, a) is not None

    def mats(self):
        """Per edge label: (A_l, A_l^T) as float64 CSR, A_l[u, v] = 1 iff u->v has label l."""
        if self._mats is None:
            g = self.g
            src = g.src()
            L = int(g.elabel.max()) + 1 if g.m else 0
            self._mats = {}
            for lab in range(L):
                sel = g.elabel == lab
                A = sp.csr_matrix((np.ones(int(sel.sum())), (src[sel], g.col[sel])), shape=(g.n, g.n))
                self._mats[lab] = (A, A.T.tocsr())
        return self._mats


def induced_pattern(view: GraphView, S) -> dict:
    """Pattern = subgraph induced by the vertex list S (variables in S order)."""
    g = view.g
    edges = []
    for i, a in enumerate(S):
        for j, b in enumerate(S):
            if i != j:
                lab = view.edge_label(a, b)
                if lab is not None:
                    edges.append([i, j, lab])
    return {"k": len(S), "vlabels": [int(g.vlabel[v]) for v in S], "edges": edges,
            "x": [], "y": [], "y_false": False}


def skeleton_pairs(p: dict):
    return sorted({(min(s, d), max(s, d)) for s, d, _ in p["edges"]})


def two_core(k: int, pairs) -> list[int]:
    """Vertices of the 2-core of an undirected graph (peel degree <= 1)."""
    adj = {i: set() for i in range(k)}
    for a, b in pairs:
        adj[a].add(b)
        adj[b].add(a)
    alive = set(range(k))
    changed = True
    while changed:
        changed = False
        for v in list(alive):
            if len(adj[v] & alive) <= 1:
                alive.discard(v)
                changed = True
    return sorted(alive)


def tree_hom_bound(view: GraphView, p: dict, prefix_sum: bool = True) -> float:
    """Upper bound on the exhaustive search size for pattern p.

    Uses the spanning tree in which each variable i > 0 hangs off its first
    earlier neighbour (the order a plain backtracking search in variable order
    extends along).  Returns the sum over prefixes 0..j of the number of
    label-respecting homomorphisms of that prefix tree (one edge direction per
    tree edge), or just the full tree's count when prefix_sum is False.
    """
    g = view.g
    k = p["k"]
    adj = {}
    for s, d, lab in p["edges"]:
        adj.setdefault((s, d), lab)
    parent = [-1] * k
    via = [None] * k
    for i in range(1, k):
        for j in range(i):
            if (j, i) in adj:
                parent[i], via[i] = j, ("out", adj[(j, i)])
                break
            if (i, j) in adj:
                parent[i], via[i] = j, ("in", adj[(i, j)])
                break
        if parent[i] < 0:
            return float("inf")  # disconnected: not produced by the samplers
    mats = view.mats()
    ind = {}

    def label_vec(L):
        if L not in ind:
            ind[L] = np.ones(g.n) if L < 0 else (g.vlabel == L).astype(np.float64)
        return ind[L]

    def count(last):
        f = [None] * (last + 1)
        for u in range(last, -1, -1):
            v = label_vec(p["vlabels"][u]).copy()
            for c in range(u + 1, last + 1):
                if parent[c] == u:
                    d, lab = via[c]
                    if lab < 0:
                        M = sum((mats[l][0] if d == "out" else mats[l][1]) for l in mats)
                    else:
                        if lab not in mats:
                            return 0.0
                        M = mats[lab][0] if d == "out" else mats[lab][1]
                    v *= M @ f[c]
            f[u] = v
        return float(f[0].sum())

    if not prefix_sum:
        return count(k - 1)
    return sum(count(j) for j in range(k))


def _attr_draw(rng, g: Graph, a: int, zipf_s, attr_values):
    return int(draw_codes(rng, attr_values, 1, zipf_s)[0])


def add_literals(rng, g: Graph, p: dict, S, lo: int, hi: int, attr_values: int, attr_zipf):
    """t ~ U[lo, hi] literals; t = 1 -> X = {}, Y = {l}; t >= 2 -> X = {l1}, Y = rest."""
    k, A = p["k"], g.num_attrs
    t = int(rng.integers(lo, hi + 1))
    lits = []
    for _ in range(t):
        if A == 0:
            break
        if rng.random() < 0.5 or k == 1:
            i = int(rng.integers(0, k))
            a = int(rng.integers(0, A))
            if rng.random() < 0.5:
                c = int(g.attrs[a, S[i]])
            else:
                c = _attr_draw(rng, g, a, attr_zipf, attr_values)
            if c < 0:
                c = 0
            lits.append({"kind": "const", "var": i, "attr": a, "value": c})
        else:
            i, j = (int(z) for z in rng.choice(k, size=2, replace=False))
            lits.append({"kind": "var", "var": i, "attr": int(rng.integers(0, A)),
                         "var2": j, "attr2": int(rng.integers(0, A))})
    if len(lits) == 1:
        p["x"], p["y"] = [], lits
    elif lits:
        p["x"], p["y"] = lits[:1], lits[1:]
    return p


# ----------------------------------------------------------------------------
# Shape-driven search (paths, stars, triangles and 4-cycles with pendants)
# ----------------------------------------------------------------------------

def shape_edges(rng, shape: str, k: int):
    """Undirected skeleton of a named shape on variables 0..k-1, each variable
    after 0 adjacent to an earlier one."""
    if shape == "path":
        return [(i, i + 1) for i in range(k - 1)]
    if shape == "star":
        return [(0, i) for i in range(1, k)]
    if shape == "triangle":
        e = [(0, 1), (1, 2), (0, 2)]
        base = 3
    elif shape == "cycle4":
        e = [(0, 1), (1, 2), (2, 3), (0, 3)]
        base = 4
    else:
        raise ValueError(shape)
    for i in range(base, k):
        e.append((int(rng.integers(0, i)), i))
    return e


def find_shape_occurrence(rng, view: GraphView, k: int, pairs, tries: int = 10_000):
    """Seeded search for a vertex set whose induced skeleton is exactly `pairs`."""
    g = view.g
    nbrs = {i: set() for i in range(k)}
    for a, b in pairs:
        nbrs[a].add(b)
        nbrs[b].add(a)
    src_of_edge = g.src()
    for _ in range(tries):
        e = int(rng.integers(0, g.m))
        S = [int(src_of_edge[e]) if rng.random() < 0.5 else int(g.col[e])]
        ok = True
        for i in range(1, k):
            earlier_nb = [j for j in sorted(nbrs[i]) if j < i]
            cand = view.skel(S[earlier_nb[0]])
            for j in earlier_nb[1:]:
                cand = np.intersect1d(cand, view.skel(S[j]), assume_unique=True)
            cand = np.setdiff1d(cand, np.array(S))
            if cand.size == 0:
                ok = False
                break
            if cand.size > 64:
                cand = rng.choice(cand, size=64, replace=False)
            picked = None
            for c in rng.permutation(cand):
                c = int(c)
                if all(not view.adjacent(c, S[j]) for j in range(i) if j not in nbrs[i]):
                    picked = c
                    break
            if picked is None:
                ok = False
                break
            S.append(picked)
        if ok:
            return S
    return None


def sample_shape_gfd(rng, view: GraphView, shape: str, k: int, lit_range, attr_values, attr_zipf,
                     u_max=U_MAX_DEFAULT, tries=10_000, label_zipf=None, n_vlabels=1, n_elabels=1):
    pairs = shape_edges(rng, shape, k)
    for _ in range(20):
        S = find_shape_occurrence(rng, view, k, pairs, tries=tries // 20)
        if S is None:
            continue
        p = induced_pattern(view, S)
        if tree_hom_bound(view, p) <= u_max:
            p = add_literals(rng, view.g, p, S, lit_range[0], lit_range[1], attr_values, attr_zipf)
            p["meta"] = {"shape": shape, "source": S, "found": True}
            return p
    # No occurrence: labels by Zipf and one direction per skeleton pair; the
    # result may be empty (recorded in meta).
    vl = draw_codes(rng, n_vlabels, k, label_zipf)
    el = draw_codes(rng, n_elabels, len(pairs), label_zipf)
    p = {"k": k, "vlabels": [int(x) for x in vl],
         "edges": [[a, b, int(l)] for (a, b), l in zip(pairs, el)],
         "x": [], "y": [], "y_false": False}
    S = [0] * k
    p = add_literals(rng, view.g, p, S, lit_range[0], lit_range[1], attr_values, attr_zipf)
    p["meta"] = {"shape": shape, "found": False}
    return p


# ----------------------------------------------------------------------------
# Random-walk patterns
# ----------------------------------------------------------------------------

def random_walk_set(rng, view: GraphView, k: int, max_steps: int = 2000):
    g = view.g
    deg_out = np.diff(g.row_ptr)
    while True:
        e = int(rng.integers(0, g.m))
        v0 = int(g.col[e]) if rng.random() < 0.5 else int(np.searchsorted(g.row_ptr, e, side="right") - 1)
        if deg_out[v0] + (view.in_ptr[v0 + 1] - view.in_ptr[v0]) > 0:
            break
    S = [v0]
    cur = v0
    for _ in range(max_steps):
        if len(S) == k:
            return S
        nb = view.skel(cur)
        cur = int(nb[rng.integers(0, nb.size)])
        if cur not in S:
            S.append(cur)
    return None


def cyclomatic(p: dict) -> int:
    return len(skeleton_pairs(p)) - p["k"] + 1


def sample_walk_gfd(rng, view: GraphView, k_range, lit_range, attr_values, attr_zipf, *,
                    core_range=None, cyc_range=None, u_max=U_MAX_DEFAULT, max_tries=5000):
    """Random-walk GFD: k ~ U[k_range]; accept by 2-core size or cyclomatic number."""
    for _ in range(max_tries):
        k = int(rng.integers(k_range[0], k_range[1] + 1))
        S = random_walk_set(rng, view, k)
        if S is None:
            continue
        p = induced_pattern(view, S)
        pairs = skeleton_pairs(p)
        if core_range is not None:
            c = len(two_core(k, pairs))
            if not (core_range[0] <= c <= core_range[1]) or c == k:
                continue
        if cyc_range is not None:
            c = cyclomatic(p)
            if not (cyc_range[0] <= c <= cyc_range[1]):
                continue
        if tree_hom_bound(view, p) > u_max:
            continue
        p = add_literals(rng, view.g, p, S, lit_range[0], lit_range[1], attr_values, attr_zipf)
        p["meta"] = {"source": S, "cyclomatic": cyclomatic(p),
                     "core": len(two_core(k, pairs))}
        return p
    raise RuntimeError("walk sampler: no acceptable pattern")
