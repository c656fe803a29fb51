"""Seeded synthetic data graphs for GFD validation workloads.

These generators only draw random inputs: vertices, directed edges, vertex and
edge labels and dictionary-encoded int32 attribute columns.  They implement none
of the validation method.  Both the GPU path and the CPU oracle read the arrays
produced here; neither is consulted to make them.

Graph model (Section II): a directed graph whose edge set is a subset of V x V,
so there is at most one edge per ordered pair; every vertex and every edge
carries one label; attributes live on vertices only.  Self-loops are never
emitted.

Random numbers: numpy PCG64 with ``SeedSequence(seed).spawn(5)`` sub-streams in
this fixed order: edges, vertex labels, edge labels, attributes, GFDs.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

ABSENT = -1  # attribute value meaning "this vertex has no such attribute"


@dataclass
class Graph:
    n: int
    m: int
    row_ptr: np.ndarray  # int64 [n+1], out-CSR, rows sorted by target id
    col: np.ndarray  # int32 [m]
    vlabel: np.ndarray  # int32 [n]
    elabel: np.ndarray  # int32 [m], aligned with col
    attrs: np.ndarray  # int32 [A, n]; ABSENT (-1) = missing
    meta: dict = field(default_factory=dict)

    @property
    def num_attrs(self) -> int:
        return int(self.attrs.shape[0])

    def src(self) -> np.ndarray:
        """Source vertex of every edge, aligned with ``col``."""
        return np.repeat(np.arange(self.n, dtype=np.int32), np.diff(self.row_ptr)).astype(np.int32)

    def sha256(self) -> str:
        h = hashlib.sha256()
        for a in (np.int64(self.n), np.int64(self.m), self.row_ptr, self.col,
                  self.vlabel, self.elabel, self.attrs):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()


def sub_streams(seed: int) -> dict:
    ss = np.random.SeedSequence(seed).spawn(5)
    names = ("edges", "vlabels", "elabels", "attrs", "gfds")
    return {nm: np.random.Generator(np.random.PCG64(s)) for nm, s in zip(names, ss)}


def zipf_probs(N: int, s: float) -> np.ndarray:
    """P(code r-1) proportional to r^-s for r = 1..N (code 0 most frequent)."""
    r = np.arange(1, N + 1, dtype=np.float64)
    p = r ** (-s)
    return p / p.sum()


def draw_codes(rng: np.random.Generator, N: int, size: int, zipf_s: float | None) -> np.ndarray:
    if zipf_s is None:
        return rng.integers(0, N, size=size, dtype=np.int64).astype(np.int32)
    cdf = np.cumsum(zipf_probs(N, zipf_s))
    cdf[-1] = 1.0
    return np.searchsorted(cdf, rng.random(size), side="right").astype(np.int32)


def _distinct_pairs(rng, n: int, m: int, draw_batch) -> np.ndarray:
    """Draw ordered pairs until exactly m distinct non-loop pairs exist.

    Pairs are kept in order of first occurrence; later repeats are rejected.
    Returns the kept pairs encoded as int64 keys src*n+dst (unsorted).
    """
    kept = np.empty(0, dtype=np.int64)
    while kept.size < m:
        need = m - kept.size
        s, d = draw_batch(int(need * 1.25) + 1024)
        ok = s != d
        keys = np.concatenate([kept, s[ok].astype(np.int64) * n + d[ok].astype(np.int64)])
        _, first = np.unique(keys, return_index=True)
        first.sort()
        kept = keys[first]
    return kept[:m]


def _csr_from_keys(keys: np.ndarray, n: int):
    keys = np.sort(keys)
    src = keys // n
    dst = (keys % n).astype(np.int32)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=row_ptr[1:])
    return row_ptr, dst


def uniform_edges(rng, n: int, m: int) -> np.ndarray:
    def draw(b):
        return rng.integers(0, n, size=b), rng.integers(0, n, size=b)
    return _distinct_pairs(rng, n, m, draw)


def chung_lu_weights(n: int, m: int, gamma: float) -> np.ndarray:
    """Expected degrees w_i ~ (i+1)^(-1/(gamma-1)), scaled to sum m, capped at sqrt(m)."""
    w = np.arange(1, n + 1, dtype=np.float64) ** (-1.0 / (gamma - 1.0))
    w *= m / w.sum()
    return np.minimum(w, np.sqrt(m))


def chung_lu_edges(rng, n: int, m: int, gamma: float) -> np.ndarray:
    """Directed Chung-Lu: source ~ w_out, target ~ w_in, independent vertex permutations."""
    w = chung_lu_weights(n, m, gamma)
    w_out = w[rng.permutation(n)]
    w_in = w[rng.permutation(n)]
    c_out = np.cumsum(w_out)
    c_in = np.cumsum(w_in)
    t_out, t_in = c_out[-1], c_in[-1]

    def inverse_cdf(c, total, b):
        # searchsorted on sorted queries is cache friendly; scatter back to draw order
        r = rng.random(b) * total
        order = np.argsort(r, kind="stable")
        out = np.empty(b, dtype=np.int64)
        out[order] = np.searchsorted(c, r[order], side="right")
        return np.minimum(out, n - 1)

    def draw(b):
        s = inverse_cdf(c_out, t_out, b)
        d = inverse_cdf(c_in, t_in, b)
        return s, d
    return _distinct_pairs(rng, n, m, draw)


def chung_lu_symmetric_pairs(rng, n: int, m_pairs: int, gamma: float) -> np.ndarray:
    """Undirected Chung-Lu: both endpoints ~ w (one permutation), expected degree
    w_i (capped at sqrt of the directed edge count); returns m_pairs distinct
    unordered pairs as keys min*n+max, in order of first occurrence."""
    w = chung_lu_weights(n, 2 * m_pairs, gamma)[rng.permutation(n)]
    c = np.cumsum(w)
    t = c[-1]

    def inverse_cdf(b):
        r = rng.random(b) * t
        order = np.argsort(r, kind="stable")
        out = np.empty(b, dtype=np.int64)
        out[order] = np.searchsorted(c, r[order], side="right")
        return np.minimum(out, n - 1)

    def draw(b):
        a, z = inverse_cdf(b), inverse_cdf(b)
        return np.minimum(a, z), np.maximum(a, z)
    return _distinct_pairs(rng, n, m_pairs, draw)


def make_graph(seed: int, n: int, m: int, *, model: str, n_vlabels: int, n_elabels: int,
               label_zipf: float | None, n_attrs: int, attr_values: int,
               attr_zipf: float | None, gamma: float = 2.1,
               absent_frac: float = 0.0) -> tuple[Graph, np.random.Generator]:
    """Build one graph; returns it with the (unused) GFD sub-stream."""
    rs = sub_streams(seed)
    if model == "chung_lu_sym":
        # every undirected pair becomes two antiparallel edges with one label
        if m % 2:
            raise ValueError("a symmetric graph has an even edge count")
        pairs = chung_lu_symmetric_pairs(rs["edges"], n, m // 2, gamma)
        plab = draw_codes(rs["elabels"], n_elabels, m // 2, label_zipf)
        lo, hi = pairs // n, pairs % n
        keys = np.concatenate([lo * n + hi, hi * n + lo])
        labs = np.concatenate([plab, plab])
        order = np.argsort(keys, kind="stable")
        keys, elabel = keys[order], labs[order].astype(np.int32)
        row_ptr, col = _csr_from_keys(keys, n)
    else:
        if model == "uniform":
            keys = uniform_edges(rs["edges"], n, m)
        elif model == "chung_lu":
            keys = chung_lu_edges(rs["edges"], n, m, gamma)
        else:
            raise ValueError(model)
        row_ptr, col = _csr_from_keys(keys, n)
        elabel = draw_codes(rs["elabels"], n_elabels, m, label_zipf)
    vlabel = draw_codes(rs["vlabels"], n_vlabels, n, label_zipf)
    attrs = np.empty((n_attrs, n), dtype=np.int32)
    for a in range(n_attrs):
        attrs[a] = draw_codes(rs["attrs"], attr_values, n, attr_zipf)
    if absent_frac > 0:
        holes = rs["attrs"].random((n_attrs, n)) < absent_frac
        attrs[holes] = ABSENT
    meta = dict(seed=seed, n=n, m=m, model=model, n_vlabels=n_vlabels, n_elabels=n_elabels,
                label_zipf=label_zipf, n_attrs=n_attrs, attr_values=attr_values,
                attr_zipf=attr_zipf, gamma=gamma if model.startswith("chung_lu") else None,
                degree_cap=float(np.sqrt(m)) if model.startswith("chung_lu") else None,
                absent_frac=absent_frac)
    g = Graph(n=n, m=m, row_ptr=row_ptr, col=col, vlabel=vlabel, elabel=elabel,
              attrs=attrs, meta=meta)
    return g, rs["gfds"]


def from_edge_list(n: int, edges, vlabel, attrs=None) -> Graph:
    """Small hand-built graphs: edges = [(src, dst, label), ...]."""
    edges = sorted((int(s), int(d), int(l)) for s, d, l in edges)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    for s, _, _ in edges:
        row_ptr[s + 1] += 1
    row_ptr = np.cumsum(row_ptr).astype(np.int64)
    col = np.array([d for _, d, _ in edges], dtype=np.int32)
    elabel = np.array([l for _, _, l in edges], dtype=np.int32)
    vlabel = np.asarray(vlabel, dtype=np.int32)
    if attrs is None:
        attrs = np.zeros((0, n), dtype=np.int32)
    attrs = np.asarray(attrs, dtype=np.int32).reshape(-1, n)
    return Graph(n=n, m=len(edges), row_ptr=row_ptr, col=col, vlabel=vlabel,
                 elabel=elabel, attrs=attrs, meta={"model": "hand"})


def in_csr(g: Graph):
    """Transpose: (in_ptr, in_src, in_elabel), rows sorted by source id."""
    src = g.src()
    order = np.lexsort((src, g.col))
    in_ptr = np.zeros(g.n + 1, dtype=np.int64)
    np.cumsum(np.bincount(g.col, minlength=g.n), out=in_ptr[1:])
    return in_ptr, src[order].astype(np.int32), g.elabel[order].astype(np.int32)
