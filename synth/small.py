"""Small seeded random graphs and GFDs for tests (any pattern shape, wildcards,
missing attributes, X -> false).  Input generation only."""
from __future__ import annotations

import numpy as np

from .graphs import Graph, ABSENT, _csr_from_keys


def random_graph(seed: int, n: int, m: int, n_vlabels: int = 3, n_elabels: int = 2,
                 n_attrs: int = 2, attr_values: int = 3, absent_frac: float = 0.2,
                 reciprocal_frac: float = 0.3) -> Graph:
    """Uniform random simple digraph; a fraction of edges gets its reverse added."""
    rng = np.random.default_rng(seed)
    m = min(m, n * (n - 1))
    keys = set()
    while len(keys) < m:
        a, b = (int(x) for x in rng.integers(0, n, size=2))
        if a == b:
            continue
        keys.add(a * n + b)
        if len(keys) < m and rng.random() < reciprocal_frac:
            keys.add(b * n + a)
    keys = np.array(sorted(keys), dtype=np.int64)
    row_ptr, col = _csr_from_keys(keys, n)
    vlabel = rng.integers(0, n_vlabels, size=n).astype(np.int32)
    elabel = rng.integers(0, n_elabels, size=len(keys)).astype(np.int32)
    attrs = rng.integers(0, attr_values, size=(n_attrs, n)).astype(np.int32)
    attrs[rng.random((n_attrs, n)) < absent_frac] = ABSENT
    return Graph(n=n, m=len(keys), row_ptr=row_ptr, col=col, vlabel=vlabel, elabel=elabel,
                 attrs=attrs, meta={"model": "small_random", "seed": seed})


def random_literal(rng, k: int, n_attrs: int, attr_values: int):
    if rng.random() < 0.5 or k == 1:
        return {"kind": "const", "var": int(rng.integers(0, k)),
                "attr": int(rng.integers(0, n_attrs)), "value": int(rng.integers(0, attr_values))}
    i, j = (int(z) for z in rng.choice(k, size=2, replace=False))
    return {"kind": "var", "var": i, "attr": int(rng.integers(0, n_attrs)),
            "var2": j, "attr2": int(rng.integers(0, n_attrs))}


def random_gfd(seed: int, k: int, n_vlabels: int = 3, n_elabels: int = 2, n_attrs: int = 2,
               attr_values: int = 3, connected: bool = True, wildcard_frac: float = 0.2,
               extra_edge_frac: float = 0.35, y_false_frac: float = 0.15) -> dict:
    """Random pattern: a random spanning tree (if connected) plus extra directed
    edges, labels possibly wildcards; 0-2 X literals and 0-2 Y literals."""
    rng = np.random.default_rng(seed)
    E = {}
    if connected:
        for i in range(1, k):
            j = int(rng.integers(0, i))
            a, b = (j, i) if rng.random() < 0.5 else (i, j)
            E[(a, b)] = None
    for a in range(k):
        for b in range(k):
            if a != b and (a, b) not in E and rng.random() < extra_edge_frac / max(1, k - 1):
                E[(a, b)] = None

    def lab(n_lab):
        return -1 if rng.random() < wildcard_frac else int(rng.integers(0, n_lab))
    edges = [[a, b, lab(n_elabels)] for (a, b) in sorted(E)]
    vl = [lab(n_vlabels) for _ in range(k)]
    x = [random_literal(rng, k, n_attrs, attr_values) for _ in range(int(rng.integers(0, 3)))] \
        if n_attrs else []
    y_false = bool(rng.random() < y_false_frac)
    y = [] if y_false or not n_attrs else \
        [random_literal(rng, k, n_attrs, attr_values) for _ in range(int(rng.integers(0, 3)))]
    return {"k": k, "vlabels": vl, "edges": edges, "x": x, "y": y, "y_false": y_false}
