"""Exhaustive brute force of GFD validation -- TEST INFRASTRUCTURE ONLY.

A second, independent transcription of the Section II definitions in pure
Python: every k-tuple of vertices is generated (itertools.product over V^k) and
tested against the definition of a match, then the GFD's literals.  Meant for
tiny graphs only (n <= 8, k <= 4); it pins the C oracle.
"""
from __future__ import annotations

import itertools

MASK = (1 << 64) - 1


def _mix(z):
    z ^= z >> 30
    z = (z * 0xBF58476D1CE4E5B9) & MASK
    z ^= z >> 27
    z = (z * 0x94D049BB133111EB) & MASK
    z ^= z >> 31
    return z


def tuple_hash(t):
    h = (0x9E3779B97F4A7C15 * len(t)) & MASK
    for v in t:
        h = _mix(h ^ (v & 0xFFFFFFFF))
    return h


def brute_validate(g, gfd, semantics="induced", K=1024):
    n, k = g.n, gfd["k"]
    E = {}
    for s in range(n):
        for e in range(g.row_ptr[s], g.row_ptr[s + 1]):
            E[(s, int(g.col[e]))] = int(g.elabel[e])
    QE = {(a, b): l for a, b, l in gfd["edges"]}
    attrs = g.attrs

    def lit(t, l):
        a = int(attrs[l["attr"], t[l["var"]]])
        if l["kind"] == "const":
            return a != -1 and a == l["value"]
        b = int(attrs[l["attr2"], t[l["var2"]]])
        return a != -1 and b != -1 and a == b

    matches, viols, mfp, vfp = 0, [], 0, 0
    for t in itertools.product(range(n), repeat=k):
        if len(set(t)) < k:
            continue
        ok = all(gfd["vlabels"][i] in (-1, int(g.vlabel[t[i]])) for i in range(k))
        for i in range(k):
            for j in range(k):
                if not ok or i == j:
                    continue
                q, d = QE.get((i, j)), E.get((t[i], t[j]))
                if q is not None:
                    ok = d is not None and q in (-1, d)
                elif semantics == "induced":
                    ok = d is None
        if not ok:
            continue
        matches += 1
        h = tuple_hash(t)
        mfp = (mfp + h) & MASK
        X = all(lit(t, l) for l in gfd.get("x", []))
        Y = False if gfd.get("y_false") else all(lit(t, l) for l in gfd.get("y", []))
        if X and not Y:
            viols.append(list(t))
            vfp = (vfp + h) & MASK
    viols.sort()
    return {"match_count": matches, "violation_count": len(viols), "match_fp": mfp,
            "violation_fp": vfp, "satisfied": not viols, "violations": viols[:K]}
