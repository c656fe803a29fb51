"""The pins must catch plausible mistakes in the oracle.

Each case plants one mistake in a private copy of oracle.c (a dropped term, a
transposed operand, a wrong constant ...), compiles it on the CPU, and checks
that the pin battery -- brute force and the St. Petersburg fixture -- rejects
the mutant.  (Dropping the "attribute present" test from a constant literal is
not listed: constants are non-negative and the missing marker is -1, so that
change is equivalent on every valid input.)
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from oracle.brute import brute_validate
from synth import configs, from_edge_list
from synth.small import random_graph, random_gfd

MUTANTS = {
    "transposed_edge_direction": ("int32_t fwd = edge_label(g, s->t[j], v);",
                                  "int32_t fwd = edge_label(g, v, s->t[j]);"),
    "dropped_induced_forward": ("} else if (s->induced && fwd != ORC_NONE) {",
                                "} else if (0) {"),
    "dropped_induced_backward": ("} else if (s->induced && bwd != ORC_NONE) {",
                                 "} else if (0) {"),
    "dropped_injectivity": ("if (s->t[j] == v) return 0;", ";"),
    "dropped_vertex_label": ("if (s->qlab[i] != ORC_ANY && g->vlabel[v] != s->qlab[i]) return 0;",
                             ";"),
    "wildcard_edge_ignored": ("if (s->qe[j][i] != ORC_ANY && fwd != s->qe[j][i]) return 0;",
                              "if (fwd != s->qe[j][i]) return 0;"),
    "edge_label_unchecked": ("if (s->qe[i][j] != ORC_ANY && bwd != s->qe[i][j]) return 0;", ";"),
    "absent_variable": ("return a != ORC_ABSENT && b != ORC_ABSENT && a == b;",
                        "return a == b;"),
    "y_false_ignored": ("if (s->y_false) Y = 0;", "if (0) Y = 0;"),
    "x_ignored": ("if (X && !Y) {", "if (!Y) {"),
    "heap_order_reversed": ("if (lex_cmp(t, s->heap, k) >= 0) return;",
                            "if (lex_cmp(t, s->heap, k) <= 0) return;"),
    "hash_seed_without_k": ("0x9E3779B97F4A7C15ULL * (uint64_t)k", "0x9E3779B97F4A7C15ULL"),
    "hash_shift": ("z ^= z >> 27;", "z ^= z >> 26;"),
    "in_row_as_out_row": ("int32_t v = g->in_src[e];", "int32_t v = g->out_dst[e];"),
}


def _battery(L):
    """Returns the name of the first pin that fails, or None."""
    for s in range(60):
        rng = np.random.default_rng(10_000 + s)
        n = int(rng.integers(3, 8))
        m = int(rng.integers(n, n * (n - 1) + 1))
        k = int(rng.integers(1, min(4, n) + 1))
        g = random_graph(s, n, m, n_vlabels=2, n_elabels=2, n_attrs=2, attr_values=3)
        gfd = random_gfd(s, k, n_vlabels=2, n_elabels=2, n_attrs=2, attr_values=3)
        og = O.OracleGraph(g, L)
        for sem in ("induced", "mono"):
            if O.validate(og, gfd, sem, 3) != brute_validate(g, gfd, sem, 3):
                return "brute_force"
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "x1_st_petersburg.json")))
    gr = d["graph"]
    g = from_edge_list(gr["n"], gr["edges"], gr["vlabel"], [gr["name"]])
    r = O.validate(O.OracleGraph(g, L), d["gfd"], "induced")
    if r["violations"] != d["expected"]["induced"]["violations"]:
        return "x1"
    return None


@pytest.fixture(scope="module")
def src():
    return open(O.SRC).read()


def test_unmutated_passes(src, tmp_path):
    path = O.compile_c(O.SRC, str(tmp_path / "ok.so"))
    assert _battery(O.load(path)) is None


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, src, tmp_path):
    old, new = MUTANTS[name]
    assert src.count(old) == 1, name
    c = tmp_path / f"{name}.c"
    c.write_text(src.replace(old, new))
    L = O.load(O.compile_c(str(c), str(tmp_path / f"{name}.so")))
    assert _battery(L) is not None, f"mutant {name} survived the pins"
