"""Launch shapes never change a result: every candidate of the autotuner's
grid (enumeration and scan block counts, probe-ahead form, violation
staging) gives the oracle's results, batched and one GFD at a time; the
tuner itself checks the same and caches its choice."""
import json

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


def test_every_candidate_gives_the_oracle_results(P):
    from paper_2608_02321_amd import tune as T
    g = random_graph(61, 2000, 22000, n_vlabels=2, n_elabels=2, n_attrs=2, attr_values=4,
                     absent_frac=0.1)
    rng = np.random.default_rng(61)
    gfds = [random_gfd(6100 + j, int(rng.integers(2, 7)), n_vlabels=2, n_elabels=2, n_attrs=2,
                       attr_values=4, wildcard_frac=0.15, extra_edge_frac=0.3) for j in range(16)]
    og = O.OracleGraph(g)
    gh = P.load(g)
    for sem in ("induced", "mono"):
        exp = [O.validate(og, d, sem, K=32, threads=4) for d in gfds]
        for knob, values in T.CANDIDATES.items():
            for v in values:
                for batched in (True, False):
                    got = P.validate(gh, gfds, K=32, semantics=sem, batched=batched, tuning={knob: v})
                    assert got == exp, (sem, knob, v, batched)
    with pytest.raises(P.GfdError):
        P.validate(gh, gfds[:1], tuning={"flat_grid": 10})
    gh.free()


def test_tuner_choice_is_cached(P, tmp_path):
    from paper_2608_02321_amd import tune as T
    g = random_graph(62, 1500, 15000, n_vlabels=2, n_elabels=2, n_attrs=2, attr_values=4)
    rng = np.random.default_rng(62)
    gfds = [random_gfd(6200 + j, int(rng.integers(2, 6)), n_vlabels=2, n_elabels=2, n_attrs=2,
                       attr_values=4) for j in range(8)]
    gh = P.load(g)
    path = str(tmp_path / "tuning.json")
    first = T.tune(gh, gfds, g.sha256(), K=16, reps=2, path=path)
    assert not first["cached"] and set(first["tuning"]) == set(T.CANDIDATES)
    assert len(first["tried"]) >= 1 + sum(len(v) - 1 for v in T.CANDIDATES.values())
    again = T.tune(gh, gfds, g.sha256(), K=16, reps=2, path=path)
    assert again["cached"] and again["tuning"] == first["tuning"]
    stored = json.load(open(path))
    assert any(k.startswith(g.sha256()) for k in stored)
    gh.free()
