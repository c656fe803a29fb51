"""The unit-counting build (libgfd_count.so, loaded through GFD_LIBRARY) in a
process of its own: its results equal the normal build's and the oracle's,
and its unit counts are consistent with them -- matches and violations equal
the summed counts, every both-direction check is settled one of three ways,
attempts bound the attempts past injectivity, which bound the matches."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys
sys.path.insert(0, {root!r})
import numpy as np
import paper_2608_02321_amd as P
from synth.small import random_graph, random_gfd
g = random_graph(51, 1500, 15000, n_vlabels=2, n_elabels=2, n_attrs=2, attr_values=4, absent_frac=0.1)
rng = np.random.default_rng(51)
gfds = [random_gfd(5100 + j, int(rng.integers(2, 7)), n_vlabels=2, n_elabels=2, n_attrs=2,
                   attr_values=4, wildcard_frac=0.15, extra_edge_frac=0.3) for j in range(12)]
gh = P.load(g)
out = {{}}
for sem in ("induced", "mono"):
    r, st = P.validate(gh, gfds, K=64, semantics=sem, batched=True, stats=True,
                       violation_cap=1 << 20, flags=P.GFD_FLAG_NO_GRAPH)
    out[sem] = {{"results": r, "units": st["units"], "counted": st["units_counted"]}}
print(json.dumps(out))
"""


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2608_02321_amd as P
    return P


def test_counting_build_units(P):
    from oracle import oracle as O
    lib = os.path.join(ROOT, "paper_2608_02321_amd", "libgfd_count.so")
    assert os.path.exists(lib), "build the library (it builds the counting variant too)"
    env = dict(os.environ, GFD_LIBRARY=lib)
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT)], capture_output=True,
                       text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    out = json.loads(r.stdout.strip().splitlines()[-1])
    from synth.small import random_graph, random_gfd
    import numpy as np
    g = random_graph(51, 1500, 15000, n_vlabels=2, n_elabels=2, n_attrs=2, attr_values=4,
                     absent_frac=0.1)
    rng = np.random.default_rng(51)
    gfds = [random_gfd(5100 + j, int(rng.integers(2, 7)), n_vlabels=2, n_elabels=2, n_attrs=2,
                       attr_values=4, wildcard_frac=0.15, extra_edge_frac=0.3) for j in range(12)]
    og = O.OracleGraph(g)
    gh = P.load(g)
    for sem in ("induced", "mono"):
        got = out[sem]
        assert got["counted"] == 1
        exp = [O.validate(og, d, sem, K=64, threads=4) for d in gfds]
        assert got["results"] == exp
        assert P.validate(gh, gfds, K=64, semantics=sem, batched=True) == exp
        u = got["units"]
        assert u["matches"] == sum(e["match_count"] for e in exp)
        assert u["violations"] == sum(e["violation_count"] for e in exp)
        assert u["attempts"] >= u["injective"] >= u["matches"] > 0
        assert u["sources"] <= u["attempts"]
        assert u["table_free"] + u["table_hit"] + u["short_row"] == u["checks_both"]
        if sem == "induced":
            assert u["checks_both"] > 0
    gh.free()
