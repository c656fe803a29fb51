"""Seeded synthetic inputs (graphs and GFDs) shared by the tests, the oracle
driver and the benchmark.  Holds no part of the validation method."""
from .graphs import Graph, ABSENT, from_edge_list, make_graph, in_csr
from . import configs, patterns

__all__ = ["Graph", "ABSENT", "from_edge_list", "make_graph", "in_csr", "configs", "patterns"]
