"""Seeded synthetic inputs shared by the tests, the oracle runs and the benchmark.

This package only draws graphs; it holds none of the enumeration method's
arithmetic.  Graphs are returned as adjacency bitset rows: a ``uint64`` array of
shape ``[n, ceil(n/64)]``, least significant bit first, bit ``j`` of row ``i``
set iff ``{i, j}`` is an edge.
"""
from .graphs import (  # noqa: F401
    row_words, pack_rows, unpack_rows, gnp, gnp_planted, moon_moser, relabel,
    complete, empty, cycle, complete_multipartite, disjoint_union, star, path,
    expected_mu, batch_mix, serving_mix, poisson_arrivals, edge_list_to_rows,
)
