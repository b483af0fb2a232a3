"""MI355X maximal clique enumeration (GreedyBB: maximum-degree-first ordering,
greedy ordered pivot, bit-parallel Bron-Kerbosch) behind the C ABI of
include/mce.h.  ``paper_1801_00202_amd.mce`` is the ctypes binding; importing
this package does not load the library."""
