"""CPU oracle for maximal clique enumeration -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The HIP library never calls it.

The C source ``mce_oracle.c`` follows the paper (San Segundo, Artieda & Strash,
"Efficiently Enumerating all Maximal Cliques with Bit-Parallelism"):

* ``brute``      -- Sec. 2 definition of a maximal clique, over all subsets.
* ``tomita``     -- Alg. 2 with the Tomita pivot (Sec. 3.2).
* ``greedy``     -- Alg. 4 with the maximum-degree-first ordering (Sec. 4.2)
  and the GreedyBB pivot (Sec. 4.3); also fixes the node ("step") count.
* ``order``      -- the maximum-degree-first ordering alone (Sec. 4.2).
* ``subproblem`` -- one (R, P, X) subproblem under a given ordering, for the
  worked example of Sec. 5.

Each result is a dict with count, nodes, children, dead_ends, hash_xor,
hash_sum, omega and hist (list, hist[k] = cliques of size k).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mce_oracle.c")
_LIB = os.path.join(_HERE, "libmce_oracle.so")

OK = 0
E_INVAL = -1
E_NOMEM = -2
E_TRUNCATED = -3


class _Result(ctypes.Structure):
    _fields_ = [
        ("count", ctypes.c_uint64),
        ("nodes", ctypes.c_uint64),
        ("children", ctypes.c_uint64),
        ("dead_ends", ctypes.c_uint64),
        ("hash_xor", ctypes.c_uint64),
        ("hash_sum", ctypes.c_uint64),
        ("omega", ctypes.c_uint32),
        ("hist_len", ctypes.c_uint32),
        ("hist", ctypes.POINTER(ctypes.c_uint64)),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into ``oracle/libmce_oracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        u32, u64, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        p64 = ctypes.POINTER(ctypes.c_uint64)
        p32 = ctypes.POINTER(ctypes.c_uint32)
        pres = ctypes.POINTER(_Result)
        lib.orc_mix64.argtypes = [u64]
        lib.orc_mix64.restype = u64
        lib.orc_clique_hash.argtypes = [p32, u32]
        lib.orc_clique_hash.restype = u64
        lib.orc_order.argtypes = [u32, p64, u32, p32]
        for name in ("orc_greedy", "orc_tomita", "orc_brute"):
            getattr(lib, name).argtypes = [u32, p64, u32, pres]
        lib.orc_greedy_range.argtypes = [u32, p64, u32, u64, u64, pres]
        lib.orc_solve_rule.argtypes = [u32, p64, u32, i32, pres]
        lib.orc_greedy_mt.argtypes = [u32, p64, u32, i32, pres]
        lib.orc_greedy_range_mt.argtypes = [u32, p64, u32, u64, u64, i32, pres]
        lib.orc_root_branches.argtypes = [u32, p64, u32, p64]
        lib.orc_greedy_list.argtypes = [u32, p64, u32, pres, p32, u64, p64, u64, p64, p64]
        lib.orc_subproblem.argtypes = [u32, p64, u32, i32, p32, p32, u32, p32, u32, p32, u32, pres]
        for name in ("orc_order", "orc_greedy", "orc_tomita", "orc_brute", "orc_greedy_range",
                     "orc_greedy_mt", "orc_greedy_range_mt", "orc_root_branches",
                     "orc_greedy_list", "orc_subproblem", "orc_solve_rule"):
            getattr(lib, name).restype = i32
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__("oracle returned %d" % code)
        self.code = code


def _rows(rows) -> tuple[np.ndarray, int, int]:
    rows = np.ascontiguousarray(rows, dtype=np.uint64)
    if rows.ndim != 2:
        raise ValueError("rows must be a 2-D uint64 array [n, row_words]")
    return rows, rows.shape[0], rows.shape[1]


def _ptr64(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _ptr32(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _new_result(n: int):
    hist = np.zeros(n + 2, dtype=np.uint64)
    r = _Result()
    r.hist_len = hist.size
    r.hist = _ptr64(hist)
    return r, hist


def _to_dict(r: _Result, hist: np.ndarray) -> dict:
    h = [int(x) for x in hist]
    while len(h) > 1 and h[-1] == 0:
        h.pop()
    return {
        "count": int(r.count), "nodes": int(r.nodes), "children": int(r.children),
        "dead_ends": int(r.dead_ends), "hash_xor": int(r.hash_xor),
        "hash_sum": int(r.hash_sum), "omega": int(r.omega), "hist": h,
    }


def _check(rc: int):
    if rc != OK:
        raise OracleError(rc)


def mix64(z: int) -> int:
    return int(_load().orc_mix64(z & 0xFFFFFFFFFFFFFFFF))


def clique_hash(sorted_ids) -> int:
    a = np.ascontiguousarray(sorted_ids, dtype=np.uint32)
    return int(_load().orc_clique_hash(_ptr32(a), a.size))


def order(rows) -> np.ndarray:
    """Maximum-degree-first ordering: position -> input id."""
    rows, n, rw = _rows(rows)
    out = np.zeros(max(n, 1), dtype=np.uint32)
    _check(_load().orc_order(n, _ptr64(rows), rw, _ptr32(out)))
    return out[:n]


def _solve(fn, rows, *extra) -> dict:
    rows, n, rw = _rows(rows)
    r, hist = _new_result(n)
    _check(fn(n, _ptr64(rows), rw, *extra, ctypes.byref(r)))
    return _to_dict(r, hist)


def greedy(rows, threads: int = 1) -> dict:
    """GreedyBB: count, hist, hashes, omega and the node counters."""
    lib = _load()
    if threads > 1:
        return _solve(lib.orc_greedy_mt, rows, threads)
    return _solve(lib.orc_greedy, rows)


def greedy_range(rows, first: int, last: int, threads: int = 1) -> dict:
    """GreedyBB over the root's children [first, last); root node counted iff first == 0."""
    lib = _load()
    if threads > 1:
        return _solve(lib.orc_greedy_range_mt, rows, first, last, threads)
    return _solve(lib.orc_greedy_range, rows, first, last)


def root_branches(rows) -> int:
    rows, n, rw = _rows(rows)
    out = np.zeros(1, dtype=np.uint64)
    _check(_load().orc_root_branches(n, _ptr64(rows), rw, _ptr64(out)))
    return int(out[0])


def tomita(rows) -> dict:
    """Alg. 2 with the Tomita pivot on the input labels (no reordering)."""
    return _solve(_load().orc_tomita, rows)


RULES = {"greedy": 0, "tomita_bb": 1, "greedy_tx": 2}


def solve_rule(rows, rule: str) -> dict:
    """Alg. 4 on the maximum-degree-first ordering with the pivot rule
    "greedy" (GreedyBB), "tomita_bb" (TomitaBB) or "greedy_tx" (GreedyBBTX,
    whose tree GreedyBBNX shares)."""
    return _solve(_load().orc_solve_rule, rows, RULES[rule])


def brute(rows) -> dict:
    return _solve(_load().orc_brute, rows)


def greedy_list(rows) -> tuple[dict, list[tuple[int, ...]]]:
    """GreedyBB result plus the list of cliques (sorted input ids each)."""
    rows_a, n, rw = _rows(rows)
    lib = _load()
    r, hist = _new_result(n)
    ids_needed = np.zeros(1, dtype=np.uint64)
    off_needed = np.zeros(1, dtype=np.uint64)
    off = np.zeros(1, dtype=np.uint64)
    ids = np.zeros(1, dtype=np.uint32)
    rc = lib.orc_greedy_list(n, _ptr64(rows_a), rw, ctypes.byref(r), _ptr32(ids), 0,
                             _ptr64(off), 1, _ptr64(ids_needed), _ptr64(off_needed))
    if rc not in (OK, E_TRUNCATED):
        raise OracleError(rc)
    ids = np.zeros(max(int(ids_needed[0]), 1), dtype=np.uint32)
    off = np.zeros(max(int(off_needed[0]), 1), dtype=np.uint64)
    r, hist = _new_result(n)
    _check(lib.orc_greedy_list(n, _ptr64(rows_a), rw, ctypes.byref(r), _ptr32(ids), ids.size,
                               _ptr64(off), off.size, _ptr64(ids_needed), _ptr64(off_needed)))
    cliques = [tuple(int(x) for x in ids[off[i]:off[i + 1]]) for i in range(int(r.count))]
    return _to_dict(r, hist), cliques


def subproblem(rows, R, P, X, mode: str = "greedy", ids=None) -> dict:
    """One (R, P, X) subproblem with labels taken as positions of the ordering
    (rows given in that numbering).  ids[label] is the id a clique member is
    reported (and hashed) as; None keeps the labels."""
    rows, n, rw = _rows(rows)
    m = {"greedy": 0, "tomita": 1, "greedy_tx": 2}[mode]
    Ra = np.ascontiguousarray(list(R) or [0], dtype=np.uint32)
    Pa = np.ascontiguousarray(list(P) or [0], dtype=np.uint32)
    Xa = np.ascontiguousarray(list(X) or [0], dtype=np.uint32)
    ida = None
    if ids is not None:
        ida = np.ascontiguousarray(ids, dtype=np.uint32)
        if ida.shape != (n,):
            raise ValueError("ids must have one entry per vertex")
    r, hist = _new_result(n)
    _check(_load().orc_subproblem(n, _ptr64(rows), rw, m, None if ida is None else _ptr32(ida),
                                  _ptr32(Ra), len(R), _ptr32(Pa), len(P), _ptr32(Xa), len(X),
                                  ctypes.byref(r)))
    return _to_dict(r, hist)
