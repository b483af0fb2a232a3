"""Seeded graph generators.

G(n, p, seed): a ``numpy.random.Generator(PCG64(seed))`` draws one uniform per
unordered pair (i < j) in row-major order, (0,1), (0,2), ..., (0,n-1), (1,2), ...;
the pair is an edge iff its uniform is below p.  This stands in for the
uniform random graphs of the paper's Table 1, whose generator is not given.

Planted cliques (a stand-in for the structured medium-density class of Table 2,
whose graph files are not used): G(n, p, seed), then from the same stream, for
each planted clique a size s ~ U{lo..hi} and a uniform s-subset of the
vertices; all pairs inside the subset become edges.

Moon-Moser graph (the Theta(3^{n/3}) family the paper's introduction cites):
3k vertices, u ~ v iff floor(u/3) != floor(v/3).
"""
from __future__ import annotations

import math

import numpy as np


def row_words(n: int) -> int:
    return max(1, (n + 63) // 64)


def pack_rows(adj: np.ndarray) -> np.ndarray:
    """Boolean adjacency matrix [n, n] -> uint64 rows [n, ceil(n/64)], LSB first."""
    adj = np.asarray(adj, dtype=bool)
    n = adj.shape[0]
    rw = row_words(n)
    pad = np.zeros((n, rw * 64), dtype=bool)
    pad[:, :n] = adj
    b = np.packbits(pad, axis=1, bitorder="little")  # byte k of a row holds columns 8k..8k+7
    return np.ascontiguousarray(b).view("<u8").astype(np.uint64).reshape(n, rw)


def unpack_rows(rows: np.ndarray, n: int | None = None) -> np.ndarray:
    rows = np.asarray(rows, dtype=np.uint64)
    if n is None:
        n = rows.shape[0]
    bits = ((rows[:, :, None] >> np.arange(64, dtype=np.uint64)) & np.uint64(1)).astype(bool)
    return bits.reshape(rows.shape[0], -1)[:, :n]


def _pairs_to_adj(n: int, mask: np.ndarray) -> np.ndarray:
    adj = np.zeros((n, n), dtype=bool)
    iu = np.triu_indices(n, 1)  # row-major order of pairs (i < j)
    adj[iu] = mask
    return adj | adj.T


def gnp(n: int, p: float, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    # the uniforms of row i's pairs (i, i+1..n-1) come next in the stream:
    # drawing them row by row gives the same stream as one draw of all pairs
    adj = np.zeros((n, n), dtype=bool)
    for i in range(n - 1):
        adj[i, i + 1:] = rng.random(n - 1 - i) < p
    return pack_rows(adj | adj.T)


def gnp_planted(n: int, p: float, seed: int, cliques: int = 12, lo: int = 20, hi: int = 40):
    """G(n,p,seed) plus planted cliques; returns (rows, list of planted vertex sets)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random(n * (n - 1) // 2)
    adj = _pairs_to_adj(n, u < p)
    planted = []
    for _ in range(cliques):
        s = int(rng.integers(lo, hi + 1))
        verts = np.sort(rng.choice(n, size=s, replace=False))
        adj[np.ix_(verts, verts)] = True
        planted.append([int(v) for v in verts])
    np.fill_diagonal(adj, False)
    return pack_rows(adj), planted


def moon_moser(k: int) -> np.ndarray:
    n = 3 * k
    g = np.arange(n) // 3
    adj = g[:, None] != g[None, :]
    return pack_rows(adj)


def relabel(rows: np.ndarray, perm) -> np.ndarray:
    """Graph with vertex v renamed perm[v]."""
    adj = unpack_rows(rows)
    perm = np.asarray(perm)
    n = adj.shape[0]
    out = np.zeros((n, n), dtype=bool)
    out[np.ix_(perm, perm)] = adj
    return pack_rows(out)


def complete(n: int) -> np.ndarray:
    adj = np.ones((n, n), dtype=bool)
    np.fill_diagonal(adj, False)
    return pack_rows(adj) if n else np.zeros((0, 1), dtype=np.uint64)


def empty(n: int) -> np.ndarray:
    return pack_rows(np.zeros((n, n), dtype=bool)) if n else np.zeros((0, 1), dtype=np.uint64)


def cycle(n: int) -> np.ndarray:
    adj = np.zeros((n, n), dtype=bool)
    for i in range(n):
        adj[i, (i + 1) % n] = adj[(i + 1) % n, i] = True
    np.fill_diagonal(adj, False)
    return pack_rows(adj)


def star(n: int) -> np.ndarray:
    adj = np.zeros((n, n), dtype=bool)
    adj[0, 1:] = adj[1:, 0] = True
    return pack_rows(adj)


def path(n: int) -> np.ndarray:
    adj = np.zeros((n, n), dtype=bool)
    for i in range(n - 1):
        adj[i, i + 1] = adj[i + 1, i] = True
    return pack_rows(adj)


def complete_multipartite(parts) -> np.ndarray:
    lab = np.concatenate([np.full(a, i) for i, a in enumerate(parts)])
    return pack_rows(lab[:, None] != lab[None, :])


def disjoint_union(*graphs) -> np.ndarray:
    mats = [unpack_rows(g) for g in graphs]
    n = sum(m.shape[0] for m in mats)
    adj = np.zeros((n, n), dtype=bool)
    o = 0
    for m in mats:
        k = m.shape[0]
        adj[o:o + k, o:o + k] = m
        o += k
    return pack_rows(adj)


def edge_list_to_rows(n: int, edges) -> np.ndarray:
    """Edge list -> rows; duplicate edges collapse, self-loops are rejected."""
    adj = np.zeros((n, n), dtype=bool)
    for u, v in edges:
        if u == v:
            raise ValueError("self-loop at vertex %d" % u)
        if not (0 <= u < n and 0 <= v < n):
            raise ValueError("vertex out of range")
        adj[u, v] = adj[v, u] = True
    return pack_rows(adj)


def expected_mu(n: int, p: float) -> float:
    """E[number of maximal cliques] of G(n,p): sum_k C(n,k) p^C(k,2) (1-p^k)^(n-k)."""
    if n == 0:
        return 1.0
    lg = math.lgamma
    tot = 0.0
    for k in range(1, n + 1):
        pk = p ** k
        if pk >= 1.0:
            continue
        t = (lg(n + 1) - lg(k + 1) - lg(n - k + 1) + (k * (k - 1) / 2) * math.log(p)
             + (n - k) * math.log1p(-pk))
        tot += math.exp(t) if t > -700 else 0.0
    return tot


def batch_mix(count: int, base_seed: int, n_lo: int = 32, n_hi: int = 512, p_lo: float = 0.1,
              p_hi: float = 0.9, mu_cap: float = 1e6):
    """Batched workload: (n, p) drawn from PCG64(base_seed), redrawn while
    E[mu](n, p) > mu_cap; graph i is G(n_i, p_i, base_seed + i)."""
    rng = np.random.Generator(np.random.PCG64(base_seed))
    specs = []
    for i in range(count):
        while True:
            n = int(rng.integers(n_lo, n_hi + 1))
            p = float(rng.uniform(p_lo, p_hi))
            if expected_mu(n, p) <= mu_cap:
                break
        specs.append((n, p, base_seed + i))
    return specs


def serving_mix(count: int, base_seed: int, n_lo: int = 64, n_hi: int = 2048, p_lo: float = 0.2,
                p_hi: float = 0.9, mu_cap: float = 1e6):
    """Serving mix: n = round(exp(U[ln n_lo, ln n_hi])), p ~ U[p_lo, p_hi], same
    E[mu] redraw; request i is G(n_i, p_i, base_seed + i)."""
    rng = np.random.Generator(np.random.PCG64(base_seed))
    specs = []
    for i in range(count):
        while True:
            n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
            p = float(rng.uniform(p_lo, p_hi))
            if expected_mu(n, p) <= mu_cap:
                break
        specs.append((n, p, base_seed + i))
    return specs


def poisson_arrivals(count: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process with the given rate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=count))
