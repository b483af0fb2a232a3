"""GPU parity at the full sizes of the benchmark workloads, through the C ABI.

Expected values come from ``tests/golden/`` (written by ``make_golden.py``
with the CPU oracle) or from the oracle at test time.  G(300, 0.8) has about
10^12 maximal cliques, beyond any oracle run: it is checked on seeded sample
nodes of its search space (``mce_count_subproblem`` against the oracle's
``subproblem`` on the same (R, P, X)).
"""
import csv
import json
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
KEYS = ("count", "nodes", "children", "dead_ends", "hash_xor", "hash_sum", "omega")


@pytest.fixture(autouse=True)
def _opts(mce):
    mce.reset_options(watchdog_ms=100000)
    yield
    mce.reset_options()


def _gold():
    with open(os.path.join(GOLDEN, "full_configs.json")) as f:
        return json.load(f)


def _same(res, ref):
    for k in KEYS:
        assert res[k] == ref[k], (k, res[k], ref[k])
    h = list(res["hist"])
    while len(h) > 1 and h[-1] == 0:
        h.pop()
    assert h == ref["hist"]


def test_gnp1000_p03_full(mce):
    ref = _gold()["gnp1000_p0.3_s0"]
    g = mce.Graph(synth.gnp(1000, 0.3, 0))
    _same(g.count(), ref)
    assert g.root_branches() == ref["root_branches"]
    g.release()


@pytest.mark.parametrize("name", ["moon_moser_15", "moon_moser_15_relabelled"])
def test_moon_moser_15(mce, name):
    ref = _gold()[name]
    rows = synth.moon_moser(15)
    if name.endswith("relabelled"):
        rows = synth.relabel(rows, np.random.Generator(np.random.PCG64(1)).permutation(45))
    g = mce.Graph(rows)
    res = g.count()
    _same(res, ref)
    # closed forms: 3^15 cliques, all of size 15, (3^15 - 1) / 2 nodes
    assert res["count"] == 3 ** 15 and res["hist"][15] == 3 ** 15
    assert res["nodes"] == (3 ** 15 - 1) // 2
    g.release()


def test_planted800_full(mce):
    ref = _gold()["planted800_p0.5_s0"]
    rows, planted = synth.gnp_planted(800, 0.5, 0)
    g = mce.Graph(rows)
    res = g.count()
    _same(res, ref)
    # every planted set lies in some maximal clique at least as large
    assert res["omega"] >= max(len(s) for s in planted)
    g.release()


def test_batch4096_full(mce):
    specs = synth.batch_mix(4096, 0)
    with open(os.path.join(GOLDEN, "batch4096_seed0.csv")) as f:
        ref = list(csv.DictReader(f))
    assert len(ref) == len(specs)
    graphs = []
    for (n, p, seed), r in zip(specs, ref):
        assert (n, seed) == (int(r["n"]), int(r["seed"])) and abs(p - float(r["p"])) < 1e-12
        graphs.append(synth.gnp(n, p, seed))
    b = mce.Graph(batch=graphs)
    out = b.count()
    b.release()

    def differs(res, r):
        # every counter and the clique-size histogram (the golden lists it
        # without trailing zeros)
        return (any(res[k] != int(r[k]) for k in KEYS) or
                list(res["hist"]) != [int(x) for x in r["hist"].split(";")])
    bad = [i for i, (res, r) in enumerate(zip(out, ref)) if differs(res, r)]
    assert not bad, "graphs %s differ (first: %s vs %s)" % (bad[:10], out[bad[0]], ref[bad[0]])


def _sample_nodes(pos_adj, count, seed, cap=125, x_frac=0.1):
    """Seeded (R, P, X) triples in position numbering: R a clique grown at
    random until its common neighbourhood C has at most `cap` vertices, X a
    random part of C, P the rest."""
    n = pos_adj.shape[0]
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    while len(out) < count:
        R, C = [], np.ones(n, dtype=bool)
        while C.sum() > cap:
            v = int(rng.choice(np.flatnonzero(C)))
            R.append(v)
            C &= pos_adj[v]
            C[v] = False
        cand = np.flatnonzero(C)
        xm = rng.random(cand.size) < x_frac
        P = [int(x) for x in cand[~xm]]
        if P:
            out.append((R, P, [int(x) for x in cand[xm]]))
    return out


def test_gnp300_p08_sampled_nodes(mce, orc):
    rows = synth.gnp(300, 0.8, 0)
    order = orc.order(rows)
    g = mce.Graph(rows)
    assert list(g.order()) == list(order)
    adj = synth.unpack_rows(rows)
    pos_adj = adj[np.ix_(order, order)]
    rows_pos = synth.pack_rows(pos_adj)
    for R, P, X in _sample_nodes(pos_adj, 6, seed=5):
        ref = orc.subproblem(rows_pos, R, P, X, ids=order)
        res = g.count_subproblem(R, P, X)
        _same(res, ref)
    g.release()


@pytest.mark.parametrize("p", [0.001, 0.003, 0.005, 0.01, 0.03])
def test_table1_n10k_rows(mce, p):
    """The n = 10^4 rows of Table 1 (G(10^4, p) seed 0), whole graph on local
    graphs, against the oracle's results stored by make_golden.py; with the
    local graphs off, the whole graph's layout gives the same."""
    with open(os.path.join(GOLDEN, "table1_n10k.json")) as f:
        ref = json.load(f)["p=%g" % p]
    rows = synth.gnp(10000, p, 0)
    for local in (1, 0):
        mce.set_option("local_graphs", local)
        g = mce.Graph(rows)
        try:
            _same(g.count(), ref)
            assert (mce.last_stats()["local_graphs"] > 0) == (local == 1)
        finally:
            g.release()
    mce.set_option("local_graphs", 1)


def test_gnp300_p08_node_golden(mce):
    """One depth-3 node of G(300, 0.8) with about 5.7e7 maximal cliques below
    it, against the oracle's result stored by make_golden.py (its run takes
    about 80 s on one core)."""
    with open(os.path.join(GOLDEN, "gnp300_p0.8_node.json")) as f:
        ref = json.load(f)
    g = mce.Graph(synth.gnp(300, 0.8, 0))
    try:
        _same(g.count_subproblem(ref["R"], ref["P"], ref["X"]), ref)
    finally:
        g.release()


@pytest.mark.parametrize("n,p,seed,limit", [(120, 0.8, 5, 80), (200, 0.6, 6, 120)])
def test_split_pieces_add_up_to_whole_search(mce, orc, n, p, seed, limit):
    """The cut of the search tree that the whole-G(300, 0.8) measurement
    uses (bench.split_pieces: the top levels expanded in the library's
    order, the nodes left counted with mce_count_subproblem) adds up to the
    whole graph's count, counters, hashes and histogram, and to the oracle."""
    import bench
    rows = synth.gnp(n, p, seed)
    g = mce.Graph(rows)
    try:
        order = g.order().astype(np.int64)
        assert list(order) == list(orc.order(rows))
        adj = synth.unpack_rows(rows)[np.ix_(order, order)]
        pieces, top = bench.split_pieces(adj, limit)
        assert len(pieces) > 10 and top["nodes"] > 1
        tot = dict(top, count=0, hash_xor=0, hash_sum=0, omega=0, hist=[0] * (n + 1))
        for R, P, X in pieces:
            r = g.count_subproblem(R, P, X)
            for k in ("count", "nodes", "children", "dead_ends"):
                tot[k] += r[k]
            tot["hash_xor"] ^= r["hash_xor"]
            tot["hash_sum"] = (tot["hash_sum"] + r["hash_sum"]) % (1 << 64)
            tot["omega"] = max(tot["omega"], r["omega"])
            for j, c in enumerate(r["hist"]):
                tot["hist"][j] += c
        full = g.count()
        ref = orc.greedy(rows, threads=8)
        for k in ("count", "nodes", "children", "dead_ends", "hash_xor", "hash_sum", "omega"):
            assert tot[k] == full[k] == ref[k], k
        hist = list(full["hist"])
        assert tot["hist"][:len(hist)] == hist and not any(tot["hist"][len(hist):])
    finally:
        g.release()


def test_subproblem_at_root_is_whole_search(mce, orc):
    rows = synth.gnp(150, 0.5, 2)
    order = orc.order(rows)
    g = mce.Graph(rows)
    full = g.count()
    res = g.count_subproblem([], list(range(150)), [])
    for k in KEYS:
        assert res[k] == full[k], k
    g.release()


def test_subproblem_validation(mce):
    g = mce.Graph(synth.gnp(40, 0.5, 3))
    for R, P, X in [([], [], []), ([1], [1, 2], []), ([], [2, 3], [3]), ([], [40], [])]:
        with pytest.raises(mce.MceError) as e:
            g.count_subproblem(R, P, X)
        assert e.value.code == mce.E_INVAL
    g.release()
