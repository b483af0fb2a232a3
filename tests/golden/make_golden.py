"""Write the expected results of the full-size workloads with the CPU oracle.

Calls only ``oracle`` (and ``synth`` for the seeded inputs).  Usage, from the
repository root:

    python tests/golden/make_golden.py [--threads T] [--only NAME ...]

Outputs (next to this script):
  full_configs.json   G(1000, 0.3) seed 0; Moon-Moser k = 15 and a relabelled
                      copy; planted G(800, 0.5) seed 0 (12 cliques of 20..40)
  table1_n10k.json    G(10^4, p) seed 0, p in {0.001, 0.003, 0.005, 0.01, 0.03}
  gnp300_p0.8_node.json  one node of G(300, 0.8) seed 0 with about 10^8 maximal
                      cliques below it (R, P, X as positions of the ordering)
  batch4096_seed0.csv the 4096-graph batch (base seed 0), one line per graph;
                      the hist column is the clique-size histogram without trailing
                      zeros, entries separated by ";"
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

MM_PERM_SEED = 1


def full_configs(threads):
    out = {}
    cases = {
        "gnp1000_p0.3_s0": lambda: synth.gnp(1000, 0.3, 0),
        "moon_moser_15": lambda: synth.moon_moser(15),
        "moon_moser_15_relabelled": lambda: synth.relabel(
            synth.moon_moser(15), np.random.Generator(np.random.PCG64(MM_PERM_SEED)).permutation(45)),
        "planted800_p0.5_s0": lambda: synth.gnp_planted(800, 0.5, 0)[0],
    }
    for name, make in cases.items():
        t0 = time.perf_counter()
        rows = make()
        r = oracle.greedy(rows, threads=threads)
        r["root_branches"] = oracle.root_branches(rows)
        r["oracle_seconds"] = round(time.perf_counter() - t0, 2)
        r["oracle_threads"] = threads
        out[name] = r
        print(name, r["count"], r["nodes"], r["oracle_seconds"], flush=True)
    return out


def gnp300_node(r_size=3, seed=17, x_frac=0.1):
    """One node (R, P, X) of the search space of G(300, 0.8) seed 0, in the
    positions of the maximum-degree-first ordering: R a clique of r_size
    vertices grown from a seeded stream, C its common neighbourhood, X a
    seeded tenth of C, P the rest.  The whole graph has about 10^12 maximal
    cliques, beyond any oracle run; this node has about 10^8."""
    rows = synth.gnp(300, 0.8, 0)
    order = oracle.order(rows)
    adj = synth.unpack_rows(rows)
    pos = adj[np.ix_(order, order)]
    rng = np.random.Generator(np.random.PCG64(seed))
    R, C = [], np.ones(300, dtype=bool)
    while len(R) < r_size:
        v = int(rng.choice(np.flatnonzero(C)))
        R.append(v)
        C &= pos[v]
        C[v] = False
    cand = np.flatnonzero(C)
    xm = rng.random(cand.size) < x_frac
    P = [int(x) for x in cand[~xm]]
    X = [int(x) for x in cand[xm]]
    t0 = time.perf_counter()
    r = oracle.subproblem(synth.pack_rows(pos), R, P, X, ids=order)
    r.update({"R": R, "P": P, "X": X, "oracle_seconds": round(time.perf_counter() - t0, 2), "oracle_threads": 1})
    print("gnp300 node", len(R), len(P), len(X), r["count"], r["nodes"], r["oracle_seconds"], flush=True)
    return r


def table1_n10k(threads):
    """G(10^4, p) seed 0 for the five p of Table 1's n = 10^4 rows."""
    out = {}
    for p in (0.001, 0.003, 0.005, 0.01, 0.03):
        t0 = time.perf_counter()
        r = oracle.greedy(synth.gnp(10000, p, 0), threads=threads)
        r["oracle_seconds"] = round(time.perf_counter() - t0, 2)
        r["oracle_threads"] = threads
        out["p=%g" % p] = r
        print("n=10^4 p=%g" % p, r["count"], r["nodes"], r["oracle_seconds"], flush=True)
    return out


def batch(threads):
    specs = synth.batch_mix(4096, 0)
    lines = ["index,n,p,seed,count,nodes,children,dead_ends,hash_xor,hash_sum,omega,hist"]
    t0 = time.perf_counter()
    for i, (n, p, seed) in enumerate(specs):
        r = oracle.greedy(synth.gnp(n, p, seed), threads=threads)
        hist = list(r["hist"])
        while len(hist) > 1 and hist[-1] == 0:
            hist.pop()
        lines.append("%d,%d,%r,%d,%d,%d,%d,%d,%d,%d,%d,%s" % (i, n, p, seed, r["count"], r["nodes"], r["children"],
                                                           r["dead_ends"], r["hash_xor"], r["hash_sum"], r["omega"],
                                                           ";".join(str(x) for x in hist)))
    print("batch", len(specs), round(time.perf_counter() - t0, 1), "s", flush=True)
    return "\n".join(lines) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--only", nargs="*", default=["full", "batch"])
    a = ap.parse_args()
    if "full" in a.only:
        with open(os.path.join(HERE, "full_configs.json"), "w") as f:
            json.dump(full_configs(a.threads), f, indent=1, sort_keys=True)
    if "table1" in a.only:
        with open(os.path.join(HERE, "table1_n10k.json"), "w") as f:
            json.dump(table1_n10k(a.threads), f, indent=1, sort_keys=True)
    if "gnp300node" in a.only:
        with open(os.path.join(HERE, "gnp300_p0.8_node.json"), "w") as f:
            json.dump(gnp300_node(), f, indent=1, sort_keys=True)
    if "batch" in a.only:
        with open(os.path.join(HERE, "batch4096_seed0.csv"), "w") as f:
            f.write(batch(a.threads))


if __name__ == "__main__":
    main()
