"""Benchmark of the MI355X GreedyBB maximal clique enumeration.

One step = one pass of the whole hot path over one synthetic graph already
resident in HBM: device-side validation, maximum-degree-first ordering,
renumbering (mce_prepare with a device pointer), the root and the persistent
search with its work queue, the reduction and the copy of the results to the
host (mce_count), then mce_release.

Default workload: G(n=1000, p=0.3), seed 0 -- the random graph of the paper's
Table 1 (n = 1000, p = 0.3) drawn with this repository's seeded generator.

Prints one JSON line.  ``--gpus N`` with N > 1 is refused: this build runs on
one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X peak of 32-bit integer vector lane operations: 256 CUs x 4 SIMDs x
# 16 lanes x 2.4 GHz.
VALU_PEAK_GOPS = 256 * 4 * 16 * 2.4
# Paper, Table 1, GreedyBB at n=1000, p=0.3 (average of 10 graphs, one Xeon
# E5-2690 v2 core): 15.487755M maximal cliques in 4.964 s.
PAPER_G1000_CLIQUES_PER_S = 15.487755e6 / 4.964

WORKLOADS = {
    "gnp1000": dict(n=1000, p=0.3, seed=0),
    "gnp100": dict(n=100, p=0.5, seed=0),
    "gnp300_05": dict(n=300, p=0.5, seed=0),
}


def algorithmic_word_ops(res: dict, n: int) -> int:
    """32-bit word operations the method itself needs (Sec. 4.1 encoding):
    per node a pivot scan and the ANDN of L over W words, per child two ANDs
    and two empty tests over W words."""
    w = (n + 31) // 32
    return w * (2 * res["nodes"] + 4 * res["children"])


def cpu_baseline(rows, threads: int) -> dict:
    import oracle
    t0 = time.perf_counter()
    ref = oracle.greedy(rows, threads=threads)
    dt = time.perf_counter() - t0
    return ref, dt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="gnp1000", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    from paper_1801_00202_amd import mce

    torch.cuda.set_device(0)
    mce.load()
    mce.reset_options(watchdog_ms=120000)
    wl = WORKLOADS[args.workload]
    rows = synth.gnp(wl["n"], wl["p"], wl["seed"])
    d_rows = torch.from_numpy(rows.view(np.int64)).cuda()
    torch.cuda.synchronize()

    def step():
        g = mce.Graph(d_rows)
        r = g.count()
        st = mce.last_stats()
        g.release()
        return r, st

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    results, kernel_us, stats = [], [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r, st = step()
        results.append(r)
        kernel_us.append(st["search_kernel_us"])
        stats.append(st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    first = results[0]
    assert all(r == first for r in results), "results differ between steps"
    ms = dt * 1000.0 / args.steps
    cliques_per_s = first["count"] * args.steps / dt
    nodes_per_s = first["nodes"] * args.steps / dt
    k_us = sum(kernel_us) / len(kernel_us)
    ops = algorithmic_word_ops(first, wl["n"])
    achieved = ops / (k_us * 1e-6) / 1e9

    line = {
        "metric": "maximal cliques/sec (GreedyBB, one GPU)",
        "value": cliques_per_s,
        "unit": "cliques/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": cliques_per_s / PAPER_G1000_CLIQUES_PER_S if args.workload == "gnp1000" else None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "G(n=%d, p=%g) seed %d" % (wl["n"], wl["p"], wl["seed"]),
                   "cliques": first["count"], "nodes": first["nodes"], "omega": first["omega"]},
        "nodes_per_s": nodes_per_s,
        "search_kernel_us": k_us,
        "prepare_us": sum(s["prepare_us"] for s in stats) / len(stats),
        "launch": {"blocks": stats[0]["blocks"], "waves_per_block": stats[0]["waves_per_block"],
                   "lds_depth": stats[0]["lds_depth"], "donations": stats[0]["donations"],
                   "units": stats[0]["units"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_GOPS, "unit": "Gop/s",
                     "frac": achieved / VALU_PEAK_GOPS, "traffic": None},
    }
    if not args.no_cpu_baseline:
        threads = args.cpu_threads or min(len(os.sched_getaffinity(0)), 16)
        ref, cdt = cpu_baseline(rows, threads)
        assert ref["count"] == first["count"] and ref["hash_xor"] == first["hash_xor"]
        line["cpu_baseline"] = {"value": ref["count"] / cdt, "unit": "cliques/s", "cores": threads,
                                "kind": "oracle",
                                "sample": "the full workload graph, root children shared among threads"}
    print(json.dumps(line))


if __name__ == "__main__":
    main()
