"""Benchmark of the MI355X GreedyBB maximal clique enumeration.

One step = one pass of the whole hot path over one synthetic graph already
resident in HBM: device-side validation, maximum-degree-first ordering and
renumbering (mce_prepare with a device pointer), the root units and the
persistent search with its work distribution, the reduction and the copy of
the totals to the host (mce_count), then mce_release.

Default workload: G(n=1000, p=0.3), seed 0 -- the random graph of the paper's
Table 1 row (n = 1000, p = 0.3), drawn with this repository's seeded
generator.

Prints one JSON line.  ``--gpus N`` with N > 1 is refused: this build runs on
one GPU.

``--g300-full K/N`` runs part K of N of the whole G(300, 0.8) graph (about
10^12 maximal cliques, some 1000 s of search: too long for one call, and for
the oracle) as subproblems, and ``--g300-combine`` adds the parts up; see
``split_pieces``.

``--copy-probe`` instead times a plain device-to-device copy of known size;
run under ``rocprofv3 --pmc FETCH_SIZE`` (then ``WRITE_SIZE``) it calibrates the
HBM byte counters that the ``traffic`` figure of the search kernel uses.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X datasheet-derived peaks (the bench measures both on the box with the
# probes of libmce_probe.so and uses the measured ones as denominators):
# 32-bit integer vector lane operations, 256 CUs x 4 SIMDs x 16 lanes x
# 2.4 GHz (bitwise integer ops have no packed form); LDS reads, 256 bytes per
# clock per CU (the probe measures about that on gfx950).
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
LDS_PEAK_TBPS = 256 * 256 * 2.4e9 / 1e12
# Paper, Table 1, GreedyBB at n=1000, p=0.3 (average of 10 graphs, one Xeon
# E5-2690 v2 core): 15.487755M maximal cliques in 4.964 s.
PAPER_G1000_CLIQUES_PER_S = 15.487755e6 / 4.964

WORKLOADS = {
    "gnp1000": dict(n=1000, p=0.3, seed=0),
    "gnp100": dict(n=100, p=0.5, seed=0),
    "gnp300_05": dict(n=300, p=0.5, seed=0),
}
KERNEL_SRC = os.path.join(ROOT, "paper_1801_00202_amd", "csrc", "kernels.hip")
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "search_kernel_gnp1000_traffic.md")


def kernel_source_hash() -> str:
    """sha256 (16 hex digits) of the device code the search kernel is built
    from: kernels.hip up to its launchers, and mce_internal.h, with comments
    and blank space taken out (so that a comment does not count as a change,
    and any change to the device code does, helpers included)."""
    parts = []
    for path, cut in ((KERNEL_SRC, True), (os.path.join(os.path.dirname(KERNEL_SRC), "mce_internal.h"), False)):
        with open(path) as f:
            src = f.read()
        if cut:
            src = src[:src.index("// ---------------------------------------------------------- launchers ----")]
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        parts.append(" ".join(src.split()))
    return hashlib.sha256("\n".join(parts).encode()).hexdigest()[:16]


def algorithmic_word_ops(res: dict, n: int) -> int:
    """32-bit word operations the method itself needs (Sec. 4.1 encoding):
    per node a pivot scan and the ANDN of L over W words, per child two ANDs
    and two empty tests over W words."""
    w = (n + 31) // 32
    return w * (2 * res["nodes"] + 4 * res["children"])


def algorithmic_lds_bytes(res: dict, n: int) -> int:
    """LDS bytes the search's stack needs: a node's frame (P, X and L, one
    32-bit word each per bitset word, plus the row kept for the next
    candidate) written when it is pushed and read back when the search
    returns to it."""
    w = (n + 31) // 32
    return 2 * 16 * w * res["nodes"]


def measured_peaks() -> dict:
    """int32 VALU lane-ops/s and LDS read bytes/s measured on this device by
    the probes of libmce_probe.so (best of three launches each)."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1801_00202_amd", "libmce_probe.so"))
    d = ctypes.c_double
    lib.mce_probe_valu.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(d), ctypes.POINTER(d)]
    lib.mce_probe_lds.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(d), ctypes.POINTER(d)]
    out = {}
    for name, fn, blocks, iters in (("valu_lane_ops_per_s", lib.mce_probe_valu, 256 * 32, 4096),
                                    ("lds_bytes_per_s", lib.mce_probe_lds, 256 * 32, 16384)):
        best = 0.0
        for _ in range(3):
            rate, sec = d(), d()
            rc = fn(blocks, iters, ctypes.byref(rate), ctypes.byref(sec))
            if rc != 0:
                raise RuntimeError("%s probe failed (%d)" % (name, rc))
            best = max(best, rate.value)
        out[name] = best
    return out


def cpu_info() -> dict:
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "cpu_logical_total": os.cpu_count(),
            "cpu_affinity": len(os.sched_getaffinity(0))}


def recorded_traffic(workload: str):
    """HBM bytes per search-kernel launch from the committed counter summary,
    or None if it was taken on another kernel source or workload."""
    if workload != "gnp1000" or not os.path.exists(TRAFFIC_PROFILE):
        return None
    m = re.search(r"^traffic_json:\s*(\{.*\})\s*$", open(TRAFFIC_PROFILE).read(), re.M)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("kernel_sha256_16") != kernel_source_hash():
        return None
    return rec


def copy_probe(mib: int, reps: int) -> None:
    import torch
    n = mib * (1 << 20) // 4
    src = torch.arange(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n, "reps": reps,
                      "GB_per_s": 8 * n / dt / 1e9}))


def batched(mce, synth, np, reps: int, tune: bool) -> dict:
    """4096 graphs (n ~ U{32..512}, p ~ U[0.1, 0.9], E[mu] <= 1e6, base seed 0)
    in one handle and one persistent launch (schedule from mce_autotune,
    replayed as a captured hipGraph), against the same graphs solved one by
    one (the plain single-graph solve)."""
    import torch
    graphs = [synth.gnp(n, p, seed) for n, p, seed in synth.batch_mix(4096, 0)]
    b = mce.Graph(batch=graphs)
    tuned = b.autotune(max_trials=12) if tune else None
    out = b.count()                      # warm-up, captures the graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = b.count()
    dt = (time.perf_counter() - t0) / reps
    device_ms = mce.last_stats()["search_us"] / 1e3
    b.release()
    cliques = sum(r["count"] for r in out)
    nodes = sum(r["nodes"] for r in out)
    # plain: one handle per graph, prepared once, solved one after the other
    handles = [mce.Graph(r) for r in graphs]
    handles[0].count()
    t0 = time.perf_counter()
    plain = [h.count() for h in handles]
    dt_plain = time.perf_counter() - t0
    for h in handles:
        h.release()
    assert plain == out, "batched and plain solves differ"
    return {"workload": "4096 graphs, n ~ U{32..512}, p ~ U[0.1,0.9], E[mu] <= 1e6, base seed 0",
            "timed": "both sides time the solves of graphs prepared beforehand (ordering and renumbering "
                     "excluded); the results of the two sides are compared in full (counters, hashes, histograms)",
            "autotune": None if tuned is None else {
                k: tuned[k] for k in ("waves_per_block", "blocks", "lds_depth", "split_threshold",
                                      "check_interval", "trials")} | {
                "auto_solve_ms": tuned["auto_us"] / 1e3, "tuned_solve_ms": tuned["best_us"] / 1e3},
            "cliques": cliques, "nodes": nodes, "ms_per_batch": dt * 1e3, "device_solve_ms": device_ms,
            "cliques_per_s": cliques / dt, "nodes_per_s": nodes / dt,
            "plain_ms": dt_plain * 1e3, "plain_cliques_per_s": cliques / dt_plain,
            "vs_plain": dt_plain / dt}


# Table 1, GreedyBB columns at n = 10^4 (mean of 10 graphs on one Xeon
# E5-2690 v2 core): p -> (maximal cliques, steps, seconds)
PAPER_N10K = {0.001: (50.006e3, 7.434e3, 0.034), 0.003: (142.630e3, 13.242e3, 0.082),
              0.005: (215.789e3, 28.616e3, 0.133), 0.010: (349.705e3, 137.628e3, 0.299),
              0.030: (3.746762e6, 1.440393e6, 2.316)}


def table1_n10k(mce, synth, np, reps: int) -> dict:
    """The n = 10^4 rows of Table 1 (G(10^4, p), seed 0): whole job per graph,
    from the device rows to the result (handle, ordering, renumbering, the
    local graphs of the root children, search), best of reps; each result is
    checked against the committed oracle golden."""
    import torch
    with open(os.path.join(ROOT, "tests", "golden", "table1_n10k.json")) as f:
        gold = json.load(f)
    keys = ("count", "nodes", "children", "dead_ends", "hash_xor", "hash_sum", "omega", "hist")
    out = {}
    for p, (mu, steps, sec) in PAPER_N10K.items():
        rows = synth.gnp(10000, p, 0)
        d = torch.from_numpy(rows.view(np.int64)).cuda()
        torch.cuda.synchronize()
        best, res, st = None, None, None
        for _ in range(reps):
            t0 = time.perf_counter()
            g = mce.Graph(d)
            res = g.count()
            dt = time.perf_counter() - t0
            st = mce.last_stats()
            g.release()
            best = dt if best is None else min(best, dt)
        out["p=%g" % p] = {"ms": best * 1e3, "search_kernel_ms": st["search_kernel_us"] / 1e3,
                           "prepare_ms": st["prepare_us"] / 1e3, "local_graphs": st["local_graphs"],
                           "matches_golden": all(res[k] == gold["p=%g" % p][k] for k in keys),
                           "cliques": res["count"], "nodes": res["nodes"], "omega": res["omega"],
                           "cliques_per_s": res["count"] / best,
                           "paper": {"cliques": mu, "steps": steps, "seconds": sec,
                                     "time_ratio": sec / best}}
    return out


def serving(mce, synth, np, count: int, warm: int) -> dict:
    """Requests from the serving mix (n log-uniform in [64, 2048], p ~ U[0.2,
    0.9], E[mu] <= 1e6; the redraw keeps n below about 950), submitted with
    mce_submit at Poisson arrival times; latency = completion - arrival on the
    host monotonic clock, measured two ways: with the request prepared at its
    arrival (mce_prepare from host rows: validation, copy, ordering and
    renumbering in the latency) and with every request prepared beforehand.
    Capacity = the closed-loop rate of the same mix (all submitted at once);
    plain = the same handles solved one after the other with mce_count; open
    loop at 0.5 and 0.8 of the capacity."""
    specs = synth.serving_mix(count + warm, 11)
    graphs = [synth.gnp(n, p, seed) for n, p, seed in specs]
    handles = [mce.Graph(r) for r in graphs]
    ns = [r.shape[0] for r in graphs]
    for h in handles:              # every handle solved once: its workspace is allocated
        h.count()
    # plain: one request after the other, each a blocking mce_count
    t0 = time.perf_counter()
    plain_cl = sum(h.count()["count"] for h in handles[warm:])
    plain_wall = time.perf_counter() - t0

    def run(arrivals, prepare: bool):
        """arrivals: seconds from the start for requests warm..; returns
        (latencies, cliques, wall)."""
        pending, lat, cliques, made = {}, [], 0, []
        nxt, t0 = 0, time.perf_counter()
        total = len(arrivals)
        while len(lat) < total:
            now = time.perf_counter() - t0
            while nxt < total and arrivals[nxt] <= now:
                i = warm + nxt
                if prepare:
                    g = mce.Graph(graphs[i])
                    made.append(g)
                else:
                    g = handles[i]
                pending[mce.submit(g)] = (i, arrivals[nxt])
                nxt += 1
            for t in list(pending):
                i, a = pending[t]
                rc, res = mce.poll(t, ns[i], 0)
                if rc == mce.PENDING:
                    continue
                if rc != mce.OK:
                    raise mce.MceError(rc, "mce_poll")
                lat.append(time.perf_counter() - t0 - a)
                cliques += res["count"]
                del pending[t]
        wall = time.perf_counter() - t0
        for g in made:
            g.release()
        return lat, cliques, wall

    lat, cl, wall = run([0.0] * count, False)        # closed loop: everything at once
    capacity = count / wall
    result = {"workload": "serving mix, n log-uniform [64, 2048], p ~ U[0.2, 0.9], E[mu] <= 1e6, seed 11",
              "requests": count, "max_n": max(ns), "capacity_rps": capacity, "capacity_cliques_per_s": cl / wall,
              "plain_rps": count / plain_wall, "plain_cliques_per_s": plain_cl / plain_wall,
              "served_vs_plain": plain_wall / wall,
              "alone_share_pct": int(os.environ.get("MCE_SERVE_ALONE_PCT", "50"))}
    for frac in (0.5, 0.8):
        arr = list(synth.poisson_arrivals(count, frac * capacity, 13))
        for prep in (False, True):
            lat, cl, wall = run(arr, prep)
            lat = np.array(lat) * 1e3
            result["load_%g%s" % (frac, "_with_prepare" if prep else "")] = {
                "qps": frac * capacity, "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "cliques_per_s": cl / wall}
    for h in handles:
        h.release()
    return result


def config_legs(mce, synth, np, oracle_mod) -> dict:
    """The other single-graph workloads, each as a whole job from device rows
    (prepare + count + release), checked against expected results:
    G(100, 0.5) seeds 0-9 (against the oracle, run here), planted G(800, 0.5)
    and Moon-Moser k = 15 (against the committed oracle goldens and the
    closed forms), and one node of G(300, 0.8) with about 10^8 cliques below
    it (mce_count_subproblem, against its committed oracle golden; the whole
    graph's 10^12 cliques are beyond any oracle run)."""
    import torch
    gold_dir = os.path.join(ROOT, "tests", "golden")
    with open(os.path.join(gold_dir, "full_configs.json")) as f:
        gold = json.load(f)
    keys = ("count", "nodes", "children", "dead_ends", "hash_xor", "hash_sum", "omega")

    def whole_job(rows, reps):
        d = torch.from_numpy(rows.view(np.int64)).cuda()
        torch.cuda.synchronize()
        best, res = None, None
        for _ in range(reps):
            t0 = time.perf_counter()
            g = mce.Graph(d)
            res = g.count()
            g.release()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        return res, best

    out = {}
    # configs: G(100, 0.5), seeds 0-9
    tot_cl, tot_nodes, tot_s, ok = 0, 0, 0.0, True
    for seed in range(10):
        rows = synth.gnp(100, 0.5, seed)
        res, dt = whole_job(rows, 3)
        ref = oracle_mod.greedy(rows)
        ok = ok and all(res[k] == ref[k] for k in keys + ("hist",))
        tot_cl += res["count"]
        tot_nodes += res["nodes"]
        tot_s += dt
    out["gnp100_p0.5_seeds0-9"] = {"cliques": tot_cl, "nodes": tot_nodes, "ms_total": tot_s * 1e3,
                                   "cliques_per_s": tot_cl / tot_s, "nodes_per_s": tot_nodes / tot_s,
                                   "matches_oracle": ok}
    for name, rows in (("moon_moser_15", synth.moon_moser(15)),
                       ("planted800_p0.5_s0", synth.gnp_planted(800, 0.5, 0)[0])):
        res, dt = whole_job(rows, 3 if name.startswith("moon") else 1)
        ref = gold[name]
        out[name] = {"cliques": res["count"], "nodes": res["nodes"], "ms": dt * 1e3,
                     "cliques_per_s": res["count"] / dt, "nodes_per_s": res["nodes"] / dt,
                     "matches_golden": all(res[k] == ref[k] for k in keys) and res["hist"] == ref["hist"],
                     "golden_oracle_seconds": ref["oracle_seconds"], "golden_oracle_threads": ref["oracle_threads"]}
    node_path = os.path.join(gold_dir, "gnp300_p0.8_node.json")
    if os.path.exists(node_path):
        with open(node_path) as f:
            ref = json.load(f)
        rows = synth.gnp(300, 0.8, 0)
        g = mce.Graph(rows)
        g.count_subproblem(ref["R"], ref["P"], ref["X"])          # warm-up
        best, res = None, None
        for _ in range(3):
            t0 = time.perf_counter()
            res = g.count_subproblem(ref["R"], ref["P"], ref["X"])
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        g.release()
        out["gnp300_p0.8_node"] = {
            "node": {"R": len(ref["R"]), "P": len(ref["P"]), "X": len(ref["X"])},
            "cliques": res["count"], "nodes": res["nodes"], "ms": best * 1e3,
            "cliques_per_s": res["count"] / best, "nodes_per_s": res["nodes"] / best,
            "matches_golden": all(res[k] == ref[k] for k in keys) and res["hist"] == ref["hist"],
            "golden_oracle_seconds": ref["oracle_seconds"], "golden_oracle_threads": ref["oracle_threads"]}
    return out


def split_pieces(adj, limit: int):
    """Cut the GreedyBB search tree of a graph into subproblems: the top of
    the tree is expanded here in the library's own order (Alg. 4 with the
    GreedyBB pivot of Sec. 4.3: the first vertex of X, else of P, in
    position order; branch set L = P minus N(pivot), in increasing
    position; P and X updated after each child, steps 12-13) until every
    node left has at most `limit` candidates; those nodes are the pieces.
    adj: boolean adjacency over positions of the ordering.  Returns the
    pieces as (R, P, X) position lists and the expanded part's counters
    (nodes including the root, children, dead ends); a maximal clique at
    the expanded levels is an error (none occurs where the pieces are
    large).  Every clique is then found by the GPU below some piece, and
    the counters of the pieces plus the expanded part's are those of the
    whole search."""
    import numpy as np
    n = adj.shape[0]
    pieces, nodes, children, dead = [], 0, 0, 0
    stack = [([], np.ones(n, dtype=bool), np.zeros(n, dtype=bool))]
    while stack:
        R, P, X = stack.pop()
        if R and int(P.sum()) <= limit:
            pieces.append((R, [int(v) for v in np.flatnonzero(P)], [int(v) for v in np.flatnonzero(X)]))
            continue
        nodes += 1
        xs, ps = np.flatnonzero(X), np.flatnonzero(P)
        piv = xs[0] if xs.size else ps[0]
        P, X = P.copy(), X.copy()
        for v in np.flatnonzero(P & ~adj[piv]):
            children += 1
            P2, X2 = P & adj[v], X & adj[v]
            if not P2.any():
                if not X2.any():
                    raise RuntimeError("a maximal clique above the pieces: lower the limit")
                dead += 1
            else:
                stack.append((R + [int(v)], P2, X2))
            P[v] = False
            X[v] = True
    return pieces, {"nodes": nodes, "children": children, "dead_ends": dead}


def g300_full(mce, synth, np, part: int, parts: int, limit: int = 200) -> dict:
    """Part `part` of `parts` of the whole G(300, 0.8) graph, seed 0: the
    pieces of split_pieces (sorted by size, dealt out in turn) counted with
    mce_count_subproblem, their results added (hash_xor by XOR, hash_sum
    mod 2^64).  Part 0 also carries the expanded levels' counters."""
    rows = synth.gnp(300, 0.8, 0)
    g = mce.Graph(rows)
    order = g.order().astype(np.int64)
    adj = synth.unpack_rows(rows)[np.ix_(order, order)]
    pieces, top = split_pieces(adj, limit)
    pieces.sort(key=lambda q: (len(q[1]), q[0]))
    mine = pieces[part::parts]
    tot = {"count": 0, "nodes": 0, "children": 0, "dead_ends": 0, "hash_xor": 0, "hash_sum": 0, "omega": 0,
           "hist": [0] * 301}
    secs = 0.0
    for i, (R, P, X) in enumerate(mine):
        t0 = time.perf_counter()
        r = g.count_subproblem(R, P, X)
        secs += time.perf_counter() - t0
        for k in ("count", "nodes", "children", "dead_ends"):
            tot[k] += r[k]
        tot["hash_xor"] ^= r["hash_xor"]
        tot["hash_sum"] = (tot["hash_sum"] + r["hash_sum"]) % (1 << 64)
        tot["omega"] = max(tot["omega"], r["omega"])
        for j, c in enumerate(r["hist"]):
            tot["hist"][j] += c
        if (i + 1) % 100 == 0 or i + 1 == len(mine):
            print("g300 part %d/%d: %d of %d pieces, %.1f s of search, %.4g cliques" % (
                part, parts, i + 1, len(mine), secs, tot["count"]), file=sys.stderr, flush=True)
    g.release()
    if part == 0:
        for k in ("nodes", "children", "dead_ends"):
            tot[k] += top[k]
    return {"g300_part": part, "parts": parts, "limit": limit, "pieces": len(mine), "pieces_total": len(pieces),
            "expanded": top, "seconds": secs, **tot}


def g300_combine(paths) -> dict:
    """The parts' results added up into the whole graph's."""
    parts = []
    for path in paths:
        with open(path) as f:
            parts.append(json.loads([line for line in f if line.startswith("{")][-1]))
    n = parts[0]["parts"]
    assert sorted(p["g300_part"] for p in parts) == list(range(n)), "every part once"
    out = {"workload": "G(n=300, p=0.8) seed 0, whole graph", "parts": n, "limit": parts[0]["limit"],
           "pieces": sum(p["pieces"] for p in parts), "expanded": parts[0]["expanded"]}
    for k in ("count", "nodes", "children", "dead_ends", "seconds"):
        out[k] = sum(p[k] for p in parts)
    out["hash_xor"] = 0
    for p in parts:
        out["hash_xor"] ^= p["hash_xor"]
    out["hash_sum"] = sum(p["hash_sum"] for p in parts) % (1 << 64)
    out["omega"] = max(p["omega"] for p in parts)
    hist = [sum(p["hist"][j] for p in parts) for j in range(len(parts[0]["hist"]))]
    while hist and hist[-1] == 0:
        hist.pop()
    out["hist"] = hist
    out["cliques_per_s"] = out["count"] / out["seconds"]
    out["nodes_per_s"] = out["nodes"] / out["seconds"]
    return out


def pivot_rules(mce, d_rows, reps: int) -> dict:
    """The workload graph under each pivot rule of Sec. 4.3 (automatic
    schedule): the same cliques, different trees; solve time of one handle."""
    out = {}
    for rule in ("greedy", "greedy_tx", "tomita_bb"):
        mce.reset_options(watchdog_ms=120000, pivot=mce.PIVOT_RULES[rule])
        g = mce.Graph(d_rows)
        g.count()
        best = None
        for _ in range(reps):
            t0 = time.perf_counter()
            r = g.count()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        g.release()
        out[rule] = {"solve_ms": best * 1e3, "nodes": r["nodes"], "children": r["children"],
                     "cliques_per_s": r["count"] / best, "nodes_per_s": r["nodes"] / best}
    mce.reset_options(watchdog_ms=120000)
    return out


def streamed_enumerate(mce, d_rows) -> dict:
    """Every clique of the workload graph as sorted input ids, streamed to
    the host in chunks of 2^24 ids (mce_enumerate_stream, automatic
    schedule); the sink only counts what arrives."""
    g = mce.Graph(d_rows)
    got = [0, 0]

    def on_chunk(verts, pairs):
        got[0] += len(pairs)
        got[1] += len(verts)

    t0 = time.perf_counter()
    r = g.enumerate_stream(on_chunk)
    dt = time.perf_counter() - t0
    g.release()
    assert got[0] == r["count"]
    return {"seconds": dt, "cliques_per_s": r["count"] / dt, "ids": got[1],
            "host_bytes_per_s": (4 * got[1] + 16 * got[0]) / dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="gnp1000", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-rules", action="store_true", help="skip the pivot-rule comparison")
    ap.add_argument("--no-enumerate", action="store_true", help="skip the streamed enumeration")
    ap.add_argument("--no-table1", action="store_true", help="skip the n = 10^4 rows of Table 1")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--no-configs", action="store_true", help="skip the other single-graph workloads")
    ap.add_argument("--no-peaks", action="store_true", help="datasheet peaks instead of measured ones")
    ap.add_argument("--only-serving", action="store_true", help="the serving leg alone (no headline line)")
    ap.add_argument("--no-tune", action="store_true", help="automatic schedule instead of mce_autotune's")
    ap.add_argument("--opts", default="", metavar="K=V,...",
                    help="fixed schedule (library options such as waves_per_block=8,blocks=512); no tuning")
    ap.add_argument("--g300-full", default="", metavar="K/N",
                    help="part K of N of the whole G(300, 0.8) graph as subproblems (one JSON line)")
    ap.add_argument("--g300-combine", nargs="+", default=None, metavar="FILE",
                    help="add up the JSON lines of the --g300-full parts")
    args = ap.parse_args()

    if args.g300_combine:
        print(json.dumps(g300_combine(args.g300_combine)))
        return

    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe, max(args.steps, 1))
        return

    import numpy as np
    import torch
    import synth
    from paper_1801_00202_amd import mce

    torch.cuda.set_device(0)
    mce.load()
    mce.reset_options(watchdog_ms=120000)
    if args.only_serving:
        print(json.dumps({"serving": serving(mce, synth, np, args.serving_requests, warm=100)}))
        return
    if args.g300_full:
        k, n = (int(x) for x in args.g300_full.split("/"))
        print(json.dumps(g300_full(mce, synth, np, k, n)))
        return
    peaks = None if args.no_peaks else measured_peaks()
    wl = WORKLOADS[args.workload]
    rows = synth.gnp(wl["n"], wl["p"], wl["seed"])
    d_rows = torch.from_numpy(rows.view(np.int64)).cuda()
    torch.cuda.synchronize()

    # Schedule: mce_autotune on one handle of the workload graph (untimed), its
    # choice applied as options to the timed steps, which each make a new handle.
    tuned = None
    if args.opts:
        fixed = {k: int(v) for k, v in (kv.split("=") for kv in args.opts.split(","))}
        for k, v in fixed.items():
            mce.set_option(k, v)
        tuned = {"split_threshold": fixed.get("split_threshold"), "check_interval": fixed.get("check_interval"),
                 "fixed": fixed}
    elif not args.no_tune:
        g0 = mce.Graph(d_rows)
        tuned = g0.autotune()
        g0.release()
        for k in ("waves_per_block", "blocks", "lds_depth", "split_threshold", "check_interval"):
            mce.set_option(k, tuned[k])

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
    achieved = ops / (k_us * 1e-6) / 1e12
    lds_bytes = algorithmic_lds_bytes(first, wl["n"])
    lds_achieved = lds_bytes / (k_us * 1e-6) / 1e12
    valu_peak = VALU_PEAK_TOPS if peaks is None else peaks["valu_lane_ops_per_s"] / 1e12
    lds_peak = LDS_PEAK_TBPS if peaks is None else peaks["lds_bytes_per_s"] / 1e12
    traffic = recorded_traffic(args.workload)

    line = {
        "metric": "maximal cliques/sec + search nodes/sec per GPU vs plain; p50/p99 latency",
        "value": cliques_per_s,
        "unit": "cliques/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        # the paper reports times on one Xeon core, not this rate: context only
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "G(n=%d, p=%g) seed %d" % (wl["n"], wl["p"], wl["seed"]),
                   "cliques": first["count"], "nodes": first["nodes"], "children": first["children"],
                   "omega": first["omega"]},
        "nodes_per_s": nodes_per_s,
        "paper_context": None if args.workload != "gnp1000" else {
            "cliques_per_s": PAPER_G1000_CLIQUES_PER_S, "ratio": cliques_per_s / PAPER_G1000_CLIQUES_PER_S,
            "machine": "one Xeon E5-2690 v2 core, Table 1 (n=1000, p=0.3), mean of 10 graphs"},
        "search_kernel_ms": k_us / 1e3,
        "prepare_ms": sum(s["prepare_us"] for s in stats) / len(stats) / 1e3,
        "launch": {"blocks": stats[0]["blocks"], "waves_per_block": stats[0]["waves_per_block"],
                   "lds_depth": stats[0]["lds_depth"], "split_threshold": None if tuned is None else
                   tuned["split_threshold"], "check_interval": None if tuned is None else tuned["check_interval"],
                   "donations": stats[0]["donations"], "units": stats[0]["units"],
                   "busy_frac": stats[0]["busy_frac"], "tail_frac": stats[0]["tail_frac"]},
        "autotune": None if tuned is None or "fixed" in tuned else {
            "trials": tuned["trials"], "auto_solve_ms": tuned["auto_us"] / 1e3, "tuned_solve_ms": tuned["best_us"] / 1e3},
        "schedule_fixed": None if tuned is None else tuned.get("fixed"),
        "roofline": {"bound": "alu", "kernel": "search_kernel", "achieved": achieved, "peak": valu_peak,
                     "unit": "T int32 lane-ops/s", "frac": achieved / valu_peak,
                     "peak_source": "datasheet" if peaks is None else "measured (libmce_probe valu probe)",
                     "peak_datasheet": VALU_PEAK_TOPS,
                     "ops_per_launch": ops,
                     "traffic": None if traffic is None else traffic["hbm_bytes_per_launch"],
                     "lds": {"achieved": lds_achieved, "peak": lds_peak, "unit": "TB/s",
                             "frac": lds_achieved / lds_peak, "bytes_per_launch": lds_bytes,
                             "peak_source": "datasheet" if peaks is None else "measured (libmce_probe lds probe)",
                             "peak_datasheet": LDS_PEAK_TBPS}},
    }
    mce.reset_options(watchdog_ms=120000)
    if not args.no_rules:
        line["pivot_rules"] = pivot_rules(mce, d_rows, reps=3)
    if not args.no_enumerate:
        line["enumerate_stream"] = streamed_enumerate(mce, d_rows)
    if not args.no_table1:
        line["table1_n10k"] = table1_n10k(mce, synth, np, reps=3)
    if not args.no_batch:
        line["batched"] = batched(mce, synth, np, reps=3, tune=not args.no_tune)
    if not args.no_serving:
        line["serving"] = serving(mce, synth, np, args.serving_requests, warm=100)
    if not args.no_configs:
        import oracle
        line["configs"] = config_legs(mce, synth, np, oracle)
    if not args.no_cpu_baseline:
        import oracle
        # all cores of the affinity mask over the whole workload graph (root
        # children shared among threads), and one thread over the first 64 of
        # the graph's root children
        threads = args.cpu_threads or len(os.sched_getaffinity(0))
        c0 = time.perf_counter()
        ref = oracle.greedy(rows, threads=threads)
        cdt = time.perf_counter() - c0
        assert ref["count"] == first["count"] and ref["hash_xor"] == first["hash_xor"]
        c0 = time.perf_counter()
        part = oracle.greedy_range(rows, 0, 64)
        sdt = time.perf_counter() - c0
        line["cpu_baseline"] = dict(cpu_info(), **{
            "value": ref["count"] / cdt, "unit": "cliques/s", "cores": threads, "kind": "oracle",
            "seconds": cdt,
            "sample": "all-core: one full solve of the workload graph, root children shared among the threads; "
                      "single-thread: root children 0..63 of the workload graph",
            "single_thread": {"value": part["count"] / sdt, "unit": "cliques/s", "cores": 1, "seconds": sdt,
                              "cliques": part["count"]}})
    if peaks is not None:
        line["measured_peaks"] = peaks
    print(json.dumps(line))


if __name__ == "__main__":
    main()
