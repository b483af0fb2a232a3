"""The C ABI of libmce.so without a GPU: the library loads, exports every
function include/mce.h declares, and rejects bad input on the host before any
HIP call (no compute call is made here)."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mce.h")


@pytest.fixture(scope="module")
def lib(mce):
    return mce.load()


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return sorted(set(re.findall(r"\b(mce_[a-z_]+)\s*\(", src)))


PROBE_HEADER = os.path.join(ROOT, "include", "mce_probe.h")


def test_probe_library_exports_its_header():
    # the peak-rate probes (a measurement aid beside libmce.so)
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1801_00202_amd", "libmce_probe.so"))
    src = re.sub(r"/\*.*?\*/", "", open(PROBE_HEADER).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(mce_probe_[a-z_]+)\s*\(", src)))
    assert names == ["mce_probe_lds", "mce_probe_valu"]
    for name in names:
        assert hasattr(lib, name), name
    d = ctypes.c_double()
    # argument checks run before any HIP call
    lib.mce_probe_valu.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.mce_probe_valu(0, 10, ctypes.byref(d), None) == -1
    assert lib.mce_probe_valu(10, 10, None, None) == -1


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("mce_prepare", "mce_count", "mce_enumerate", "mce_submit", "mce_poll",
                 "mce_cancel", "mce_release", "mce_strerror"):
        assert must in names


def test_every_declared_symbol_is_exported(lib, mce):
    names = _declared()
    assert names, "no declarations found"
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(mce.EXPORTS) == names


def test_header_constants_match_binding(mce):
    src = open(HEADER).read()
    consts = {k: int(v, 0) for k, v in
              re.findall(r"#define\s+(MCE_[A-Z_0-9]+)\s+\(?(-?(?:0x)?[0-9a-fA-F]+)u?\)?", src)}
    assert consts["MCE_OK"] == mce.OK and consts["MCE_PENDING"] == mce.PENDING
    assert consts["MCE_E_INVAL"] == mce.E_INVAL and consts["MCE_E_NOMEM"] == mce.E_NOMEM
    assert consts["MCE_E_TRUNCATED"] == mce.E_TRUNCATED and consts["MCE_E_DEVICE"] == mce.E_DEVICE
    assert consts["MCE_E_BUSY"] == mce.E_BUSY and consts["MCE_E_CANCELLED"] == mce.E_CANCELLED
    for name, key in mce.OPTIONS.items():
        assert consts["MCE_OPT_" + name.upper()] == key
    assert consts["MCE_MAX_N"] == mce.MAX_N and consts["MCE_F_DEVICE_PTR"] == mce.F_DEVICE_PTR


def test_result_struct_layout(mce):
    # 6 x u64, omega, hist_len, hist pointer, status, reserved
    assert ctypes.sizeof(mce.Result) == 6 * 8 + 4 + 4 + 8 + 4 + 4


def test_strerror(lib, mce):
    msgs = {c: lib.mce_strerror(c).decode() for c in
            (mce.OK, mce.PENDING, mce.E_INVAL, mce.E_NOMEM, mce.E_TRUNCATED, mce.E_DEVICE, mce.E_BUSY,
             mce.E_CANCELLED)}
    assert all(msgs.values()) and len(set(msgs.values())) == len(msgs)
    assert lib.mce_strerror(12345).decode() == "unknown status"


def _prepare(lib, rows, row_words=None, n=None, batch=None, flags=0, out=True):
    h = ctypes.c_void_p()
    ptr = rows.ctypes.data if rows is not None else None
    if n is None:
        n = rows.shape[0] if rows is not None else 0
    if row_words is None:
        row_words = rows.shape[1] if rows is not None else 0
    return lib.mce_prepare(n, ptr, row_words, batch, flags, None, ctypes.byref(h) if out else None)


def test_prepare_rejects_bad_graphs(lib, mce):
    ok = synth.gnp(70, 0.5, 0)
    assert _prepare(lib, ok, out=False) == mce.E_INVAL            # no handle pointer
    assert _prepare(lib, ok, flags=0x80) == mce.E_INVAL           # unknown flag
    assert _prepare(lib, ok, n=70, row_words=1) == mce.E_INVAL    # rows too short for n
    assert _prepare(lib, None, n=5, row_words=1) == mce.E_INVAL   # NULL rows
    big = np.zeros((mce.MAX_N + 1, (mce.MAX_N + 64) // 64), dtype=np.uint64)
    assert _prepare(lib, big) == mce.E_INVAL                      # n above the limit
    loop = ok.copy()
    loop[3, 0] |= np.uint64(1 << 3)
    assert _prepare(lib, loop) == mce.E_INVAL                     # self-loop
    asym = synth.empty(70)
    asym[1, 0] |= np.uint64(1 << 5)
    assert _prepare(lib, asym) == mce.E_INVAL                     # 1~5 but not 5~1
    pad = ok.copy()
    pad[2, 1] |= np.uint64(1 << 63)                               # column 127 >= n
    assert _prepare(lib, pad) == mce.E_INVAL


def test_prepare_rejects_bad_batches(lib, mce):
    g0, g1 = synth.gnp(40, 0.5, 1), synth.gnp(90, 0.3, 2)
    flat = np.concatenate([g0.ravel(), g1.ravel()])
    ns = (ctypes.c_uint32 * 2)(40, 90)
    offs = (ctypes.c_uint64 * 2)(0, g0.size)

    def run(num, ns_, offs_, words):
        b = mce.Batch(num, ns_, offs_)
        h = ctypes.c_void_p()
        return lib.mce_prepare(0, flat.ctypes.data, words, ctypes.byref(b), 0, None, ctypes.byref(h))

    assert run(0, ns, offs, flat.size) == mce.E_INVAL                       # empty batch
    assert run(2, None, offs, flat.size) == mce.E_INVAL                     # no sizes
    assert run(2, ns, (ctypes.c_uint64 * 2)(0, g0.size + 1), flat.size) == mce.E_INVAL  # past the end
    assert run(2, (ctypes.c_uint32 * 2)(40, 5000), offs, flat.size) == mce.E_INVAL      # n too large
    bad = flat.copy()
    bad[g0.size + 3 * g1.shape[1]] |= np.uint64(1 << 3)                     # self-loop in graph 1
    b = mce.Batch(2, ns, offs)
    h = ctypes.c_void_p()
    assert lib.mce_prepare(0, bad.ctypes.data, bad.size, ctypes.byref(b), 0, None, ctypes.byref(h)) == mce.E_INVAL


def test_null_handles(lib, mce):
    res = mce.Result()
    assert lib.mce_count(None, ctypes.byref(res), None) == mce.E_INVAL
    assert lib.mce_count_range(None, 0, 1, ctypes.byref(res), None) == mce.E_INVAL
    one = (ctypes.c_uint32 * 1)(0)
    assert lib.mce_count_subproblem(None, None, 0, one, 1, None, 0, ctypes.byref(res), None) == mce.E_INVAL
    assert lib.mce_enumerate(None, None, 0, None, 0, None, None, ctypes.byref(res), None) == mce.E_INVAL
    n = ctypes.c_uint32()
    assert lib.mce_num_graphs(None, ctypes.byref(n)) == mce.E_INVAL
    assert lib.mce_get_order(None, 0, None, 0) == mce.E_INVAL
    t = ctypes.c_uint64()
    assert lib.mce_submit(None, 0, ctypes.byref(t)) == mce.E_INVAL
    assert lib.mce_poll(987654321, ctypes.byref(res), 0) == mce.E_INVAL   # unknown ticket
    assert lib.mce_poll(1, None, 0) == mce.E_INVAL
    assert lib.mce_release(None) == mce.OK
    assert lib.mce_last_stats(None) == mce.E_INVAL
    assert lib.mce_autotune(None, 0, None, None) == mce.E_INVAL
    assert lib.mce_clear_tuning(None) == mce.E_INVAL


def test_tune_and_stats_struct_layout(mce):
    # five u32 choices, trials, two doubles
    assert ctypes.sizeof(mce.Tune) == 6 * 4 + 2 * 8
    # three doubles, four u32, five u64, two u32, three doubles
    assert ctypes.sizeof(mce.Stats) == 3 * 8 + 4 * 4 + 5 * 8 + 2 * 4 + 3 * 8


def test_options(lib, mce):
    v = ctypes.c_int64()
    try:
        assert lib.mce_set_option(999, 1) == mce.E_INVAL
        assert lib.mce_get_option(999, ctypes.byref(v)) == mce.E_INVAL
        assert lib.mce_get_option(1, None) == mce.E_INVAL
        assert lib.mce_set_option(mce.OPTIONS["waves_per_block"], 17) == mce.E_INVAL
        assert lib.mce_set_option(mce.OPTIONS["queue_cap"], 1000) == mce.E_INVAL    # not a power of two
        assert lib.mce_set_option(mce.OPTIONS["lds_depth"], -2) == mce.E_INVAL
        assert lib.mce_set_option(mce.OPTIONS["graph"], 3) == mce.E_INVAL
        assert lib.mce_set_option(mce.OPTIONS["pivot"], 3) == mce.E_INVAL
        assert lib.mce_set_option(mce.OPTIONS["local_graphs"], 2) == mce.E_INVAL
        for name, key in mce.OPTIONS.items():
            val = 2 if name in ("graph", "pivot") else 0 if name == "local_graphs" else 4
            assert lib.mce_set_option(key, val) == mce.OK
            assert lib.mce_get_option(key, ctypes.byref(v)) == mce.OK and v.value == val
    finally:
        mce.reset_options()
    for name, key in mce.OPTIONS.items():
        assert lib.mce_get_option(key, ctypes.byref(v)) == mce.OK and v.value == mce.DEFAULTS[name]


def test_python_edge_list_helper():
    rows = synth.edge_list_to_rows(4, [(0, 1), (1, 0), (2, 3)])
    adj = synth.unpack_rows(rows)
    assert adj.sum() == 4 and adj[0, 1] and adj[3, 2]
    with pytest.raises(ValueError):
        synth.edge_list_to_rows(3, [(1, 1)])


@pytest.mark.parametrize("n,p,seed,limit", [(60, 0.7, 3, 30), (90, 0.5, 4, 40)])
def test_split_pieces_cover_the_search(orc, n, p, seed, limit):
    """The cut of the search tree used by the whole-G(300, 0.8) measurement
    (bench.split_pieces), checked on the CPU with the oracle: the pieces'
    subproblems plus the expanded levels' counters give the whole search's
    count, nodes, children, dead ends, hashes and histogram."""
    import bench
    rows = synth.gnp(n, p, seed)
    order = np.asarray(orc.order(rows), dtype=np.int64)
    adj = synth.unpack_rows(rows)[np.ix_(order, order)]
    pieces, top = bench.split_pieces(adj, limit)
    assert len(pieces) > 5 and top["nodes"] > 1
    pos_rows = synth.pack_rows(adj)
    tot = dict(top, count=0, hash_xor=0, hash_sum=0, omega=0)
    hist = [0] * (n + 1)
    for R, P, X in pieces:
        r = orc.subproblem(pos_rows, R, P, X, ids=order)
        for k in ("count", "nodes", "children", "dead_ends"):
            tot[k] += r[k]
        tot["hash_xor"] ^= r["hash_xor"]
        tot["hash_sum"] = (tot["hash_sum"] + r["hash_sum"]) % (1 << 64)
        tot["omega"] = max(tot["omega"], r["omega"])
        for j, c in enumerate(r["hist"]):
            hist[j] += c
    ref = orc.greedy(rows)
    for k in ("count", "nodes", "children", "dead_ends", "hash_xor", "hash_sum", "omega"):
        assert tot[k] == ref[k], k
    rh = list(ref["hist"])
    assert hist[:len(rh)] == rh and not any(hist[len(rh):])
