"""ctypes binding of libmce.so (include/mce.h).  Argument marshalling only: every
step of the enumeration runs in the HIP library.  There is no fallback: if the
library is missing or cannot be loaded, every call raises.

Graphs are adjacency bitset rows, ``uint64[n, row_words]`` (LSB first), as a
numpy array, a CPU tensor, or a device tensor (passed by pointer with
``MCE_F_DEVICE_PTR``).  PyTorch is only used to hand over device memory and the
current HIP stream.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmce.so")

OK = 0
PENDING = 1
E_INVAL = -1
E_NOMEM = -2
E_TRUNCATED = -3
E_DEVICE = -4
E_BUSY = -5
E_CANCELLED = -6
F_DEVICE_PTR = 0x1
MAX_N = 16384

OPTIONS = {
    "waves_per_block": 1,
    "blocks": 2,
    "lds_depth": 3,
    "split_threshold": 4,
    "check_interval": 5,
    "queue_cap": 6,
    "watchdog_ms": 7,
    "graph": 8,
    "refresh_children": 9,
    "pivot": 10,
    "local_graphs": 11,
}
DEFAULTS = {
    "waves_per_block": 0, "blocks": 0, "lds_depth": -1, "split_threshold": 0,
    "check_interval": 0, "queue_cap": 0, "watchdog_ms": 0, "graph": 1, "refresh_children": 0,
    "pivot": 0, "local_graphs": 1,
}
# values of the "pivot" option (MCE_OPT_PIVOT)
PIVOT_RULES = {"greedy": 0, "tomita_bb": 1, "greedy_tx": 2}


class MceError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = _lib().mce_strerror(code).decode() if _LIB is not None else str(code)
        super().__init__("%s: %s (%d)" % (what or "mce", msg, code))


class Result(ctypes.Structure):
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
        ("status", ctypes.c_int32),
        ("reserved", ctypes.c_uint32),
    ]


class Batch(ctypes.Structure):
    _fields_ = [
        ("num_graphs", ctypes.c_uint32),
        ("n", ctypes.POINTER(ctypes.c_uint32)),
        ("row_offset_words", ctypes.POINTER(ctypes.c_uint64)),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("prepare_us", ctypes.c_double),
        ("search_us", ctypes.c_double),
        ("search_kernel_us", ctypes.c_double),
        ("blocks", ctypes.c_uint32),
        ("waves_per_block", ctypes.c_uint32),
        ("lds_depth", ctypes.c_uint32),
        ("lds_bytes_per_block", ctypes.c_uint32),
        ("donations", ctypes.c_uint64),
        ("units", ctypes.c_uint64),
        ("spills", ctypes.c_uint64),
        ("checks", ctypes.c_uint64),
        ("flushes", ctypes.c_uint64),
        ("attempts", ctypes.c_uint32),
        ("local_graphs", ctypes.c_uint32),
        ("busy_frac", ctypes.c_double),
        ("ramp_frac", ctypes.c_double),
        ("tail_frac", ctypes.c_double),
    ]


class Tune(ctypes.Structure):
    _fields_ = [
        ("waves_per_block", ctypes.c_uint32),
        ("blocks", ctypes.c_uint32),
        ("lds_depth", ctypes.c_uint32),
        ("split_threshold", ctypes.c_uint32),
        ("check_interval", ctypes.c_uint32),
        ("trials", ctypes.c_uint32),
        ("auto_us", ctypes.c_double),
        ("best_us", ctypes.c_double),
    ]


EXPORTS = (
    "mce_prepare", "mce_num_graphs", "mce_get_order", "mce_root_branches", "mce_count",
    "mce_count_range", "mce_count_subproblem", "mce_enumerate", "mce_submit", "mce_poll", "mce_cancel", "mce_release",
    "mce_strerror", "mce_set_option", "mce_get_option", "mce_last_stats", "mce_autotune", "mce_clear_tuning",
    "mce_enumerate_stream", "mce_count_noalloc",
)

# mce_clique_sink_t
SINK = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32),
                        ctypes.POINTER(ctypes.c_uint64), ctypes.c_uint64)

_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmce.so is not built (run __graft_entry__.build() or "
                              "python paper_1801_00202_amd/build.py)")
        # One HIP runtime per process: when PyTorch is present its HIP runtime
        # must be the one libmce binds to (same soname), so that device
        # pointers and streams handed over from torch are valid in the library.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(LIB_PATH)
        u32, u64, i32, vp = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p
        p64 = ctypes.POINTER(ctypes.c_uint64)
        p32 = ctypes.POINTER(ctypes.c_uint32)
        pres = ctypes.POINTER(Result)
        lib.mce_prepare.argtypes = [u32, vp, u32, ctypes.POINTER(Batch), u32, vp, ctypes.POINTER(vp)]
        lib.mce_num_graphs.argtypes = [vp, p32]
        lib.mce_get_order.argtypes = [vp, u32, p32, u32]
        lib.mce_root_branches.argtypes = [vp, u32, p64]
        lib.mce_count.argtypes = [vp, pres, vp]
        lib.mce_count_range.argtypes = [vp, u64, u64, pres, vp]
        lib.mce_count_subproblem.argtypes = [vp, p32, u32, p32, u32, p32, u32, pres, vp]
        lib.mce_enumerate.argtypes = [vp, vp, u64, vp, u64, p64, p64, pres, vp]
        lib.mce_submit.argtypes = [vp, u32, p64]
        lib.mce_poll.argtypes = [u64, pres, ctypes.c_int32]
        lib.mce_cancel.argtypes = [u64]
        lib.mce_release.argtypes = [vp]
        lib.mce_strerror.argtypes = [i32]
        lib.mce_strerror.restype = ctypes.c_char_p
        lib.mce_set_option.argtypes = [i32, ctypes.c_int64]
        lib.mce_get_option.argtypes = [i32, ctypes.POINTER(ctypes.c_int64)]
        lib.mce_last_stats.argtypes = [ctypes.POINTER(Stats)]
        lib.mce_autotune.argtypes = [vp, u32, ctypes.POINTER(Tune), vp]
        lib.mce_clear_tuning.argtypes = [vp]
        lib.mce_enumerate_stream.argtypes = [vp, u64, SINK, vp, pres, vp]
        lib.mce_count_noalloc.argtypes = [u32, vp, u32, pres, vp]
        for name in EXPORTS:
            if name != "mce_strerror":
                getattr(lib, name).restype = i32
        _LIB = lib
    return _LIB


def load():
    """Load libmce.so (raises ImportError if it is missing)."""
    return _lib()


def _check(rc: int, what: str):
    if rc != OK:
        raise MceError(rc, what)


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # torch.cuda.Stream


def _new_result(n: int):
    hist = np.zeros(n + 1, dtype=np.uint64)
    r = Result()
    r.hist_len = hist.size
    r.hist = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    return r, hist


def _to_dict(r: Result, hist: np.ndarray) -> dict:
    # the histogram without trailing zeros (at least one entry)
    nz = np.flatnonzero(hist)
    h = hist[:max(int(nz[-1]) + 1 if nz.size else 1, 1)].tolist()
    return {
        "count": int(r.count), "nodes": int(r.nodes), "children": int(r.children),
        "dead_ends": int(r.dead_ends), "hash_xor": int(r.hash_xor), "hash_sum": int(r.hash_sum),
        "omega": int(r.omega), "hist": h, "status": int(r.status),
    }


def _as_rows(rows):
    """-> (pointer, n, row_words, flags, keepalive)."""
    try:
        import torch
        if isinstance(rows, torch.Tensor):
            if rows.dtype not in (torch.int64, torch.uint64):
                raise TypeError("rows tensor must be 64-bit")
            if rows.dim() != 2:
                raise ValueError("rows must be [n, row_words]")
            rows = rows.contiguous()
            flags = F_DEVICE_PTR if rows.is_cuda else 0
            return rows.data_ptr(), rows.shape[0], rows.shape[1], flags, rows
    except ImportError:
        pass
    a = np.ascontiguousarray(rows, dtype=np.uint64)
    if a.ndim != 2:
        raise ValueError("rows must be a 2-D uint64 array [n, row_words]")
    return a.ctypes.data, a.shape[0], a.shape[1], 0, a


class Graph:
    """A prepared graph (or batch of graphs) resident on the device."""

    def __init__(self, rows=None, *, batch=None, stream=None):
        lib = _lib()
        self._h = ctypes.c_void_p()
        self._n = []
        if batch is None:
            ptr, n, rw, flags, keep = _as_rows(rows)
            if n == 0:
                ptr = None
            _check(lib.mce_prepare(n, ptr, rw, None, flags, _stream_ptr(stream),
                                   ctypes.byref(self._h)), "mce_prepare")
            self._n = [n]
        else:
            graphs = list(batch)
            mats = [np.ascontiguousarray(g, dtype=np.uint64) for g in graphs]
            ns = np.array([m.shape[0] for m in mats], dtype=np.uint32)
            offs = np.zeros(len(mats), dtype=np.uint64)
            words = 0
            for i, m in enumerate(mats):
                offs[i] = words
                words += m.shape[0] * ((m.shape[0] + 63) // 64)
            packed = np.zeros(max(words, 1), dtype=np.uint64)
            for i, m in enumerate(mats):
                rw = (m.shape[0] + 63) // 64
                if m.shape[0]:
                    packed[int(offs[i]):int(offs[i]) + m.shape[0] * rw] = m[:, :rw].reshape(-1)
            b = Batch()
            b.num_graphs = len(mats)
            b.n = ns.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
            b.row_offset_words = offs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
            _check(lib.mce_prepare(0, packed.ctypes.data, words, ctypes.byref(b), 0,
                                   _stream_ptr(stream), ctypes.byref(self._h)), "mce_prepare")
            self._n = [int(x) for x in ns]

    @property
    def handle(self):
        return self._h

    @property
    def num_graphs(self) -> int:
        return len(self._n)

    def order(self, i: int = 0) -> np.ndarray:
        n = self._n[i]
        out = np.zeros(max(n, 1), dtype=np.uint32)
        _check(_lib().mce_get_order(self._h, i, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                    out.size), "mce_get_order")
        return out[:n]

    def root_branches(self, i: int = 0) -> int:
        out = ctypes.c_uint64()
        _check(_lib().mce_root_branches(self._h, i, ctypes.byref(out)), "mce_root_branches")
        return int(out.value)

    def count(self, stream=None):
        """Single graph: a result dict.  Batch: a list of result dicts."""
        k = len(self._n)
        arr = (Result * k)()
        # one histogram buffer for all graphs, each result pointing at its part
        lens = np.asarray(self._n, dtype=np.int64) + 1
        offs = np.concatenate(([0], np.cumsum(lens)))
        buf = np.zeros(int(offs[-1]), dtype=np.uint64)
        base = buf.ctypes.data
        p64 = ctypes.POINTER(ctypes.c_uint64)
        for i in range(k):
            arr[i].hist_len = int(lens[i])
            arr[i].hist = ctypes.cast(base + 8 * int(offs[i]), p64)
        _check(_lib().mce_count(self._h, arr, _stream_ptr(stream)), "mce_count")
        out = [_to_dict(arr[i], buf[offs[i]:offs[i + 1]]) for i in range(k)]
        return out[0] if k == 1 else out

    def count_range(self, first: int, last: int, stream=None) -> dict:
        r, h = _new_result(self._n[0])
        _check(_lib().mce_count_range(self._h, first, last, ctypes.byref(r), _stream_ptr(stream)),
               "mce_count_range")
        return _to_dict(r, h)

    def count_subproblem(self, R, P, X, stream=None) -> dict:
        """The search below node (R, P, X), vertices given as positions of the
        ordering (see order())."""
        def arr(x):
            a = np.ascontiguousarray(list(x) or [0], dtype=np.uint32)
            return a, len(x)
        (ra, nr), (pa, npp), (xa, nx) = arr(R), arr(P), arr(X)
        p32 = ctypes.POINTER(ctypes.c_uint32)
        r, h = _new_result(self._n[0])
        _check(_lib().mce_count_subproblem(self._h, ra.ctypes.data_as(p32), nr, pa.ctypes.data_as(p32), npp,
                                           xa.ctypes.data_as(p32), nx, ctypes.byref(r), _stream_ptr(stream)),
               "mce_count_subproblem")
        return _to_dict(r, h)

    def enumerate(self, verts=None, offsets=None, stream=None):
        """Returns (result, verts, offsets) with device tensors.  Without given
        buffers, a first call sizes them from the count."""
        import torch
        lib = _lib()
        n = self._n[0]
        vneed = ctypes.c_uint64()
        oneed = ctypes.c_uint64()
        if verts is None or offsets is None:
            r, h = _new_result(n)
            rc = lib.mce_enumerate(self._h, None, 0, None, 0, ctypes.byref(vneed), ctypes.byref(oneed),
                                   ctypes.byref(r), _stream_ptr(stream))
            if rc not in (OK, E_TRUNCATED):
                raise MceError(rc, "mce_enumerate")
            dev = torch.device("cuda", torch.cuda.current_device())
            verts = torch.zeros(max(int(vneed.value), 1), dtype=torch.int32, device=dev)
            offsets = torch.zeros(max(int(oneed.value), 2), dtype=torch.int64, device=dev)
        r, h = _new_result(n)
        rc = lib.mce_enumerate(self._h, verts.data_ptr(), verts.numel(), offsets.data_ptr(),
                               offsets.numel(), ctypes.byref(vneed), ctypes.byref(oneed),
                               ctypes.byref(r), _stream_ptr(stream))
        res = _to_dict(r, h)
        res["verts_needed"] = int(vneed.value)
        res["offsets_needed"] = int(oneed.value)
        if rc not in (OK, E_TRUNCATED):
            raise MceError(rc, "mce_enumerate")
        res["truncated"] = rc == E_TRUNCATED
        return res, verts, offsets

    def enumerate_stream(self, on_chunk, chunk_verts: int = 0, stream=None) -> dict:
        """mce_enumerate_stream: on_chunk(verts, pairs) is called per chunk
        with numpy copies (pairs[j] = (begin, end) of clique j in verts);
        a true return value stops the enumeration.  Returns the totals, with
        "cancelled" set when on_chunk stopped it."""
        failure = []

        def _sink(_user, v, o, count):
            try:
                pairs = np.ctypeslib.as_array(o, shape=(2 * int(count),)).reshape(-1, 2).copy()
                nv = int(pairs[:, 1].max()) if count else 0
                verts = np.ctypeslib.as_array(v, shape=(max(nv, 1),))[:nv].copy()
                return 1 if on_chunk(verts, pairs) else 0
            except BaseException as e:  # stop the library, re-raise below
                failure.append(e)
                return 1

        cb = SINK(_sink)
        r, h = _new_result(self._n[0])
        rc = _lib().mce_enumerate_stream(self._h, int(chunk_verts), cb, None, ctypes.byref(r), _stream_ptr(stream))
        if failure:
            raise failure[0]
        if rc not in (OK, E_CANCELLED):
            raise MceError(rc, "mce_enumerate_stream")
        out = _to_dict(r, h)
        out["cancelled"] = rc == E_CANCELLED
        return out

    def autotune(self, max_trials: int = 0, stream=None) -> dict:
        """mce_autotune: time candidate schedules on this handle and keep the
        fastest (results must agree exactly across all of them)."""
        t = Tune()
        _check(_lib().mce_autotune(self._h, int(max_trials), ctypes.byref(t), _stream_ptr(stream)),
               "mce_autotune")
        return {f: getattr(t, f) for f, _ in Tune._fields_}

    def clear_tuning(self):
        _check(_lib().mce_clear_tuning(self._h), "mce_clear_tuning")

    def release(self):
        if self._h:
            _check(_lib().mce_release(self._h), "mce_release")
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            if self._h and _LIB is not None:
                _LIB.mce_release(self._h)
        except Exception:
            pass


def cliques_from_output(verts, offsets, count: int):
    """Host list of cliques (tuples of sorted input ids) from enumerate buffers."""
    v = verts.cpu().numpy().astype(np.int64)
    o = offsets.cpu().numpy()[: 2 * count]
    return [tuple(int(x) for x in v[o[2 * i]:o[2 * i + 1]]) for i in range(count)]


NOALLOC_MAX_N = 2048


def count_noalloc(rows, stream=None) -> dict:
    """mce_count_noalloc: the whole path of one graph given as a DEVICE
    tensor [n, row_words] of 64-bit words, with no allocation in the
    library."""
    import torch
    if not isinstance(rows, torch.Tensor) or not rows.is_cuda:
        raise TypeError("count_noalloc takes the rows as a device tensor")
    if rows.dtype not in (torch.int64, torch.uint64) or rows.dim() != 2:
        raise ValueError("rows must be a 2-D 64-bit tensor [n, row_words]")
    rows = rows.contiguous()
    n, rw = rows.shape
    r, h = _new_result(n)
    _check(_lib().mce_count_noalloc(n, rows.data_ptr() if n else None, rw, ctypes.byref(r), _stream_ptr(stream)),
           "mce_count_noalloc")
    return _to_dict(r, h)


def submit(graph: Graph, flags: int = 0) -> int:
    t = ctypes.c_uint64()
    _check(_lib().mce_submit(graph.handle, flags, ctypes.byref(t)), "mce_submit")
    return int(t.value)


def poll(ticket: int, n: int, timeout_us: int = -1):
    """-> (status, result dict or None)."""
    r, h = _new_result(n)
    rc = _lib().mce_poll(ticket, ctypes.byref(r), timeout_us)
    if rc == OK:
        return rc, _to_dict(r, h)
    return rc, None


def cancel(ticket: int) -> int:
    return int(_lib().mce_cancel(ticket))


def set_option(name: str, value: int):
    _check(_lib().mce_set_option(OPTIONS[name], int(value)), "mce_set_option")


def reset_options(**overrides):
    """Restore every option to its default, then apply overrides."""
    for k, v in DEFAULTS.items():
        set_option(k, overrides.get(k, v))


def get_option(name: str) -> int:
    v = ctypes.c_int64()
    _check(_lib().mce_get_option(OPTIONS[name], ctypes.byref(v)), "mce_get_option")
    return int(v.value)


def last_stats() -> dict:
    s = Stats()
    _check(_lib().mce_last_stats(ctypes.byref(s)), "mce_last_stats")
    return {f: getattr(s, f) for f, _ in Stats._fields_}


def strerror(code: int) -> str:
    return _lib().mce_strerror(code).decode()
