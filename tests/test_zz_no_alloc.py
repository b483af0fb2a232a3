"""mce_count_noalloc (the entry point that allocates nothing) against the
allocating path it mirrors, mce_prepare + mce_count, and the oracle: two calls
in a row, the second on a smaller graph, plus the size limit, rows wider than
ceil(n/64) words and a stack deeper than one spill chunk."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

KEYS = ("count", "nodes", "children", "dead_ends", "hash_xor", "hash_sum", "omega", "hist")


def same(a, b):
    for k in KEYS:
        assert a[k] == b[k], "%s: %r != %r" % (k, a[k], b[k])


@pytest.fixture(autouse=True)
def _opts(mce):
    mce.reset_options(watchdog_ms=20000)
    yield
    mce.reset_options(watchdog_ms=20000)


def _dev(rows):
    import torch
    return torch.from_numpy(np.ascontiguousarray(rows).view(np.int64)).cuda()


def _allocating(mce, rows):
    g = mce.Graph(rows)
    try:
        return g.count()
    finally:
        g.release()


def test_noalloc_two_calls_second_smaller(mce, orc):
    for rows in (synth.gnp(700, 0.4, 3), synth.gnp(150, 0.5, 4)):
        got = mce.count_noalloc(_dev(rows))
        same(got, _allocating(mce, rows))
        same(got, orc.greedy(rows, threads=8))


def test_noalloc_limits_and_shapes(mce, orc):
    import torch
    # the largest graph it takes, then a deep chain (K_300: 300 nested nodes,
    # deeper than the LDS window plus one spill chunk), then wide rows
    rows = synth.gnp(2048, 0.05, 5)
    same(mce.count_noalloc(_dev(rows)), _allocating(mce, rows))
    rows = synth.complete(300)
    same(mce.count_noalloc(_dev(rows)), orc.greedy(rows))
    base = synth.gnp(90, 0.5, 6)
    wide = np.zeros((90, 4), dtype=np.uint64)
    wide[:, :base.shape[1]] = base
    same(mce.count_noalloc(_dev(wide)), orc.greedy(base))
    # n = 0: the empty clique
    r = mce.count_noalloc(torch.zeros((0, 1), dtype=torch.int64, device="cuda"))
    assert r["count"] == 1 and r["nodes"] == 0
    # one vertex over the limit, and a non-simple graph
    with pytest.raises(mce.MceError) as e:
        mce.count_noalloc(_dev(synth.gnp(mce.NOALLOC_MAX_N + 1, 0.01, 7)))
    assert e.value.code == mce.E_INVAL
    bad = synth.gnp(80, 0.5, 8)
    bad[3, 0] |= np.uint64(1 << 3)
    with pytest.raises(mce.MceError) as e:
        mce.count_noalloc(_dev(bad))
    assert e.value.code == mce.E_INVAL
