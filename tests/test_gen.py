"""The seeded input generator: determinism, CSR well-formedness and workload statistics."""
import numpy as np

import gen


def _check_csr(g):
    off, idx = g.offsets, g.indices
    assert off[0] == 0 and off[-1] == idx.shape[0]
    assert np.all(np.diff(off) >= 0)
    n = g.n
    assert idx.min(initial=0) >= 0 and idx.max(initial=0) < n
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(off))
    assert np.all(src != idx)                                   # no self-loops
    key = src * n + idx
    assert np.unique(key).shape[0] == key.shape[0]              # no duplicates
    rkey = idx.astype(np.int64) * n + src
    assert np.array_equal(np.sort(key), np.sort(rkey))          # symmetric


def test_tiny_deterministic_and_shaped():
    a, b = gen.c0(), gen.c0()
    assert np.array_equal(a.offsets, b.offsets) and np.array_equal(a.indices, b.indices)
    assert np.array_equal(a.membership, b.membership)
    _check_csr(a)
    assert a.n == 2000
    assert np.bincount(a.membership).tolist() == [100] * 20
    assert a.meta["inter_edges"] == 2000
    c = gen.c0(seed=5)
    assert not np.array_equal(a.indices, c.indices)


def test_chung_lu_small_statistics():
    g = gen.chung_lu(20000, 40.0, 2.5, 11, 500, 2.0, 0.2, 0.15, 0.05, 1, seed=3, intra_mult=1.8,
                     nthreads=4)
    _check_csr(g)
    sizes = np.bincount(g.membership)
    assert sizes.min() >= 11 and sizes.max() <= 500 + 11
    assert 0.1 < g.meta["mixing"] < 0.35
    h = gen.chung_lu(20000, 40.0, 2.5, 11, 500, 2.0, 0.2, 0.15, 0.05, 1, seed=3, intra_mult=1.8,
                     nthreads=1)
    assert np.array_equal(g.indices, h.indices)                 # thread-count independent
