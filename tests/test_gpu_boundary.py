"""The C-ABI boundary at its limits, against the oracle: exact uncapped cuts of dense sets
(bounds far above 62 key levels, including bounds above 126 that take the two-step
next-vertex reduction), the square-root and linear criteria on dense clusters whose cut
bounds exceed 62, and the rejection of malformed CSR input (duplicate entries,
out-of-range ids, self-loops, asymmetric entries, bad offsets) with WCC_EGRAPH."""
import numpy as np
import pytest

import oracle
from graphs import complete, csr_from_edges, two_cliques

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

UNCAPPED = 2**31 - 1


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _w():
    import paper_2509_02590_amd as w
    return w


def _t(a, dtype=None):
    a = np.ascontiguousarray(a if dtype is None else a.astype(dtype))
    return torch.from_numpy(a).to(_dev())


def _rec_key(r):
    return sorted(tuple(int(x) for x in (q["minv"], q["n"], q["k"], q["lam"], q["ssize"], q["shash"])) for q in r)


def _dense(rng, n, p):
    m = rng.random((n, n)) < p
    a, b = np.nonzero(np.triu(m, 1))
    return list(zip(a.tolist(), b.tolist()))


def _shift(edges, base):
    return [(a + base, b + base) for a, b in edges]


# ------------------------------------------------------------------ uncapped cuts
def _split_sets():
    """Disjoint dense sets, each with its cut value pinned by a closed form where one
    exists (K_n: n - 1; two K_a joined by b < a - 1 disjoint edges: b)."""
    rng = np.random.default_rng(71)
    sets = []
    sets.append((100, complete(100)))                  # lambda = 99, one Phase-0 singleton
    sets.append(two_cliques(80, 70))                   # lambda = 70 < delta = 79
    sets.append(two_cliques(140, 130))                 # lambda = 130, bound 139 > 126
    sets.append((150, _dense(rng, 150, 0.7)))          # delta around 90
    sets.append((220, _dense(rng, 220, 0.8)))          # delta above 150
    h = 90                                             # two dense halves, 65 random bridges
    e = _dense(rng, h, 0.95) + _shift(_dense(rng, h, 0.95), h)
    e += list({(int(rng.integers(0, h)), int(rng.integers(h, 2 * h))) for _ in range(65)})
    sets.append((2 * h, e))
    return sets


def _pack(sets):
    edges, base, so = [], 0, [0]
    for n, e in sets:
        edges += _shift(e, base)
        base += n
        so.append(base)
    off, adj = csr_from_edges(base, edges)
    return off, adj, np.arange(base, dtype=np.int32), np.array(so, np.int64)


def test_uncapped_mincut_split_dense_sets():
    w = _w()
    sets = _split_sets()
    off, adj, verts, so = _pack(sets)
    pinned = {0: 99, 1: 70, 2: 130}
    for i, (n, e) in enumerate(sets):
        vs = verts[so[i]:so[i + 1]]
        lam, side = w.mincut_split(_t(off, np.int32), _t(adj), _t(vs), UNCAPPED)
        wl, ws = oracle.mincut_split(off, adj, vs, UNCAPPED)
        assert lam == wl, (i, n, lam, wl)
        assert np.array_equal(side.cpu().numpy().astype(bool), ws), i
        if i in pinned:
            assert lam == pinned[i]


def test_capped_batch_above_62_levels():
    """One batch over the same sets with caps below, at and above their cut values."""
    w = _w()
    sets = _split_sets()
    off, adj, verts, so = _pack(sets)
    for caps in ([UNCAPPED] * len(sets), [63, 64, 127, 80, 130, 66], [99, 71, 131, 200, 300, 62]):
        caps = np.array(caps, np.int32)
        lam, side = w.mincut_split_batch(_t(off, np.int32), _t(adj), _t(verts), _t(so), _t(caps))
        lam, side = lam.cpu().numpy(), side.cpu().numpy().astype(bool)
        for i in range(len(sets)):
            wl, ws = oracle.mincut_split(off, adj, verts[so[i]:so[i + 1]], int(caps[i]))
            assert lam[i] == wl, (i, caps[i])
            assert np.array_equal(side[so[i]:so[i + 1]], ws), (i, caps[i])


# ------------------------------------------------------------------ criteria with large bounds
def _dense_clusters(rng):
    """Three clusters of a few thousand vertices whose k-cores have minimum degree above
    62: one dense random cluster (accepted under sqrt), one of two dense halves joined by
    fewer edges than the cut bound (split), one sparse enough to be pruned first."""
    parts, base = [], 0
    def add(n, edges):
        nonlocal base
        parts.append((base, n, _shift(edges, base)))
        base += n
    n0 = 5000
    src = rng.integers(0, n0, 420000)
    dst = rng.integers(0, n0, 420000)
    add(n0, [(int(a), int(b)) for a, b in zip(src, dst) if a != b])
    h = 2000
    e = []
    for off in (0, h):
        s = rng.integers(0, h, 150000)
        d = rng.integers(0, h, 150000)
        e += [(int(a) + off, int(b) + off) for a, b in zip(s, d) if a != b]
    e += [(int(rng.integers(0, h)), int(rng.integers(h, 2 * h))) for _ in range(40)]
    add(2 * h, e)
    n2 = 2500
    s = rng.integers(0, n2, 60000)
    d = rng.integers(0, n2, 60000)
    add(n2, [(int(a), int(b)) for a, b in zip(s, d) if a != b])
    memb = np.concatenate([np.full(n, i, np.int32) for i, (_, n, _) in enumerate(parts)])
    off, adj = csr_from_edges(base, [e for _, _, es in parts for e in es])
    return off, adj, memb


@pytest.mark.parametrize("criterion,lin", [("sqrt", (1, 1)), ("linear", (1, 50))])
@pytest.mark.parametrize("exec_mode", ["plain", "batched"])
def test_large_bound_criteria(criterion, lin, exec_mode):
    w = _w()
    rng = np.random.default_rng(5)
    off, adj, memb = _dense_clusters(rng)
    assert oracle.threshold(5000, criterion, *lin) > 62
    for mode in ("kcore", "paper"):
        if mode == "paper":
            # (without pruning, the sparse cluster would be cut one vertex at a time)
            memb = np.where(memb == 2, -1, memb).astype(np.int32)
        want, wrec = oracle.wcc(off, adj, memb, criterion=criterion, lin_num=lin[0], lin_den=lin[1], mode=mode)
        got, st, grec = w.wcc_run(_t(off, np.int32), _t(adj), _t(memb), criterion=criterion, lin_num=lin[0],
                                  lin_den=lin[1], mode=mode, exec_mode=exec_mode, graph=False,
                                  records_cap=4 * len(memb))
        got = got.cpu().numpy()
        assert np.array_equal(got, want), (mode, int((got != want).sum()))
        assert _rec_key(grec) == _rec_key(wrec), mode
        assert max(int(r["k"]) for r in wrec) > 62


# ------------------------------------------------------------------ malformed input
def _expect_egraph(off, adj, memb, offsets32=True):
    w = _w()
    o = _t(off, np.int32 if offsets32 else np.int64)
    with pytest.raises(w.WccError) as ei:
        w.wcc_run(o, _t(adj, np.int32), _t(memb, np.int32), validate=True)
    assert ei.value.code == -2


@pytest.mark.parametrize("offsets32", [True, False])
def test_validate_rejects_malformed_csr(offsets32):
    w = _w()
    n = 40
    rng = np.random.default_rng(9)
    edges = sorted({(min(a, b), max(a, b)) for a, b in rng.integers(0, n, (300, 2)) if a != b})
    off, adj = csr_from_edges(n, edges)
    memb = (np.arange(n) % 3).astype(np.int32)
    # a valid graph passes and matches the run without validation
    o = _t(off, np.int32 if offsets32 else np.int64)
    a, _, _ = w.wcc_run(o, _t(adj), _t(memb), validate=True, s_pre=2, s_post=2)
    b, _, _ = w.wcc_run(o, _t(adj), _t(memb), s_pre=2, s_post=2)
    assert torch.equal(a, b)
    u, v = edges[7]
    # duplicate: the edge {u, v} stored twice in both rows (symmetric, so only the
    # duplicate check can see it)
    rows = [list(adj[off[i]:off[i + 1]]) for i in range(n)]
    rows[u].append(v)
    rows[v].append(u)
    doff = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    dadj = np.array([x for r in rows for x in r], np.int32)
    _expect_egraph(doff, dadj, memb, offsets32)
    # the same duplicate inside a hub row far longer than a tile
    hub = 2500
    e2 = [(0, j) for j in range(1, hub)]
    hoff, hadj = csr_from_edges(hub, e2)
    rows = [list(hadj[hoff[i]:hoff[i + 1]]) for i in range(hub)]
    rows[0].append(1234)
    rows[1234].append(0)
    hoff = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    hadj = np.array([x for r in rows for x in r], np.int32)
    _expect_egraph(hoff, hadj, np.zeros(hub, np.int32), offsets32)
    # out-of-range ids, on both ends of the range
    for badv in (n, -1, 2**31 - 1):
        bad = adj.copy()
        bad[3] = badv
        _expect_egraph(off, bad, memb, offsets32)
    # self-loop
    bad = adj.copy()
    bad[int(off[5])] = 5
    _expect_egraph(off, bad, memb, offsets32)
    # asymmetric entry
    bad = adj.copy()
    row = int(np.searchsorted(off, 10, side="right") - 1)
    bad[10] = next(x for x in range(n) if x != row and x not in set(adj[off[row]:off[row + 1]]))
    _expect_egraph(off, bad, memb, offsets32)
    # offsets that decrease, or that do not end at the entry count
    bad_off = off.copy()
    bad_off[4], bad_off[5] = bad_off[5], bad_off[4]
    if bad_off[4] != bad_off[5]:
        _expect_egraph(bad_off, adj, memb, offsets32)
