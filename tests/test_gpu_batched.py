"""The batched form (device-driven size-bin level launches, HIP-graph replay, launch
shapes) against the CPU oracle: the same bit-exact membership and split records as the
plain level-synchronous path, whatever the launch shape or replay."""

import numpy as np
import pytest

import gen
import oracle
from graphs import complete, csr_from_edges, cycle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


def _run(off, adj, memb, **kw):
    w = _w()
    out, st, rec = w.wcc_run(_t(off, np.int32), _t(adj, np.int32), _t(memb, np.int32),
                             records_cap=2 * len(memb) + 16, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy(), st, rec


def _compare(off, adj, memb, mode="kcore", s=10, **kw):
    want, wrec = oracle.wcc(off, adj, memb, s_pre=s, s_post=s, mode=mode)
    got, st, grec = _run(off, adj, memb, s_pre=s, s_post=s, mode=mode, exec_mode="batched", **kw)
    assert np.array_equal(got, want), "membership differs (%d of %d)" % ((got != want).sum(), len(want))
    assert _rec_key(grec) == _rec_key(wrec)
    return st


@pytest.mark.parametrize("mode", ["kcore", "paper"])
def test_batched_tiny(mode):
    g = gen.c0()
    st = _compare(g.offsets, g.indices, g.membership, mode=mode, graph=False)
    assert st.accepted > 0 and st.item_launches >= 1


@pytest.mark.parametrize("mode", ["kcore", "paper"])
def test_batched_random_clustered(mode):
    rng = np.random.default_rng(91 if mode == "kcore" else 92)
    for trial in range(8):
        n = int(rng.integers(50, 400))
        nclust = int(rng.integers(1, 8))
        memb = rng.integers(-1, nclust, n).astype(np.int32)
        edges = set()
        for a in range(n):
            for b in range(a + 1, n):
                same = memb[a] == memb[b] and memb[a] >= 0
                if rng.random() < (float(rng.choice([0.1, 0.3])) if same else 0.01):
                    edges.add((a, b))
        off, adj = csr_from_edges(n, sorted(edges))
        for s in (1, 10):
            _compare(off, adj, memb, mode=mode, s=s, graph=False)


def test_batched_special_cases():
    e = complete(11) + complete(11, 11) + [(10, 11)]
    off, adj = csr_from_edges(22, e)
    for mode in ("kcore", "paper"):
        _compare(off, adj, np.zeros(22, np.int32), mode=mode, graph=False)
    e = cycle(99) + [(98, 99)]
    off, adj = csr_from_edges(100, e)
    for mode in ("kcore", "paper"):
        _compare(off, adj, np.zeros(100, np.int32), mode=mode, graph=False)
    # nothing to do: no intra-cluster edge
    got, st, _ = _run(off, adj, np.arange(100, dtype=np.int32), exec_mode="batched", graph=False)
    assert np.all(got == -1) and st.items == 0


@pytest.mark.parametrize("mode", ["kcore", "paper"])
def test_batched_chunglu_medium(mode):
    g = gen.chung_lu(60000, 30.0, 2.5, 11, 2000, 2.0, 0.2, 0.15, 0.05, seed=77, intra_mult=1.8)
    _compare(g.offsets, g.indices, g.membership, mode=mode, graph=False)


def test_batched_launch_shapes():
    """Other size-bin boundaries and workgroup counts give the same bit-exact result."""
    w = _w()
    g = gen.chung_lu(60000, 30.0, 2.5, 11, 2000, 2.0, 0.2, 0.15, 0.05, seed=77, intra_mult=1.8)
    try:
        for cfg in (dict(small_lds_kb=8, big_max_pct=25), dict(small_lds_kb=16, wg_per_cu=2, big_max_pct=10),
                    dict(small_lds_kb=64, wg_per_cu=1, big_lds_kb=128, big_max_pct=100)):
            w.set_exec_config(**cfg)
            assert w.get_exec_config()["small_lds_kb"] == cfg["small_lds_kb"]
            _compare(g.offsets, g.indices, g.membership, graph=False)
    finally:
        w.set_exec_config()
    with pytest.raises(w.WccError):
        w.set_exec_config(small_lds_kb=100)


def test_batched_graph_replay():
    """Recorded once, replayed several times with eager work in between; every replay
    is checked against the oracle (the output buffer is scribbled over before each)."""
    w = _w()
    g = gen.chung_lu(30000, 30.0, 2.5, 11, 1500, 2.0, 0.2, 0.15, 0.05, seed=5, intra_mult=1.8)
    want, wrec = oracle.wcc(g.offsets, g.indices, g.membership)
    o, a, m = _t(g.offsets, np.int32), _t(g.indices, np.int32), _t(g.membership, np.int32)
    out = torch.empty_like(m)
    replays = 0
    for it in range(6):
        out.fill_(-7)
        x = torch.randn(512, 512, device=out.device)
        y = (x @ x).sum().item()  # unrelated eager work and a synchronisation
        assert np.isfinite(y)
        got, st, rec = w.wcc_run(o, a, m, out=out, exec_mode="batched")
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), want), it
        replays += st.graph_replays
    assert replays >= 3


def test_batched_graph_guard_on_changed_sizes():
    """In-place changes of the inputs between replays: a change of the planned sizes is
    detected on the device and the call runs eagerly; other changes replay correctly."""
    w = _w()
    g = gen.chung_lu(30000, 30.0, 2.5, 11, 1500, 2.0, 0.2, 0.15, 0.05, seed=6, intra_mult=1.8)
    o, a = _t(g.offsets, np.int32), _t(g.indices, np.int32)
    m = _t(g.membership, np.int32)
    out = torch.empty_like(m)
    for _ in range(3):
        w.wcc_run(o, a, m, out=out, exec_mode="batched")
    # 1) relabel cluster ids (same sizes): replayed, still exact
    memb2 = np.where(g.membership >= 0, g.membership * 3 + 1, -1).astype(np.int32)
    m.copy_(torch.from_numpy(memb2))
    got, st, _ = w.wcc_run(o, a, m, out=out, exec_mode="batched")
    assert np.array_equal(got.cpu().numpy(), oracle.wcc(g.offsets, g.indices, memb2)[0])
    assert st.graph_replays == 1
    # 2) merge two clusters (fewer initial items): detected, eager, exact
    memb3 = memb2.copy()
    ids = np.unique(memb3[memb3 >= 0])
    memb3[memb3 == ids[1]] = ids[0]
    m.copy_(torch.from_numpy(memb3))
    got, st, _ = w.wcc_run(o, a, m, out=out, exec_mode="batched")
    assert np.array_equal(got.cpu().numpy(), oracle.wcc(g.offsets, g.indices, memb3)[0])
    assert st.graph_replays == 0


def test_batched_c1_full_matches_plain_and_oracle():
    """The 1M-vertex / 20M-edge workload: batched (recorded and replayed) == plain == oracle."""
    w = _w()
    g = gen.c1()
    want, wrec = oracle.wcc(g.offsets, g.indices, g.membership)
    o, a, m = _t(g.offsets, np.int32), _t(g.indices, np.int32), _t(g.membership, np.int32)
    out = torch.empty_like(m)
    got_plain, _, prec = w.wcc_run(o, a, m, records_cap=len(want) + 16)
    assert np.array_equal(got_plain.cpu().numpy(), want)
    assert _rec_key(prec) == _rec_key(wrec)
    for it in range(4):
        out.fill_(-7)
        got, st, _ = w.wcc_run(o, a, m, out=out, exec_mode="batched")
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), want), it
    assert st.graph_replays == 1
    # a small size-bin boundary: the large list can hold thousands of items and is sorted
    # largest-first on the device at every level
    try:
        w.set_exec_config(small_lds_kb=4)
        got, st, _ = w.wcc_run(o, a, m, exec_mode="batched", graph=False)
        assert np.array_equal(got.cpu().numpy(), want)
    finally:
        w.set_exec_config()


def test_autotune_picks_a_shape_and_caches_it(tmp_path, monkeypatch):
    """The autotuner times every candidate shape, installs the fastest (output stays
    bit-exact), and a second call with a cache file reads the shape back untimed."""
    w = _w()
    g = gen.chung_lu(30000, 30.0, 2.5, 11, 1500, 2.0, 0.2, 0.15, 0.05, seed=8, intra_mult=1.8)
    o, a, m = _t(g.offsets, np.int32), _t(g.indices, np.int32), _t(g.membership, np.int32)
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("WCC_TUNE_CACHE", str(cache))
    try:
        best, ms, tried = w.autotune(o, a, m, reps=1)
        assert tried > 20 and ms > 0
        assert w.get_exec_config() == best
        _compare(g.offsets, g.indices, g.membership, graph=False)
        w.set_exec_config()
        best2, _, tried2 = w.autotune(o, a, m, reps=1)
        assert tried2 == 0 and best2 == best
        with pytest.raises(w.WccError):
            w.autotune(o, a, m, reps=0)
    finally:
        w.set_exec_config()
