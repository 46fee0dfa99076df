"""The Connectivity Modifier (CM, Alg. 4, with its check CMC, Alg. 5) on the GPU through
the C ABI, against the oracle: final membership and every split record, with the
components CDA, the label-propagation CDA and a caller-supplied CDA; and the built-in
CDA step alone (GetCommunities) on parts of a graph."""
import numpy as np
import pytest

import gen
import oracle
from graphs import complete, csr_from_edges

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


def _compare(off, adj, memb, cda, iters=5, s=10, criterion="log10"):
    w = _w()
    want, wrec = oracle.cm(off, adj, memb, cda=cda, cda_iters=iters, s_pre=s, s_post=s, criterion=criterion)
    got, st, grec = w.cm_run(_t(off, np.int32), _t(adj, np.int32), _t(memb, np.int32), cda=cda, cda_iters=iters,
                             s_pre=s, s_post=s, criterion=criterion, records_cap=4 * len(memb) + 16)
    got = got.cpu().numpy()
    assert np.array_equal(got, want), "membership differs in %d vertices" % int((got != want).sum())
    assert _rec_key(grec) == _rec_key(wrec)
    return st


def _worked_example():
    e = complete(12) + complete(12, 12) + complete(12, 24) + [(9, 21), (10, 22), (11, 23), (23, 24)]
    return csr_from_edges(36, e)


def test_cm_worked_example():
    off, adj = _worked_example()
    memb = np.zeros(36, np.int32)
    _compare(off, adj, memb, "components")
    st = _compare(off, adj, memb, "labelprop", iters=3)
    assert st.accepted == 3


def _random_clustered(rng, n, nclust, p_in, p_out):
    memb = rng.integers(-1, nclust, n).astype(np.int32)
    edges = set()
    for a in range(n):
        for b in range(a + 1, n):
            same = memb[a] == memb[b] and memb[a] >= 0
            if rng.random() < (p_in if same else p_out):
                edges.add((a, b))
    off, adj = csr_from_edges(n, sorted(edges))
    return off, adj, memb


@pytest.mark.parametrize("cda,iters", [("components", 0), ("labelprop", 1), ("labelprop", 2), ("labelprop", 5)])
def test_cm_random_clustered(cda, iters):
    rng = np.random.default_rng(500 + iters)
    for trial in range(8):
        off, adj, memb = _random_clustered(rng, int(rng.integers(60, 300)), int(rng.integers(1, 5)),
                                           float(rng.choice([0.1, 0.25])), 0.01)
        for s in (3, 10):
            _compare(off, adj, memb, cda, iters, s=s)


@pytest.mark.parametrize("cda", ["components", "labelprop"])
def test_cm_tiny_and_chunglu(cda):
    g = gen.c0()
    _compare(g.offsets, g.indices, g.membership, cda)
    g = gen.chung_lu(20000, 24.0, 2.5, 11, 600, 2.0, 0.2, 0.15, 0.05, seed=91, intra_mult=1.8)
    st = _compare(g.offsets, g.indices, g.membership, cda)
    assert st.accepted > 10


def test_cm_callback_single_community_equals_wcc():
    """A caller CDA that keeps every part whole (its community is its part label): CM then
    checks each side of a cut as a single unit, exactly as WCC without pruning does."""
    w = _w()
    g = gen.c0()
    dev = _dev()
    calls = []

    def one_community(n, part_of, comm_out, stream):
        calls.append(n)
        # comm_out = part_of, on the device
        part = _ptr_tensor(part_of, n, dev)
        out = _ptr_tensor(comm_out, n, dev)
        out.copy_(part)
        torch.cuda.synchronize()
        return 0

    want, wrec = oracle.wcc(g, mode="paper")
    got, st, grec = w.cm_run(_t(g.offsets, np.int32), _t(g.indices), _t(g.membership), callback=one_community,
                             records_cap=4 * g.n)
    assert calls, "the callback was not called"
    assert np.array_equal(got.cpu().numpy(), want)
    assert _rec_key(grec) == _rec_key(wrec)


def _ptr_tensor(ptr, n, dev):
    """A device int32 tensor over caller memory (ptr: device address)."""
    class _A:
        __cuda_array_interface__ = {"shape": (n,), "typestr": "<i4", "data": (ptr, False), "version": 2}
    return torch.as_tensor(_A(), device=dev)


@pytest.mark.parametrize("iters", [0, 1, 2, 4])
def test_cda_labelprop_matches_oracle(iters):
    """The built-in label propagation on every cluster of a graph at once, against the
    oracle's CDA on each cluster's induced subgraph (labels compared as global ids)."""
    w = _w()
    g = gen.chung_lu(8000, 20.0, 2.5, 11, 400, 2.0, 0.2, 0.15, 0.05, seed=12, intra_mult=1.8)
    memb = g.membership.copy()
    memb[::31] = -1
    got = w.cda(_t(g.offsets, np.int32), _t(g.indices), _t(memb, np.int32), "labelprop", iters).cpu().numpy()
    sub = oracle.cluster_csr(g.offsets, g.indices, memb)
    want = np.full(g.n, -1, np.int64)
    cs, vert, ro, adj = sub["cl_start"], sub["vert"], sub["row_off"], sub["adj"]
    for c in range(len(cs) - 1):
        a, b = int(cs[c]), int(cs[c + 1])
        off = ro[a:b + 1] - ro[a]
        lab, _ = oracle.cda(off, adj[ro[a]:ro[b]], "labelprop", iters)
        want[vert[a:b]] = vert[a:b][lab]                 # local label -> global id
    assert np.array_equal(got, want)
    comp = w.cda(_t(g.offsets, np.int32), _t(g.indices), _t(memb, np.int32), "components").cpu().numpy()
    assert np.array_equal(comp, w.ccr_components(_t(g.offsets, np.int32), _t(g.indices),
                                                 _t(memb, np.int32)).cpu().numpy())
