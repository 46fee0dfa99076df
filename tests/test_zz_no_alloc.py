"""wcc_run_noalloc (the allocation-free variant of wcc_run, workspace in a fixed device
array) through the C ABI: two calls in a row, the second on a smaller input, each equal
to wcc_run on the same input (membership bit for bit, the same split records); inputs
beyond its limits are rejected with WCC_EUNSUPPORTED."""
import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _rec_key(r):
    return sorted(tuple(int(x) for x in (q["minv"], q["n"], q["k"], q["lam"], q["ssize"], q["shash"])) for q in r)


def _inputs(g):
    dev = _dev()
    return (torch.from_numpy(g.offsets.astype(np.int32)).to(dev), torch.from_numpy(g.indices).to(dev),
            torch.from_numpy(g.membership).to(dev))


def test_noalloc_matches_wcc_run_twice():
    import paper_2509_02590_amd as w
    big = gen.chung_lu(30000, 30.0, 2.5, 11, 2000, 2.0, 0.2, 0.15, 0.05, seed=77, intra_mult=1.8)
    small = gen.c0()
    assert big.indices.shape[0] <= 1 << 20 and big.n <= 1 << 16
    for g in (big, small):
        o, a, m = _inputs(g)
        for mode in ("kcore", "paper"):
            want, _, wrec = w.wcc_run(o, a, m, mode=mode, records_cap=4 * g.n)
            out = torch.full_like(m, -7)
            got, st, grec = w.wcc_run(o, a, m, out=out, mode=mode, records_cap=4 * g.n, noalloc=True)
            torch.cuda.synchronize()
            assert torch.equal(got, want), (g.n, mode)
            assert _rec_key(grec) == _rec_key(wrec), (g.n, mode)
            assert st.accepted == int(want.max().item()) + 1


def test_noalloc_rejects_inputs_beyond_its_limits():
    import paper_2509_02590_amd as w
    g = gen.chung_lu(70000, 10.0, 2.5, 11, 2000, 2.0, 0.2, 0.15, 0.05, seed=78, intra_mult=1.8)
    o, a, m = _inputs(g)
    with pytest.raises(w.WccError) as ei:
        w.wcc_run(o, a, m, noalloc=True)
    assert ei.value.code == -9
