"""The served form (request loop with concurrent slots admitted by HBM footprint) against
the same jobs run alone: every standalone result equals the oracle, every result is
bit-identical alone and in the mix, jobs overlap on the device, and the footprint budget
is respected."""
import numpy as np
import pytest

import gen
import oracle

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


def _jobs():
    """Mixed sizes, criteria, modes and execution forms."""
    specs = [
        (20000, 30.0, 2.5, 1500, 21, dict()),
        (60000, 30.0, 2.5, 2000, 22, dict(mode="paper")),
        (8000, 20.0, 2.8, 500, 23, dict(exec_mode="batched")),
        (40000, 50.0, 2.2, 3000, 24, dict(criterion="log2")),
        (15000, 40.0, 2.5, 1000, 25, dict(exec_mode="batched", mode="paper")),
        (30000, 25.0, 2.6, 1200, 26, dict(criterion="sqrt")),
        (5000, 30.0, 2.5, 400, 27, dict()),
        (50000, 35.0, 2.4, 2500, 28, dict(exec_mode="batched")),
    ]
    jobs = []
    for n, deg, alpha, smax, seed, kw in specs:
        g = gen.chung_lu(n, deg, alpha, 11, smax, 2.0, 0.2, 0.15, 0.05, seed=seed, intra_mult=1.8)
        jobs.append((g, kw))
    return jobs


def _upload(g):
    return _t(g.offsets, np.int32), _t(g.indices, np.int32), _t(g.membership, np.int32)


def test_served_results_equal_alone_and_overlap():
    w = _w()
    jobs = _jobs()
    dev = [_upload(g) for g, _ in jobs]
    alone = []
    for (g, kw), (o, a, m) in zip(jobs, dev):
        out, _, _ = w.wcc_run(o, a, m, **kw)
        alone.append(out.cpu().numpy())
    # the oracle agrees with every standalone run (all criteria, modes and forms)
    for i in range(len(jobs)):
        g, kw = jobs[i]
        want, _ = oracle.wcc(g.offsets, g.indices, g.membership, mode=kw.get("mode", "kcore"),
                             criterion=kw.get("criterion", "log10"))
        assert np.array_equal(alone[i], want), i
    outs = [torch.full_like(m, -7) for _, _, m in dev]
    with w.Server(slots=4) as srv:
        ids = {}
        for i, ((g, kw), (o, a, m)) in enumerate(zip(jobs, dev)):
            ids[srv.submit(o, a, m, outs[i], tag=i, **kw)] = i
        assert srv.wait(60000)
        res = srv.poll()
    assert len(res) == len(jobs)
    for r in res:
        assert r["status"] == 0, r
        i = r["tag"]
        assert ids[r["job_id"]] == i
        assert np.array_equal(outs[i].cpu().numpy(), alone[i]), i
        assert r["t_submit_ms"] <= r["t_start_ms"] <= r["t_end_ms"]
    # with 4 slots and 8 jobs submitted together, some jobs ran at the same time
    iv = sorted((r["t_start_ms"], r["t_end_ms"]) for r in res)
    overlaps = sum(1 for k in range(len(iv) - 1) if iv[k + 1][0] < iv[k][1])
    assert overlaps >= 1
    assert len({r["slot"] for r in res}) >= 2


def test_served_budget_limits_concurrency_and_rejects_oversized():
    w = _w()
    jobs = _jobs()[:4]
    dev = [_upload(g) for g, _ in jobs]
    outs = [torch.empty_like(m) for _, _, m in dev]
    alone = [w.wcc_run(o, a, m, **kw)[0].cpu().numpy() for (g, kw), (o, a, m) in zip(jobs, dev)]
    # learn the footprints, then allow a little more than the largest single job
    with w.Server(slots=4) as srv:
        for i, ((g, kw), (o, a, m)) in enumerate(zip(jobs, dev)):
            srv.submit(o, a, m, outs[i], tag=i, **kw)
        srv.wait(60000)
        fp = {r["tag"]: r["footprint_bytes"] for r in srv.poll()}
    budget = int(max(fp.values()) * 1.2)
    with w.Server(slots=4, pool_bytes=budget) as srv:
        for i, ((g, kw), (o, a, m)) in enumerate(zip(jobs, dev)):
            srv.submit(o, a, m, outs[i], tag=i, **kw)
        assert srv.wait(60000)
        res = srv.poll()
    for r in res:
        assert r["status"] == 0
        assert np.array_equal(outs[r["tag"]].cpu().numpy(), alone[r["tag"]])
    # at every start, the footprints of the jobs running then fit the budget
    for r in res:
        running = [q for q in res if q["t_start_ms"] <= r["t_start_ms"] < q["t_end_ms"]]
        assert sum(q["footprint_bytes"] for q in running) <= budget
    # a job larger than the whole budget fails alone; the others still run
    small = min(fp.values())
    with w.Server(slots=2, pool_bytes=int(small * 1.1)) as srv:
        big = max(range(len(jobs)), key=lambda i: fp[i])
        little = min(range(len(jobs)), key=lambda i: fp[i])
        srv.submit(*dev[big], outs[big], tag=big, **jobs[big][1])
        srv.submit(*dev[little], outs[little], tag=little, **jobs[little][1])
        assert srv.wait(60000)
        res = {r["tag"]: r for r in srv.poll()}
    assert res[big]["status"] == -3
    assert res[little]["status"] == 0
    assert np.array_equal(outs[little].cpu().numpy(), alone[little])


def test_served_admits_jobs_arriving_while_others_run():
    """Jobs submitted after the first wave started are admitted as slots free up."""
    w = _w()
    jobs = _jobs()
    dev = [_upload(g) for g, _ in jobs]
    alone = [w.wcc_run(o, a, m, **kw)[0].cpu().numpy() for (g, kw), (o, a, m) in zip(jobs, dev)]
    outs = [torch.empty_like(m) for _, _, m in dev]
    with w.Server(slots=2) as srv:
        for i in range(4):
            srv.submit(*dev[i], outs[i], tag=i, **jobs[i][1])
        first = []
        while not first:
            first = srv.poll()
        for i in range(4, len(jobs)):
            srv.submit(*dev[i], outs[i], tag=i, **jobs[i][1])
        assert srv.wait(60000)
        res = first + srv.poll()
    assert sorted(r["tag"] for r in res) == list(range(len(jobs)))
    for r in res:
        assert r["status"] == 0
        assert np.array_equal(outs[r["tag"]].cpu().numpy(), alone[r["tag"]])
    late = [r for r in res if r["tag"] >= 4]
    assert min(r["t_submit_ms"] for r in late) > min(r["t_start_ms"] for r in res)
