"""Benchmark of the WCC hot path on one MI355X.

A step is one whole wcc_run (front end, CCR, pruning, every minimum cut and split, and the
final relabel) over the 250M-vertex / 2B-edge Chung-Lu workload with a planted power-law
clustering (the largest single-GPU configuration, on which batched and plain execution
are compared), input already resident in HBM.  Prints ONE JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c4|c2|c1|c0|served]
                  [--exec batched|plain] [--no-compare] [--compare-steps C] [--mode kcore|paper]
                  [--no-cpu-baseline] [--autotune]

The timed form (default batched: device-driven level launches replayed from a HIP
graph) gives `value`; the other form is timed after it on the same input (C steps after
one warmup run) and reported in `other_exec` together with whether both produced the
same membership.  The launch shape is the library's default; --autotune times every
candidate shape on the input first (minutes on the 2B-edge workload).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "WCC input edges processed/s (batched vs plain GPU), HBM GB/s; p50/p99 job ms"
HBM_PEAK_GBS = 8000.0

# HBM bytes per k_items launch on the default workload and form, from rocprofv3 FETCH_SIZE
# and WRITE_SIZE passes scaled by a known-size copy (profiles/k_items_chunglu-250M-2B_traffic.md).
# They describe the kernel sources with this digest only: after any change of the item
# kernel the figure is stale and reported as null until the counters are taken again.
TRAFFIC = {"sources_sha256_16": "e8d78f4f8308d328", "workload": "chunglu-250M-2B", "exec": "batched",
           "mode": "kcore", "bytes_per_launch": 93242861703.0}
KERNEL_SOURCES = ["paper_2509_02590_amd/csrc/wcc_items.hip", "paper_2509_02590_amd/csrc/wcc_common.h"]


def kernel_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name):
    import gen
    if name == "c0":
        return gen.c0()
    if name == "c1":
        return gen.c1()
    if name == "c2":
        return gen.c2()
    if name == "c4":
        gen.set_verbose(True)  # (progress lines on stderr during the two-minute generation)
        return gen.c4()
    raise SystemExit("unknown workload %s" % name)


def served(args, wcc, torch):
    """Served form on a Poisson stream of whole WCC jobs (the 256-job recipe)."""
    import numpy as np
    import gen
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    jobs = []
    for j in range(args.jobs):
        g = gen.c3_job(j)
        off = torch.from_numpy(g.offsets.astype(np.int32)).to(dev)
        idx = torch.from_numpy(g.indices).to(dev)
        mem = torch.from_numpy(g.membership).to(dev)
        jobs.append(dict(off=off, idx=idx, mem=mem, out=torch.empty_like(mem), n=g.n, m=g.m))
        if (j + 1) % 32 == 0:
            log("generated %d jobs (%.0f s)" % (j + 1, time.perf_counter() - t0))
    torch.cuda.synchronize()
    tot_m = sum(j["m"] for j in jobs)
    log("%d jobs, %.3e edges in total, generated and resident in %.0f s" % (len(jobs), tot_m, time.perf_counter() - t0))
    kw = dict(s_pre=10, s_post=10, mode=args.mode)
    skw = dict(kw, exec_mode=args.served_exec)
    # one at a time on the plain path: service times and the reference outputs
    for j in jobs[:4]:
        wcc.wcc_run(j["off"], j["idx"], j["mem"], **kw)
    service = []
    for j in jobs:
        ts = time.perf_counter()
        out, _, _ = wcc.wcc_run(j["off"], j["idx"], j["mem"], **kw)
        torch.cuda.synchronize()
        service.append(1000.0 * (time.perf_counter() - ts))
        j["alone"] = out
    service = np.array(service)
    capacity = 1000.0 / service.mean()
    rate = args.rate if args.rate > 0 else 2.0 * capacity
    rng = np.random.Generator(np.random.Philox(key=3999))
    arrivals = np.cumsum(rng.exponential(1000.0 / rate, len(jobs)))
    arrivals -= arrivals[0]
    # the one-at-a-time plain path under the same arrivals (FIFO, measured service times)
    end = 0.0
    lat_plain = []
    for a, sv in zip(arrivals, service):
        end = max(end, a) + sv
        lat_plain.append(end - a)
    plain_span = end
    # served form
    res = []
    with wcc.Server(slots=args.slots) as srv:
        h0 = time.perf_counter()
        for i, (a, j) in enumerate(zip(arrivals, jobs)):
            while 1000.0 * (time.perf_counter() - h0) < a:
                res += srv.poll()
                time.sleep(0.0002)
            srv.submit(j["off"], j["idx"], j["mem"], j["out"], tag=i, **skw)
        srv.wait()
        res += srv.poll()
    bad = [r for r in res if r["status"] != 0]
    if bad:
        raise SystemExit("served jobs failed: %s" % bad[:3])
    lat = np.array([r["t_end_ms"] - r["t_submit_ms"] for r in res])
    span = max(r["t_end_ms"] for r in res) - min(r["t_submit_ms"] for r in res)
    equal = all(bool(torch.equal(jobs[r["tag"]]["out"], jobs[r["tag"]]["alone"])) for r in res)
    line = {
        "metric": METRIC, "value": tot_m / (span / 1000.0), "unit": "edges/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": span, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "served-%d-jobs" % len(jobs), "jobs": len(jobs), "edges": tot_m,
                   "slots": args.slots, "served_exec": args.served_exec,
                   "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES", "default"), "rate_jobs_per_s": rate, "plain_capacity_jobs_per_s": capacity,
                   "prune": args.mode, "criterion": "log10", "s_pre": 10, "s_post": 10},
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "equal_output_alone_and_mixed": equal,
        "plain_one_at_a_time": {"value": tot_m / (plain_span / 1000.0), "p50_ms": float(np.percentile(lat_plain, 50)),
                                "p99_ms": float(np.percentile(lat_plain, 99)),
                                "service_ms_mean": float(service.mean())},
    }
    print(json.dumps(line), flush=True)


def cm_sets(comp, torch):
    """Sets of the CM-style call from CCR labels: components larger than s_pre = 10, their
    vertices ascending, grouped by label; caps k(n) under log10."""
    n = comp.numel()
    lab = torch.where(comp >= 0, comp, torch.full_like(comp, n)).long()
    size = torch.bincount(lab, minlength=n + 1)[:n]
    keep = (comp >= 0) & (size[lab.clamp(max=n - 1)] > 10)
    vid = torch.nonzero(keep).flatten()
    order = torch.argsort(lab[vid], stable=True)
    verts = vid[order].to(torch.int32).contiguous()
    ksz = size[size > 10]
    set_off = torch.zeros(ksz.numel() + 1, dtype=torch.int64, device=comp.device)
    set_off[1:] = torch.cumsum(ksz, 0)
    caps = torch.ones_like(ksz, dtype=torch.int32)
    p = 10
    while True:
        big = ksz >= p
        if not bool(big.any()):
            break
        caps += big.to(torch.int32)
        p *= 10
    return verts, set_off, caps


def cm_split(g, off, idx, mem, wcc, torch, reps):
    """The CM-style call: CCR components (larger than s_pre = 10) of every cluster, then one
    mincut_split_batch over all of them with cap = k(n) (log10)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    comp = wcc.ccr_components(off, idx, mem)
    torch.cuda.synchronize()
    t_ccr = time.perf_counter() - t0
    verts, set_off, caps = cm_sets(comp, torch)
    best = 1e30
    for _ in range(max(1, reps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam, side = wcc.mincut_split_batch(off, idx, verts, set_off, caps)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    below = int((lam < caps).sum().item())
    return {"sets": int(caps.numel()), "vertices": int(verts.numel()), "ms_ccr": 1000.0 * t_ccr,
            "ms_split_batch": 1000.0 * best, "edges_per_s": g.m / best, "below_cap": below}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def sample_clusters(memb, seed=20, n_small=400, n_mid=6, n_top=3):
    """Whole input clusters: random small and mid-size ones plus the n_top largest."""
    import numpy as np
    sizes = np.bincount(memb[memb >= 0])
    rng = np.random.default_rng(seed)
    ids = np.nonzero(sizes > 0)[0]
    small = ids[sizes[ids] <= 3000]
    mid = ids[(sizes[ids] > 3000) & (sizes[ids] <= 50000)]
    top = ids[np.argsort(-sizes[ids], kind="stable")[:n_top]]
    return np.unique(np.concatenate([rng.choice(small, min(n_small, len(small)), replace=False),
                                     rng.choice(mid, min(n_mid, len(mid)), replace=False), top]))


def cpu_baseline(g, mode, threads):
    """The oracle, as it stands, on the same workload: one full run when the workload has
    at most 2.5e8 edges, else on a sample of whole input clusters that includes the
    largest ones (WCC treats clusters independently).  Edges counted: the input edges
    whose rows the oracle scans (entries of the sampled vertices' rows, halved)."""
    import numpy as np
    import oracle
    if g.m <= 250_000_000:
        t0 = time.perf_counter()
        oracle.wcc(g, s_pre=10, s_post=10, mode=mode, nthreads=threads, log=False)
        dt = time.perf_counter() - t0
        return {"value": g.m / dt, "unit": "edges/s", "cores": threads, "kind": "oracle", "cpu": cpu_model(),
                "sample": "one full run of the same %s workload (%d edges), %.2f s" % (g.meta["workload"], g.m, dt)}
    memb = g.membership
    pick = sample_clusters(memb)
    sel = np.isin(memb, pick)
    memb_s = np.where(sel, memb, -1).astype(np.int32)
    m_s = int(np.diff(g.offsets)[sel].sum()) // 2
    sizes = np.bincount(memb[memb >= 0])
    t0 = time.perf_counter()
    oracle.wcc(g.offsets, g.indices, memb_s, s_pre=10, s_post=10, mode=mode, nthreads=threads, log=False)
    dt = time.perf_counter() - t0
    return {"value": m_s / dt, "unit": "edges/s", "cores": threads, "kind": "oracle", "cpu": cpu_model(),
            "sample": "%d whole input clusters of the %s workload (%d vertices, %d edges in their rows, "
                      "largest cluster %d vertices), %.2f s" % (len(pick), g.meta["workload"], int(sel.sum()), m_s,
                                                                 int(sizes[pick].max()), dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c4")
    ap.add_argument("--compare-steps", type=int, default=5,
                    help="timed steps of the other execution form (after one warmup run)")
    ap.add_argument("--exec", dest="exec_mode", default="batched")
    ap.add_argument("--no-compare", dest="compare", action="store_false",
                    help="skip timing the other execution form")
    ap.add_argument("--mode", default="kcore")
    ap.add_argument("--jobs", type=int, default=256, help="served: jobs in the stream")
    ap.add_argument("--slots", type=int, default=8, help="served: concurrent jobs")
    ap.add_argument("--served-exec", default="plain", help="served: execution form of each job")
    ap.add_argument("--rate", type=float, default=0.0,
                    help="served: arrivals per second (default: twice the plain path's capacity)")
    ap.add_argument("--autotune", action="store_true",
                    help="time every candidate launch shape on this input first (else: the tune file's shape "
                         "for this device and input, or the default shape)")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false", help=argparse.SUPPRESS)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cm", action="store_true",
                    help="also time the CM-style mincut_split_batch over every CCR component")
    ap.add_argument("--traffic-bytes", type=float, default=None,
                    help="HBM bytes per item launch measured by rocprofv3 counters (overrides the "
                         "recorded figure)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run 5 device-to-device copies of BYTES (the known-size kernel that "
                         "scales rocprofv3 FETCH_SIZE / WRITE_SIZE readings) and exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy // 4
        src = torch.ones(n, dtype=torch.int32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copied %d bytes 5 times" % (4 * n))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(sharding across GPUs is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == "served":
        # concurrent jobs need hardware queues of their own (HIP's default is 4)
        os.environ["GPU_MAX_HW_QUEUES"] = "16"
        import torch
        import paper_2509_02590_amd as wcc
        served(args, wcc, torch)
        return

    import numpy as np
    import torch
    import paper_2509_02590_amd as wcc

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    g = workload(args.workload)
    log("workload %s: n=%d m=%d clusters=%d mixing=%.3f (generated in %.1f s)"
        % (g.meta["workload"], g.n, g.m, g.meta["clusters"], g.meta["mixing"], time.perf_counter() - t0))
    obits = np.int32 if g.indices.shape[0] < 2**31 else np.int64
    off = torch.from_numpy(g.offsets.astype(obits)).to(dev)
    idx = torch.from_numpy(g.indices).to(dev)
    mem = torch.from_numpy(g.membership).to(dev)
    out = torch.empty_like(mem)
    torch.cuda.synchronize()
    tuned = None
    if args.autotune:
        t0 = time.perf_counter()
        shape, tms, ntried = wcc.autotune(off, idx, mem, reps=2, s_pre=10, s_post=10, mode=args.mode)
        tuned = {"shape": shape, "best_ms": tms, "shapes_timed": ntried, "seconds": time.perf_counter() - t0}
        log("autotune: %s (%.2f ms, %d shapes, %.1f s)" % (shape, tms, ntried, tuned["seconds"]))

    def timed(exec_mode, steps, warmup):
        kw = dict(s_pre=10, s_post=10, mode=args.mode, exec_mode=exec_mode)
        for i in range(warmup):
            wcc.wcc_run(off, idx, mem, out=out, **kw)
            log("%s warmup %d done" % (exec_mode, i))
        torch.cuda.synchronize()
        stats = []
        t_start = time.perf_counter()
        for i in range(steps):
            _, st, _ = wcc.wcc_run(off, idx, mem, out=out, **kw)
            stats.append(st.as_dict())
            if g.m > 250_000_000:
                log("%s step %d: %.1f ms" % (exec_mode, i, st.ms_total))
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        log("%s: timed %d steps: %.2f ms/step, %.3e edges/s"
            % (exec_mode, steps, 1000.0 * elapsed / steps, g.m * steps / elapsed))
        return elapsed, stats, out.clone()

    elapsed, stats, res = timed(args.exec_mode, args.steps, args.warmup)
    ms_step = 1000.0 * elapsed / args.steps
    value = g.m / (elapsed / args.steps)
    other = None
    if args.compare:
        other_mode = "plain" if args.exec_mode == "batched" else "batched"
        cs = max(1, args.compare_steps)
        o_elapsed, o_stats, o_res = timed(other_mode, cs, 1)
        other = {"exec": other_mode, "value": g.m / (o_elapsed / cs), "steps": cs, "warmup": 1,
                 "ms_per_step": 1000.0 * o_elapsed / cs, "equal_output": bool(torch.equal(res, o_res))}

    # roofline of the dominant kernel (the per-item kernel), timed with HIP events that
    # the library records around every item launch on the stream it is launched on
    s0 = stats[-1]
    launches = max(s0["item_launches"], 1)
    avg_launch_s = s0["ms_item_kernel"] / 1000.0 / launches
    alg_bytes_per_launch = s0["item_alg_bytes"] / launches
    achieved = alg_bytes_per_launch / avg_launch_s / 1e9 if avg_launch_s > 0 else 0.0
    traffic = args.traffic_bytes
    if traffic is None and (TRAFFIC["sources_sha256_16"] == kernel_digest() and
                            TRAFFIC["workload"] == g.meta["workload"] and TRAFFIC["exec"] == args.exec_mode
                            and TRAFFIC["mode"] == args.mode):
        traffic = TRAFFIC["bytes_per_launch"]
    # whole-job floor: one pass over the input (index + neighbour-cluster gather per entry,
    # offsets + membership + output per vertex)
    obytes = 4 if obits == np.int32 else 8
    b_floor = g.indices.shape[0] * 8 + g.n * (obytes + 4 + 4)
    t_step = elapsed / args.steps
    b_alg_step = b_floor + s0["item_alg_bytes"]
    # "bound" names the roofline the fraction is taken against: the item kernel moves
    # integers only (no MFMA work, little ALU work), so HBM bandwidth is its only
    # roofline; what limits it is latency (one dependent chain of scan steps per item),
    # which is why the fraction is small ("limiter")
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": "k_items", "limiter": "latency (dependent maximum-adjacency scan steps)",
                "avg_launch_ms": avg_launch_s * 1e3,
                "alg_bytes_per_launch": alg_bytes_per_launch, "launches_per_step": s0["item_launches"],
                "step_fractions": {
                    "floor": b_floor / t_step / 1e9 / HBM_PEAK_GBS,
                    "alg": b_alg_step / t_step / 1e9 / HBM_PEAK_GBS,
                    "counters": (traffic * s0["item_launches"] / t_step / 1e9 / HBM_PEAK_GBS
                                 if traffic is not None else None),
                    "note": "whole step: one input pass (floor), that plus the item launches' "
                            "algorithmic bytes (alg), the item launches' counter-measured bytes "
                            "(counters), each over the step time and 8 TB/s"}}
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": g.meta["workload"], "vertices": g.n, "edges": g.m,
                   "clusters": g.meta["clusters"], "mixing": round(g.meta["mixing"], 4),
                   "exec": args.exec_mode, "prune": args.mode, "criterion": "log10",
                   "s_pre": 10, "s_post": 10},
        "roofline": roofline,
        "floor_gbs": b_floor / (elapsed / args.steps) / 1e9,
        "step_stats": {k: s0[k] for k in ("items", "mincuts", "accepted", "levels", "scan_steps",
                                           "scan_rounds", "ms_front", "ms_items", "ms_item_kernel",
                                           "graph_replays")},
    }
    if args.cm:
        line["cm_split_batch"] = cm_split(g, off, idx, mem, wcc, torch, reps=max(1, min(args.steps, 3)))
        log("cm split batch: %s" % line["cm_split_batch"])
    line["exec_config"] = wcc.get_exec_config()
    if tuned is not None:
        line["autotune"] = tuned
    if other is not None:
        line["other_exec"] = other
    if not args.no_cpu_baseline:
        try:
            threads = min(16, len(os.sched_getaffinity(0)))
        except AttributeError:
            threads = min(16, os.cpu_count() or 1)
        line["cpu_baseline"] = cpu_baseline(g, args.mode, threads)
        log("cpu baseline: %.3e edges/s on %d threads" % (line["cpu_baseline"]["value"], threads))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
