"""Writes tests/golden/c2_paper_digest.json: the oracle's PAPER-mode WCC (Alg. 1-3 as
printed, log10, s_pre = s_post = 10) on the whole 10M-vertex / 200M-edge workload,
reduced to SHA-256 digests of its output membership and of its sorted split records.

The oracle replays every single-vertex split of the large clusters one cut at a time, so
the whole run takes it tens of minutes; the GPU test compares its own run with these
digests instead of running the oracle.  Calls only the oracle and the input generator.

  python3 tests/golden/make_c2_paper_digest.py [threads]
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import gen  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_paper_digest.json")


def membership_digest(m):
    return hashlib.sha256(np.ascontiguousarray(m, "<i4").tobytes()).hexdigest()


def records_digest(r):
    """Records sorted by (smallest vertex, n, k, lambda, |S|, hash of S), as little-endian
    int64 rows of those six fields."""
    cols = [r["minv"].astype(np.int64), r["n"].astype(np.int64), r["k"].astype(np.int64),
            r["lam"].astype(np.int64), r["ssize"].astype(np.int64), r["shash"].astype(np.uint64).view(np.int64)]
    order = np.lexsort(cols[::-1])
    rows = np.stack([c[order] for c in cols], axis=1)
    return hashlib.sha256(np.ascontiguousarray(rows, "<i8").tobytes()).hexdigest()


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    g = gen.c2()
    t0 = time.time()
    out, rec = oracle.wcc(g, mode="paper", criterion="log10", s_pre=10, s_post=10, nthreads=threads)
    dt = time.time() - t0
    doc = {
        "workload": g.meta["workload"], "vertices": int(g.n), "edges": int(g.m),
        "mode": "paper", "criterion": "log10", "s_pre": 10, "s_post": 10,
        "membership_sha256": membership_digest(out),
        "records_sha256": records_digest(rec),
        "records": int(len(rec)), "saved_sets": int(len(np.unique(out[out >= 0]))),
        "labelled_vertices": int((out >= 0).sum()),
        "oracle_seconds": round(dt, 1), "oracle_threads": threads,
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")
    print(json.dumps(doc))


if __name__ == "__main__":
    main()
