"""Seeded synthetic WCC inputs (graph CSR + planted clustering).

Thin ctypes wrapper around ``wccgen.c``.  Holds none of the WCC method's arithmetic:
it only manufactures inputs that the oracle and the GPU path both consume.

Workload recipes (they stand in for the paper's real networks of Table 1 and its
Leiden-CPM input clusterings, Sec. 3, which are not available here):

* ``tiny``   -- 2,000 vertices, 20 planted clusters of 100 (ER p=0.1), four of them two
  50-vertex ER(p=0.2) halves joined by one bridge, two with a 10-vertex pendant path,
  plus 2,000 distinct uniform inter-cluster edges.
* ``c1``     -- 1M vertices, ~20M edges, Chung-Lu (Pareto exponent 2.5, mean degree 40),
  power-law cluster sizes 11..5,000 (exponent 2.0), mixing 0.2, 15% of clusters two
  halves joined by 1-3 bridges, 5% two disconnected blocks.
* ``c2``     -- 10M vertices, ~200M edges, exponent 2.3, sizes 11..100,000 (exponent 1.8),
  mixing 0.25, 20% bridged with halving nested up to 3 levels.
* ``c3_job`` -- one job of the served stream: 10k..2M vertices (log-uniform), mean degree
  20..60, exponent 2.2..2.8, clusters shaped as in ``c1``.
* ``c4``     -- 250M vertices, ~2B edges, exponent 2.2, max expected degree 1M, sizes
  11..1,000,000 (exponent 1.9), mixing 0.3, 10% bridged or disconnected.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wccgen.c")
_LIB = os.path.join(_HERE, "_build", "libwccgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the generator into gen/_build/libwccgen.so."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _ClParams(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("mean_deg", ctypes.c_double),
                ("alpha", ctypes.c_double), ("wmax", ctypes.c_double),
                ("smin", ctypes.c_int64), ("smax", ctypes.c_int64),
                ("beta", ctypes.c_double), ("mu", ctypes.c_double),
                ("f_bridged", ctypes.c_double), ("f_disc", ctypes.c_double),
                ("depth_max", ctypes.c_int32), ("nthreads", ctypes.c_int32),
                ("intra_mult", ctypes.c_double), ("inter_mult", ctypes.c_double)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        L.gen_tiny.restype = vp
        L.gen_tiny.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                               ctypes.c_int64, ctypes.c_double, ctypes.c_int64, ctypes.c_int64,
                               ctypes.c_int64]
        L.gen_chung_lu.restype = vp
        L.gen_chung_lu.argtypes = [ctypes.POINTER(_ClParams), ctypes.c_uint64]
        for f in ("gen_n", "gen_nnz", "gen_nclusters", "gen_inter_edges"):
            getattr(L, f).restype = ctypes.c_int64
            getattr(L, f).argtypes = [vp]
        L.gen_export.restype = None
        L.gen_export.argtypes = [vp, vp, vp, vp]
        L.gen_free.restype = None
        L.gen_free.argtypes = [vp]
        L.gen_set_verbose.restype = None
        L.gen_set_verbose.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def set_verbose(on: bool = True) -> None:
    """Progress lines on stderr from the generator's phases (each eighth of a phase)."""
    _load().gen_set_verbose(1 if on else 0)


@dataclass
class Graph:
    """Undirected simple graph in symmetric CSR form plus a disjoint clustering."""
    n: int
    offsets: np.ndarray      # int64, n+1
    indices: np.ndarray      # int32, 2m
    membership: np.ndarray   # int32, n (-1 = unassigned)
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.indices.shape[0] // 2)


def _take(h) -> Graph:
    L = _load()
    if not h:
        raise MemoryError("generator failed")
    try:
        n, nnz = L.gen_n(h), L.gen_nnz(h)
        off = np.empty(n + 1, np.int64)
        idx = np.empty(max(nnz, 0), np.int32)
        mem = np.empty(n, np.int32)
        L.gen_export(h, off.ctypes.data, idx.ctypes.data, mem.ctypes.data)
        meta = {"clusters": int(L.gen_nclusters(h)), "inter_edges": int(L.gen_inter_edges(h))}
    finally:
        L.gen_free(h)
    g = Graph(int(n), off, idx, mem, meta)
    g.meta["m"] = g.m
    g.meta["mixing"] = (g.meta["inter_edges"] / g.m) if g.m else 0.0
    return g


def tiny(seed: int = 1000, n_clusters: int = 20, csize: int = 100, p: float = 0.1,
         n_bridged: int = 4, p_half: float = 0.2, n_pendant: int = 2, path_len: int = 10,
         n_noise: int = 2000) -> Graph:
    return _take(_load().gen_tiny(seed, n_clusters, csize, p, n_bridged, p_half, n_pendant,
                                  path_len, n_noise))


def chung_lu(n: int, mean_deg: float, alpha: float, smin: int, smax: int, beta: float,
             mu: float, f_bridged: float, f_disc: float, depth_max: int = 1,
             wmax: float = 0.0, seed: int = 1, nthreads: int | None = None,
             intra_mult: float = 1.0, inter_mult: float = 1.0) -> Graph:
    if nthreads is None:
        nthreads = min(16, os.cpu_count() or 1)
    P = _ClParams(n, mean_deg, alpha, wmax, smin, smax, beta, mu, f_bridged, f_disc,
                  depth_max, nthreads, intra_mult, inter_mult)
    g = _take(_load().gen_chung_lu(ctypes.byref(P), seed))
    g.meta.update(dict(alpha=alpha, mean_deg=mean_deg, sizes=(smin, smax), beta=beta, mu=mu))
    return g


# ---------------------------------------------------------------- named workloads
def c0(seed: int = 1000) -> Graph:
    g = tiny(seed)
    g.meta["workload"] = "tiny-2k"
    return g


def c1(seed: int = 1001, n: int = 1_000_000) -> Graph:
    # intra_mult offsets the duplicate pairs that Chung-Lu sampling draws inside small
    # clusters with hub vertices, so that m ~ 2.0e7 and the mixing ~ 0.2 are reached.
    g = chung_lu(n, 40.0, 2.5, 11, 5000, 2.0, 0.2, 0.15, 0.05, 1, seed=seed, intra_mult=1.8)
    g.meta["workload"] = "chunglu-1M-20M"
    return g


def c2(seed: int = 1002, n: int = 10_000_000) -> Graph:
    # intra_mult offsets duplicate intra-cluster pairs so that m ~ 2.0e8 and the
    # mixing ~ 0.25 are reached (measured: m = 201,915,650, mixing 0.247)
    g = chung_lu(n, 40.0, 2.3, 11, 100_000, 1.8, 0.25, 0.20, 0.0, 3, seed=seed, intra_mult=1.4)
    g.meta["workload"] = "chunglu-10M-200M"
    return g


def c3_job(j: int, seed_base: int = 3000) -> Graph:
    """Job j of the served stream; its shape parameters are drawn from a job-keyed
    counter generator so the stream is reproducible."""
    r = np.random.Generator(np.random.Philox(key=seed_base + j))
    n = int(round(math.exp(r.uniform(math.log(1e4), math.log(2e6)))))
    mean_deg = float(r.uniform(20, 60))
    alpha = float(r.uniform(2.2, 2.8))
    g = chung_lu(n, mean_deg, alpha, 11, 5000, 2.0, 0.2, 0.15, 0.05, 1, seed=seed_base + j,
                 intra_mult=1.8)
    g.meta["workload"] = "served-job-%d" % j
    return g


def c4(seed: int = 1004, n: int = 250_000_000) -> Graph:
    # intra_mult offsets duplicate intra-cluster pairs (at a tenth of the size it gives
    # m ~ 2.0e8 and mixing ~ 0.29; the full size is reported by the run that uses it)
    g = chung_lu(n, 16.0, 2.2, 11, 1_000_000, 1.9, 0.3, 0.07, 0.03, 1, wmax=1e6, seed=seed, intra_mult=1.5)
    g.meta["workload"] = "chunglu-250M-2B"
    return g
