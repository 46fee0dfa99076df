"""CPU oracle of the WCC hot path -- TEST INFRASTRUCTURE ONLY.

ctypes binding of ``wcc_oracle.c``.  Only the tests, ``__graft_entry__.smoke()`` and
``bench.py``'s cpu_baseline leg may import this package; the GPU library never does.
It shares no code with ``paper_2509_02590_amd``.

What it computes (Dindoost et al., arXiv 2509.02590): CCR (Alg. 1), WCC (Alg. 2) and the
well-connectedness check isWCC (Alg. 3) with an exact global minimum cut (GetMinCut /
MinCutPartition, Sec. 2.1) and the criterion f(n) of Sec. 2; the Connectivity Modifier
(CM, Alg. 4, and its check CMC, Alg. 5) with a built-in community detection step.  The canonical choice among
equal minimum cuts, the integer form of the threshold and the optional KCORE pruning
mode are documented in ``wcc_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wcc_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None

CRIT = {"log10": 0, "log2": 1, "sqrt": 2, "linear": 3}
MODE = {"paper": 0, "kcore": 1}
CDA = {"components": 0, "labelprop": 1}

RECORD_DTYPE = np.dtype([("minv", np.int32), ("n", np.int32), ("k", np.int32),
                         ("lam", np.int32), ("ssize", np.int32), ("pad", np.int32),
                         ("shash", np.uint64)])


def build(force: bool = True) -> str:
    """Compile the oracle into oracle/_build/liboracle.so (plain gcc, host only)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [("criterion", ctypes.c_int32), ("lin_num", ctypes.c_int32),
                ("lin_den", ctypes.c_int32), ("s_pre", ctypes.c_int32),
                ("s_post", ctypes.c_int32), ("prune_mode", ctypes.c_int32)]


def params(criterion="log10", s_pre=10, s_post=10, mode="kcore", lin_num=1, lin_den=1) -> Params:
    return Params(CRIT[criterion] if isinstance(criterion, str) else criterion, lin_num, lin_den,
                  s_pre, s_post, MODE[mode] if isinstance(mode, str) else mode)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.orc_threshold.restype = i64
        L.orc_threshold.argtypes = [i32, i64, i64, i64]
        L.orc_components.restype = i32
        L.orc_components.argtypes = [i32, vp, vp, vp, vp]
        L.orc_kcore.restype = i32
        L.orc_kcore.argtypes = [i32, vp, vp, i32, vp]
        L.orc_mincut.restype = i32
        L.orc_mincut.argtypes = [i32, vp, vp, i32, vp]
        L.orc_wcc.restype = i32
        L.orc_wcc.argtypes = [i64, vp, vp, vp, ctypes.POINTER(Params), vp, vp, i64,
                              ctypes.POINTER(ctypes.c_int64), i32]
        L.orc_mincut_split.restype = i32
        L.orc_mincut_split.argtypes = [i64, vp, vp, vp, i32, i32, vp]
        L.orc_cluster_csr.restype = i32
        L.orc_cluster_csr.argtypes = [i64, vp, vp, vp] + [ctypes.POINTER(ctypes.c_int64)] * 3 + [vp] * 5
        L.orc_cm.restype = i32
        L.orc_cm.argtypes = [i64, vp, vp, vp, ctypes.POINTER(Params), i32, i32, vp, vp, i64,
                             ctypes.POINTER(ctypes.c_int64), i32]
        L.orc_cda.restype = i32
        L.orc_cda.argtypes = [i32, i32, i32, vp, vp, vp]
        L.orc_set_hash.restype = ctypes.c_uint64
        L.orc_set_hash.argtypes = [vp, i64]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data if a is not None else None


def _csr(off, adj):
    off = np.ascontiguousarray(off, np.int64)
    adj = np.ascontiguousarray(adj, np.int32)
    return off, adj


def threshold(n: int, criterion="log10", lin_num=1, lin_den=1) -> int:
    c = CRIT[criterion] if isinstance(criterion, str) else criterion
    return int(_load().orc_threshold(c, n, lin_num, lin_den))


def components(off, adj, alive=None) -> np.ndarray:
    off, adj = _csr(off, adj)
    n = off.shape[0] - 1
    comp = np.empty(n, np.int32)
    al = None if alive is None else np.ascontiguousarray(alive, np.uint8)
    rc = _load().orc_components(n, _p(off), _p(adj), _p(al), _p(comp))
    if rc < 0:
        raise RuntimeError("orc_components failed: %d" % rc)
    return comp


def kcore(off, adj, k: int) -> np.ndarray:
    off, adj = _csr(off, adj)
    n = off.shape[0] - 1
    alive = np.empty(max(n, 1), np.uint8)
    rc = _load().orc_kcore(n, _p(off), _p(adj), k, _p(alive))
    if rc < 0:
        raise RuntimeError("orc_kcore failed: %d" % rc)
    return alive[:n].astype(bool)


def mincut(off, adj, cap: int = 2**31 - 1):
    """Canonical capped minimum cut of a connected graph on local ids -> (lam, side)."""
    off, adj = _csr(off, adj)
    n = off.shape[0] - 1
    side = np.zeros(max(n, 1), np.uint8)
    lam = _load().orc_mincut(n, _p(off), _p(adj), cap, _p(side))
    if lam < 0:
        raise RuntimeError("orc_mincut failed: %d" % lam)
    return int(lam), side[:n].astype(bool)


def wcc(g_or_off, adj=None, membership=None, *, criterion="log10", s_pre=10, s_post=10,
        mode="kcore", lin_num=1, lin_den=1, nthreads=None, log=True):
    """Full WCC -> (membership_out, records).  Accepts a gen.Graph or (off, adj, membership)."""
    if adj is None:
        g = g_or_off
        off, adj, membership = g.offsets, g.indices, g.membership
    else:
        off = g_or_off
    off, adj = _csr(off, adj)
    mem = np.ascontiguousarray(membership, np.int32)
    N = off.shape[0] - 1
    out = np.empty(max(N, 1), np.int32)
    P = params(criterion, s_pre, s_post, mode, lin_num, lin_den)
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    cap = max(2 * N, 16) if log else 0
    recs = np.zeros(cap, RECORD_DTYPE) if log else None
    nlog = ctypes.c_int64(0)
    rc = _load().orc_wcc(N, _p(off), _p(adj), _p(mem), ctypes.byref(P), _p(out), _p(recs), cap,
                         ctypes.byref(nlog), nthreads)
    if rc != 0:
        raise RuntimeError("orc_wcc failed: %d" % rc)
    if log and nlog.value > cap:
        raise RuntimeError("record buffer too small")
    return out[:N], (recs[:nlog.value] if log else None)


def cm(g_or_off, adj=None, membership=None, *, cda="components", cda_iters=5, criterion="log10",
       s_pre=10, s_post=10, lin_num=1, lin_den=1, nthreads=None, log=True):
    """Full CM (Alg. 4-5) with a built-in CDA -> (membership_out, records)."""
    if adj is None:
        g = g_or_off
        off, adj, membership = g.offsets, g.indices, g.membership
    else:
        off = g_or_off
    off, adj = _csr(off, adj)
    mem = np.ascontiguousarray(membership, np.int32)
    N = off.shape[0] - 1
    out = np.empty(max(N, 1), np.int32)
    P = params(criterion, s_pre, s_post, "paper", lin_num, lin_den)
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    cap = max(2 * N, 16) if log else 0
    recs = np.zeros(cap, RECORD_DTYPE) if log else None
    nlog = ctypes.c_int64(0)
    rc = _load().orc_cm(N, _p(off), _p(adj), _p(mem), ctypes.byref(P), CDA[cda] if isinstance(cda, str) else cda,
                        cda_iters, _p(out), _p(recs), cap, ctypes.byref(nlog), nthreads)
    if rc != 0:
        raise RuntimeError("orc_cm failed: %d" % rc)
    if log and nlog.value > cap:
        raise RuntimeError("record buffer too small")
    return out[:N], (recs[:nlog.value] if log else None)


def cda(off, adj, which="labelprop", iters=5):
    """The CDA alone on a graph of local ids -> (community label per vertex, count)."""
    off, adj = _csr(off, adj)
    n = off.shape[0] - 1
    comm = np.empty(max(n, 1), np.int32)
    nc = _load().orc_cda(CDA[which] if isinstance(which, str) else which, iters, n, _p(off), _p(adj), _p(comm))
    if nc < 0:
        raise RuntimeError("orc_cda failed: %d" % nc)
    return comm[:n], int(nc)


def mincut_split(off, adj, verts, cap: int):
    off, adj = _csr(off, adj)
    v = np.ascontiguousarray(verts, np.int32)
    side = np.zeros(max(v.shape[0], 1), np.uint8)
    lam = _load().orc_mincut_split(off.shape[0] - 1, _p(off), _p(adj), _p(v), v.shape[0], cap,
                                   _p(side))
    if lam < 0:
        raise RuntimeError("orc_mincut_split failed: %d" % lam)
    return int(lam), side[:v.shape[0]].astype(bool)


def cluster_csr(off, adj, membership):
    """Cluster-major induced subgraphs -> dict(cl_ids, cl_start, vert, row_off, adj)."""
    off, adj = _csr(off, adj)
    mem = np.ascontiguousarray(membership, np.int32)
    N = off.shape[0] - 1
    L = _load()
    K, na, E = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    rc = L.orc_cluster_csr(N, _p(off), _p(adj), _p(mem), ctypes.byref(K), ctypes.byref(na),
                           ctypes.byref(E), None, None, None, None, None)
    if rc:
        raise RuntimeError("orc_cluster_csr failed")
    cl_ids = np.empty(max(K.value, 1), np.int32)
    cl_start = np.empty(K.value + 1, np.int64)
    vert = np.empty(max(na.value, 1), np.int32)
    row_off = np.empty(na.value + 1, np.int64)
    sub = np.empty(max(E.value, 1), np.int32)
    rc = L.orc_cluster_csr(N, _p(off), _p(adj), _p(mem), ctypes.byref(K), ctypes.byref(na),
                           ctypes.byref(E), _p(cl_ids), _p(cl_start), _p(vert), _p(row_off), _p(sub))
    if rc:
        raise RuntimeError("orc_cluster_csr failed")
    return dict(cl_ids=cl_ids[:K.value], cl_start=cl_start, vert=vert[:na.value], row_off=row_off,
                adj=sub[:E.value])


def set_hash(verts) -> int:
    v = np.ascontiguousarray(verts, np.int32)
    return int(_load().orc_set_hash(_p(v), v.shape[0]))
