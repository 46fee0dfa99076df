"""ctypes binding of the gfx950 WCC library (include/wcc.h).

Argument marshalling only: tensors are passed as device pointers with the caller's
current HIP stream; every step of the computation runs in the library's HIP kernels.
The library must have been built (paper_2509_02590_amd.build.build()); importing this
module without it raises ImportError -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libwcc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libwcc.so is not built (%s); run paper_2509_02590_amd.build.build()" % LIB_PATH)

lib = ctypes.CDLL(LIB_PATH)

WCC_OK = 0
ERRORS = {-1: "EINVAL", -2: "EGRAPH", -3: "ENOMEM", -4: "EHIP", -5: "ENOTCONNECTED",
          -6: "ECANCELLED", -7: "ETIMEOUT", -8: "ENODEV", -9: "EUNSUPPORTED"}
CRIT = {"log10": 0, "log2": 1, "sqrt": 2, "linear": 3}
MODE = {"paper": 0, "kcore": 1}
EXEC = {"plain": 0, "batched": 1}
FLAG_VALIDATE = 1
FLAG_NO_GRAPH = 2


class WccError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        msg = lib.wcc_strerror(code).decode()
        detail = lib.wcc_last_error_detail().decode() if code == -4 else ""
        super().__init__("%s: %s (%s) %s" % (what, msg, ERRORS.get(code, code), detail))


class Csr(ctypes.Structure):
    _fields_ = [("num_vertices", ctypes.c_int64), ("num_entries", ctypes.c_int64),
                ("row_offsets", ctypes.c_void_p), ("offset_bits", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("col_indices", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("criterion", ctypes.c_int32), ("lin_num", ctypes.c_int32),
                ("lin_den", ctypes.c_int32), ("s_pre", ctypes.c_int32),
                ("s_post", ctypes.c_int32), ("prune_mode", ctypes.c_int32),
                ("mincut_rule", ctypes.c_int32), ("exec_mode", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("clusters", ctypes.c_int64), ("intra_entries", ctypes.c_int64),
                ("items", ctypes.c_int64), ("mincuts", ctypes.c_int64),
                ("accepted", ctypes.c_int64), ("levels", ctypes.c_int64),
                ("scan_steps", ctypes.c_int64), ("scan_rounds", ctypes.c_int64),
                ("ms_front", ctypes.c_double), ("ms_items", ctypes.c_double),
                ("ms_item_kernel", ctypes.c_double), ("item_launches", ctypes.c_int64),
                ("ms_total", ctypes.c_double), ("item_alg_bytes", ctypes.c_int64),
                ("graph_replays", ctypes.c_int64), ("reserved", ctypes.c_int64 * 3)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ExecConfig(ctypes.Structure):
    _fields_ = [("small_lds_kb", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32),
                ("big_lds_kb", ctypes.c_int32), ("big_max_pct", ctypes.c_int32),
                ("chain_min_n", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


RECORD_DTYPE = np.dtype([("minv", np.int32), ("n", np.int32), ("k", np.int32),
                         ("lam", np.int32), ("ssize", np.int32), ("pad", np.int32),
                         ("shash", np.uint64)])

_vp, _i32, _i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
lib.wcc_strerror.restype = ctypes.c_char_p
lib.wcc_strerror.argtypes = [ctypes.c_int]
lib.wcc_default_params.restype = None
lib.wcc_default_params.argtypes = [ctypes.POINTER(Params)]
lib.wcc_run.restype = ctypes.c_int
lib.wcc_run.argtypes = [ctypes.POINTER(Csr), _vp, ctypes.POINTER(Params), _vp, ctypes.POINTER(Stats),
                        _vp, _i64, ctypes.POINTER(ctypes.c_int64), _vp]
lib.wcc_mincut_split.restype = ctypes.c_int
lib.wcc_mincut_split.argtypes = [ctypes.POINTER(Csr), _vp, _i32, _i32, ctypes.POINTER(ctypes.c_int32), _vp, _vp]
lib.wcc_mincut_split_batch.restype = ctypes.c_int
lib.wcc_mincut_split_batch.argtypes = [ctypes.POINTER(Csr), _vp, _vp, _i32, _vp, _vp, _vp, _vp]
lib.wcc_cluster_csr.restype = ctypes.c_int
lib.wcc_cluster_csr.argtypes = [ctypes.POINTER(Csr), _vp] + [ctypes.POINTER(ctypes.c_int64)] * 3 + [_vp] * 6
lib.wcc_threshold.restype = ctypes.c_int64
lib.wcc_threshold.argtypes = [_i32, _i64, _i32, _i32]
lib.wcc_release.restype = ctypes.c_int
class ServerCfg(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("reserved", ctypes.c_int32), ("pool_bytes", ctypes.c_int64)]


class Job(ctypes.Structure):
    _fields_ = [("g", Csr), ("membership_in", _vp), ("membership_out", _vp), ("params", Params),
                ("tag", ctypes.c_int64)]


class Result(ctypes.Structure):
    _fields_ = [("job_id", ctypes.c_int64), ("tag", ctypes.c_int64), ("status", ctypes.c_int32),
                ("slot", ctypes.c_int32), ("t_submit_ms", ctypes.c_double), ("t_start_ms", ctypes.c_double),
                ("t_end_ms", ctypes.c_double), ("footprint_bytes", ctypes.c_int64), ("stats", Stats)]


lib.wcc_server_create.restype = ctypes.c_int
lib.wcc_server_create.argtypes = [ctypes.POINTER(ServerCfg), ctypes.POINTER(_vp)]
lib.wcc_server_submit.restype = ctypes.c_int
lib.wcc_server_submit.argtypes = [_vp, ctypes.POINTER(Job), ctypes.POINTER(ctypes.c_int64)]
lib.wcc_server_poll.restype = ctypes.c_int
lib.wcc_server_poll.argtypes = [_vp, ctypes.POINTER(Result), _i32, ctypes.POINTER(ctypes.c_int32)]
lib.wcc_server_wait.restype = ctypes.c_int
lib.wcc_server_wait.argtypes = [_vp, _i64]
lib.wcc_server_destroy.restype = ctypes.c_int
lib.wcc_server_destroy.argtypes = [_vp]
lib.wcc_ccr_components.restype = ctypes.c_int
lib.wcc_ccr_components.argtypes = [ctypes.POINTER(Csr), _vp, _vp, _vp]
lib.wcc_autotune.restype = ctypes.c_int
lib.wcc_autotune.argtypes = [ctypes.POINTER(Csr), _vp, ctypes.POINTER(Params), _i32, ctypes.POINTER(ExecConfig),
                             ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32), _vp]
lib.wcc_get_exec_config.restype = ctypes.c_int
lib.wcc_get_exec_config.argtypes = [ctypes.POINTER(ExecConfig)]
lib.wcc_set_exec_config.restype = ctypes.c_int
lib.wcc_set_exec_config.argtypes = [ctypes.POINTER(ExecConfig)]
lib.wcc_last_error_detail.restype = ctypes.c_char_p

CDA = {"components": 0, "labelprop": 1, "callback": 2}
# int (*)(const wcc_csr *g, const int32_t *part_of, int32_t *comm_out, void *user, void *stream)
CDA_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.POINTER(Csr), _vp, _vp, _vp, _vp)


class CmParams(ctypes.Structure):
    _fields_ = [("cda", ctypes.c_int32), ("cda_iters", ctypes.c_int32), ("fn", CDA_FN), ("user", _vp)]


lib.wcc_run_noalloc.restype = ctypes.c_int
lib.wcc_run_noalloc.argtypes = lib.wcc_run.argtypes
lib.wcc_cm_run.restype = ctypes.c_int
lib.wcc_cm_run.argtypes = [ctypes.POINTER(Csr), _vp, ctypes.POINTER(Params), ctypes.POINTER(CmParams), _vp,
                           ctypes.POINTER(Stats), _vp, _i64, ctypes.POINTER(ctypes.c_int64), _vp]
lib.wcc_cda.restype = ctypes.c_int
lib.wcc_cda.argtypes = [ctypes.POINTER(Csr), _vp, ctypes.POINTER(CmParams), _vp, _vp]
lib.wcc_abi_version.restype = ctypes.c_int


def _check(rc, what):
    if rc != WCC_OK:
        raise WccError(rc, what)


def _stream(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def make_csr(offsets, indices) -> Csr:
    """wcc_csr view of two device tensors (offsets int32/int64 of N+1, indices int32)."""
    import torch
    assert offsets.is_cuda and indices.is_cuda, "CSR tensors must be on the GPU"
    assert offsets.dtype in (torch.int32, torch.int64) and indices.dtype == torch.int32
    assert offsets.is_contiguous() and indices.is_contiguous()
    n = offsets.numel() - 1
    return Csr(n, indices.numel(), offsets.data_ptr() if n >= 0 else None,
               32 if offsets.dtype == torch.int32 else 64, 0, indices.data_ptr() if indices.numel() else None)


def params(criterion="log10", s_pre=10, s_post=10, mode="kcore", exec_mode="plain", lin_num=1,
           lin_den=1, validate=False, graph=True) -> Params:
    p = Params()
    lib.wcc_default_params(ctypes.byref(p))
    p.criterion = CRIT[criterion] if isinstance(criterion, str) else criterion
    p.lin_num, p.lin_den = lin_num, lin_den
    p.s_pre, p.s_post = s_pre, s_post
    p.prune_mode = MODE[mode] if isinstance(mode, str) else mode
    p.exec_mode = EXEC[exec_mode] if isinstance(exec_mode, str) else exec_mode
    p.flags = (FLAG_VALIDATE if validate else 0) | (0 if graph else FLAG_NO_GRAPH)
    return p


def wcc_run(offsets, indices, membership, *, out=None, records_cap=0, noalloc=False, **kw):
    """WCC over a device CSR and membership -> (membership_out, Stats, records or None).
    noalloc=True calls wcc_run_noalloc (fixed workspace; small inputs only; pass `out`
    and a records buffer size of 0 to make the call itself allocate nothing)."""
    import torch
    g = make_csr(offsets, indices)
    assert membership.is_cuda and membership.dtype == torch.int32 and membership.numel() == g.num_vertices
    if out is None:
        out = torch.empty_like(membership)
    p = params(**kw)
    st = Stats()
    rec = None
    nrec = ctypes.c_int64(0)
    if records_cap:
        rec = torch.empty(records_cap * RECORD_DTYPE.itemsize, dtype=torch.uint8, device=membership.device)
    fn = lib.wcc_run_noalloc if noalloc else lib.wcc_run
    rc = fn(ctypes.byref(g), membership.data_ptr() if membership.numel() else None,
                     ctypes.byref(p), out.data_ptr() if out.numel() else None, ctypes.byref(st),
                     rec.data_ptr() if rec is not None else None, records_cap, ctypes.byref(nrec),
                     _stream(torch, membership.device))
    _check(rc, "wcc_run")
    records = None
    if rec is not None:
        k = min(nrec.value, records_cap)
        records = np.frombuffer(rec[:k * RECORD_DTYPE.itemsize].cpu().numpy().tobytes(), RECORD_DTYPE)
        if nrec.value > records_cap:
            raise WccError(-3, "records buffer too small (%d needed)" % nrec.value)
    return out, st, records


def mincut_split(offsets, indices, verts, cap):
    """(lambda, side) for the set `verts` (sorted unique device int32)."""
    import torch
    g = make_csr(offsets, indices)
    side = torch.zeros(max(verts.numel(), 1), dtype=torch.uint8, device=verts.device)
    lam = ctypes.c_int32(0)
    rc = lib.wcc_mincut_split(ctypes.byref(g), verts.data_ptr() if verts.numel() else None, verts.numel(),
                              cap, ctypes.byref(lam), side.data_ptr(), _stream(torch, verts.device))
    _check(rc, "wcc_mincut_split")
    return lam.value, side[:verts.numel()]


def mincut_split_batch(offsets, indices, verts, set_offsets, caps):
    """(lambdas, sides) for disjoint sets given in CSR-of-sets form on the device."""
    import torch
    g = make_csr(offsets, indices)
    ns = set_offsets.numel() - 1
    lam = torch.zeros(max(ns, 1), dtype=torch.int32, device=verts.device)
    sides = torch.zeros(max(verts.numel(), 1), dtype=torch.uint8, device=verts.device)
    rc = lib.wcc_mincut_split_batch(ctypes.byref(g), verts.data_ptr() if verts.numel() else None,
                                    set_offsets.data_ptr(), ns, caps.data_ptr() if ns else None,
                                    lam.data_ptr(), sides.data_ptr(), _stream(torch, verts.device))
    _check(rc, "wcc_mincut_split_batch")
    return lam[:ns], sides[:verts.numel()]


def cluster_csr(offsets, indices, membership):
    """Cluster-major induced subgraphs as device tensors (dict)."""
    import torch
    g = make_csr(offsets, indices)
    K, na, E = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    s = _stream(torch, membership.device)
    rc = lib.wcc_cluster_csr(ctypes.byref(g), membership.data_ptr(), ctypes.byref(K), ctypes.byref(na),
                             ctypes.byref(E), None, None, None, None, None, s)
    _check(rc, "wcc_cluster_csr")
    dev = membership.device
    cl_ids = torch.empty(max(K.value, 1), dtype=torch.int32, device=dev)
    cl_start = torch.empty(K.value + 1, dtype=torch.int64, device=dev)
    vert = torch.empty(max(na.value, 1), dtype=torch.int32, device=dev)
    row_off = torch.empty(na.value + 1, dtype=torch.int64, device=dev)
    adj = torch.empty(max(E.value, 1), dtype=torch.int32, device=dev)
    rc = lib.wcc_cluster_csr(ctypes.byref(g), membership.data_ptr(), ctypes.byref(K), ctypes.byref(na),
                             ctypes.byref(E), cl_ids.data_ptr(), cl_start.data_ptr(), vert.data_ptr(),
                             row_off.data_ptr(), adj.data_ptr(), s)
    _check(rc, "wcc_cluster_csr")
    return dict(cl_ids=cl_ids[:K.value], cl_start=cl_start, vert=vert[:na.value], row_off=row_off,
                adj=adj[:E.value])


def threshold(n, criterion="log10", lin_num=1, lin_den=1) -> int:
    c = CRIT[criterion] if isinstance(criterion, str) else criterion
    return int(lib.wcc_threshold(c, n, lin_num, lin_den))


def release():
    lib.wcc_release()


def get_exec_config() -> dict:
    """Launch shape of the item kernels on the current device."""
    c = ExecConfig()
    _check(lib.wcc_get_exec_config(ctypes.byref(c)), "wcc_get_exec_config")
    return c.as_dict()


def set_exec_config(cfg=None, **kw):
    """Sets the launch shape (dict or keyword fields); no argument restores the defaults."""
    if cfg is None and not kw:
        _check(lib.wcc_set_exec_config(None), "wcc_set_exec_config")
        return
    cur = get_exec_config()
    cur.update(cfg or {})
    cur.update(kw)
    c = ExecConfig(**cur)
    _check(lib.wcc_set_exec_config(ctypes.byref(c)), "wcc_set_exec_config")


def autotune(offsets, indices, membership, reps=2, **kw):
    """Times every candidate launch shape on this input (batched form), installs the
    fastest and returns (shape dict, best ms per run, shapes timed)."""
    import torch
    g = make_csr(offsets, indices)
    p = params(**kw)
    best = ExecConfig()
    ms = ctypes.c_double(0)
    tried = ctypes.c_int32(0)
    rc = lib.wcc_autotune(ctypes.byref(g), membership.data_ptr() if membership.numel() else None, ctypes.byref(p),
                          reps, ctypes.byref(best), ctypes.byref(ms), ctypes.byref(tried),
                          _stream(torch, membership.device))
    _check(rc, "wcc_autotune")
    return best.as_dict(), ms.value, tried.value


class Server:
    """The served form: a request loop with `slots` concurrent jobs admitted by HBM
    footprint.  Device tensors of a submitted job are kept referenced until its result
    has been polled."""

    def __init__(self, slots=4, pool_bytes=0):
        cfg = ServerCfg(slots, 0, pool_bytes)
        h = _vp()
        _check(lib.wcc_server_create(ctypes.byref(cfg), ctypes.byref(h)), "wcc_server_create")
        self._h = h
        self._keep = {}

    def submit(self, offsets, indices, membership, out, tag=0, **kw):
        g = make_csr(offsets, indices)
        j = Job(g, membership.data_ptr() if membership.numel() else None,
                out.data_ptr() if out.numel() else None, params(**kw), tag)
        jid = ctypes.c_int64(0)
        _check(lib.wcc_server_submit(self._h, ctypes.byref(j), ctypes.byref(jid)), "wcc_server_submit")
        self._keep[jid.value] = (offsets, indices, membership, out)
        return jid.value

    def poll(self, max_results=256):
        buf = (Result * max_results)()
        n = ctypes.c_int32(0)
        _check(lib.wcc_server_poll(self._h, buf, max_results, ctypes.byref(n)), "wcc_server_poll")
        res = []
        for r in buf[:n.value]:
            self._keep.pop(r.job_id, None)
            res.append({"job_id": r.job_id, "tag": r.tag, "status": r.status, "slot": r.slot,
                        "t_submit_ms": r.t_submit_ms, "t_start_ms": r.t_start_ms, "t_end_ms": r.t_end_ms,
                        "footprint_bytes": r.footprint_bytes, "stats": r.stats.as_dict()})
        return res

    def wait(self, timeout_ms=-1):
        rc = lib.wcc_server_wait(self._h, timeout_ms)
        if rc == -7:
            return False
        _check(rc, "wcc_server_wait")
        return True

    def close(self):
        if self._h:
            _check(lib.wcc_server_destroy(self._h), "wcc_server_destroy")
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _cm_params(cda, cda_iters, callback):
    c = CmParams()
    c.cda = CDA[cda] if isinstance(cda, str) else cda
    c.cda_iters = cda_iters
    fn = None
    if callback is not None:
        c.cda = CDA["callback"]
        # callback(num_vertices, part_of_ptr, comm_out_ptr, stream_ptr) -> 0 or a WCC error code
        def tramp(g, part_of, comm_out, user, stream):
            try:
                return int(callback(g.contents.num_vertices, part_of, comm_out, stream))
            except Exception:
                return -1
        fn = CDA_FN(tramp)
        c.fn = fn
    return c, fn


def cm_run(offsets, indices, membership, *, cda="labelprop", cda_iters=5, callback=None, out=None,
           records_cap=0, **kw):
    """The Connectivity Modifier (CM with its check CMC) -> (membership_out, Stats, records).
    callback(num_vertices, part_of_ptr, comm_out_ptr, stream_ptr) supplies a CDA of the
    caller's own (device pointers as ints); it must not call into the library."""
    import torch
    g = make_csr(offsets, indices)
    assert membership.is_cuda and membership.dtype == torch.int32 and membership.numel() == g.num_vertices
    if out is None:
        out = torch.empty_like(membership)
    p = params(**kw)
    c, keep = _cm_params(cda, cda_iters, callback)
    st = Stats()
    rec = None
    nrec = ctypes.c_int64(0)
    if records_cap:
        rec = torch.empty(records_cap * RECORD_DTYPE.itemsize, dtype=torch.uint8, device=membership.device)
    rc = lib.wcc_cm_run(ctypes.byref(g), membership.data_ptr() if membership.numel() else None, ctypes.byref(p),
                        ctypes.byref(c), out.data_ptr() if out.numel() else None, ctypes.byref(st),
                        rec.data_ptr() if rec is not None else None, records_cap, ctypes.byref(nrec),
                        _stream(torch, membership.device))
    del keep
    _check(rc, "wcc_cm_run")
    records = None
    if rec is not None:
        k = min(nrec.value, records_cap)
        records = np.frombuffer(rec[:k * RECORD_DTYPE.itemsize].cpu().numpy().tobytes(), RECORD_DTYPE)
        if nrec.value > records_cap:
            raise WccError(-3, "records buffer too small (%d needed)" % nrec.value)
    return out, st, records


def cda(offsets, indices, part_of, which="labelprop", iters=5, out=None):
    """A built-in CDA alone on the parts of part_of -> device int32 community labels."""
    import torch
    g = make_csr(offsets, indices)
    if out is None:
        out = torch.empty_like(part_of)
    c, _ = _cm_params(which, iters, None)
    rc = lib.wcc_cda(ctypes.byref(g), part_of.data_ptr() if part_of.numel() else None, ctypes.byref(c),
                     out.data_ptr() if out.numel() else None, _stream(torch, part_of.device))
    _check(rc, "wcc_cda")
    return out


def ccr_components(offsets, indices, membership, out=None):
    """Component of every vertex inside its cluster's induced subgraph (smallest global id;
    -1 for unassigned vertices) as a device int32 tensor."""
    import torch
    g = make_csr(offsets, indices)
    if out is None:
        out = torch.empty_like(membership)
    rc = lib.wcc_ccr_components(ctypes.byref(g), membership.data_ptr() if membership.numel() else None,
                                out.data_ptr() if out.numel() else None, _stream(torch, membership.device))
    _check(rc, "wcc_ccr_components")
    return out
