"""Python binding of the C ABI in include/qc.h (ctypes).

Argument marshalling only: every step of the computation runs in the HIP
library ``libqc_hip.so``. PyTorch supplies device memory (tensors) and the
stream (``torch.cuda.current_stream()``). The binding refuses to run when the
library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqc_hip.so")

QC_OK = 0
QC_E_INVAL = 1
QC_E_NOT_SYMMETRIC = 2
QC_E_OOM = 3
QC_E_DEVICE = 4
QC_E_OVERFLOW = 5
QC_E_STATE = 6
QC_E_BUSY = 7
QC_E_TIMEOUT = 8
QC_E_CANCELLED = 9
QC_E_TOO_LARGE = 10

# Device scratch of qc_cluster_noalloc (QC_NOALLOC_SCRATCH_BYTES in qc.h).
NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024

TIE_STRICT = 0
TIE_MERGE = 1

PREC_FP64ACC = 0
PREC_FP32C = 1
PREC_BF16 = 2

GRAPH_CANONICALIZE = 1
GRAPH_DIRECTED = 2

# Every symbol include/qc.h declares (checked by the tests).
EXPORTED = [
    "qc_status_str", "qc_device_count", "qc_graph_create", "qc_graph_create_weighted",
    "qc_graph_destroy",
    "qc_graph_info", "qc_graph_bfs_plan", "qc_distances", "qc_get_histograms", "qc_potential",
    "qc_ggd_labels", "qc_last_recheck_count", "qc_graph_sync", "qc_timing_enable",
    "qc_timing_read", "qc_potential_dense", "qc_debug_alloc_fault", "qc_get_potential64",
    "qc_cluster", "qc_cluster_noalloc", "qc_distances_real", "qc_cluster_real",
    "qc_batch_create", "qc_batch_node_offsets", "qc_batch_run", "qc_batch_recheck_count",
    "qc_batch_search_stats", "qc_batch_sweep_bf16", "qc_batch_stage_tiles", "qc_batch_destroy",
]

BATCH_HIPGRAPH = 1
BATCH_FP32C = 2
BATCH_AUTOTUNE = 4
BATCH_SERIAL = 8

EXPORTED += ["qc_request_footprint", "qc_server_create", "qc_server_submit", "qc_server_poll",
             "qc_server_wait", "qc_server_cancel", "qc_server_stats", "qc_server_destroy"]


class ServerOpts(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_int64),
                ("tie_mode", ctypes.c_uint32), ("want_potentials", ctypes.c_int32),
                ("queue_timeout_s", ctypes.c_double), ("max_bypass", ctypes.c_int32)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("footprint_bytes", ctypes.c_int64), ("n", ctypes.c_int32),
                ("n_sigmas", ctypes.c_int32), ("dmax", ctypes.c_int32), ("slot", ctypes.c_int32),
                ("status", ctypes.c_int32)]

STAGE_BFS = 0
STAGE_HIST = 1
STAGE_POTENTIAL = 2
STAGE_GGD = 3
STAGE_JUMP = 4
STAGE_DENSE = 5
STAGE_SSSP = 6
STAGE_NAMES = ["bfs", "hist", "potential", "ggd_parent", "pointer_jump", "dense", "sssp"]


class QCError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_str(status)}")


_lib = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2305_14641_amd.build` "
                "(or __graft_entry__.build()); there is no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        I32 = ctypes.c_int32
        I64 = ctypes.c_int64
        U32 = ctypes.c_uint32
        L.qc_status_str.argtypes = [I32]
        L.qc_status_str.restype = ctypes.c_char_p
        L.qc_device_count.argtypes = [P]
        L.qc_graph_create.argtypes = [I32, I64, P, P, U32, P, P]
        L.qc_graph_create_weighted.argtypes = [I32, I64, P, P, P, U32, P, P]
        L.qc_graph_destroy.argtypes = [P]
        L.qc_graph_info.argtypes = [P, P, P, P, P]
        L.qc_graph_bfs_plan.argtypes = [P, P, P, P, P]
        L.qc_distances.argtypes = [P, P, P, P]
        L.qc_get_histograms.argtypes = [P, P, P, P]
        L.qc_potential.argtypes = [P, P, I32, P, P, U32, P]
        L.qc_ggd_labels.argtypes = [P, I32, U32, P, P]
        L.qc_last_recheck_count.argtypes = [P, P]
        L.qc_graph_sync.argtypes = [P, P]
        L.qc_timing_enable.argtypes = [I32]
        L.qc_timing_read.argtypes = [I32, P, P]
        L.qc_potential_dense.argtypes = [P, I64, I64, I64, P, I32, P, P, P]
        L.qc_debug_alloc_fault.argtypes = [I64, P]
        L.qc_get_potential64.argtypes = [P, P, P]
        L.qc_cluster.argtypes = [I32, I64, P, P, P, I32, U32, P, P, P, P, P]
        L.qc_cluster_noalloc.argtypes = [I32, I64, P, P, P, I32, U32, P, P, P, P, P]
        L.qc_distances_real.argtypes = [I32, I64, P, P, P, U32, P, I64, P]
        L.qc_cluster_real.argtypes = [I32, I64, P, P, P, U32, P, I32, U32, P, P, P, P, P]
        L.qc_batch_create.argtypes = [P, I32, P, I32, U32, U32, P, P]
        L.qc_batch_node_offsets.argtypes = [P, P]
        L.qc_batch_run.argtypes = [P, P, P, P, P]
        L.qc_batch_sweep_bf16.argtypes = [P, P, P, P]
        L.qc_batch_stage_tiles.argtypes = [P, P, P, P, P, P]
        L.qc_batch_recheck_count.argtypes = [P, P]
        L.qc_batch_search_stats.argtypes = [P, P, P]
        L.qc_batch_destroy.argtypes = [P]
        L.qc_request_footprint.argtypes = [I32, I64, I32]
        L.qc_request_footprint.restype = I64
        L.qc_server_create.argtypes = [P, P]
        L.qc_server_submit.argtypes = [P, I32, I64, P, P, P, I32, P]
        L.qc_server_poll.argtypes = [P, I64, P]
        L.qc_server_wait.argtypes = [P, I64, P, P, P, P]
        L.qc_server_cancel.argtypes = [P, I64]
        L.qc_server_stats.argtypes = [P, P, P]
        L.qc_server_destroy.argtypes = [P]
        for name in EXPORTED[1:]:
            if name != "qc_request_footprint":
                getattr(L, name).restype = I32
        _lib = L
    return _lib


def status_str(status: int) -> str:
    return lib().qc_status_str(int(status)).decode()


def _check(status: int, what: str):
    if status != QC_OK:
        raise QCError(status, what)


def device_count() -> int:
    c = ctypes.c_int32(0)
    _check(lib().qc_device_count(ctypes.byref(c)), "qc_device_count")
    return int(c.value)


def debug_alloc_fault(fail_at: int) -> int:
    """Make the fail_at-th device allocation from now on fail (0 disarms);
    returns the number of device-allocator blocks the library holds."""
    live = ctypes.c_int64(0)
    _check(lib().qc_debug_alloc_fault(int(fail_at), ctypes.byref(live)), "qc_debug_alloc_fault")
    return int(live.value)


def timing_enable(on: bool = True):
    """Bracket every kernel launch with HIP events (on its own stream)."""
    _check(lib().qc_timing_enable(1 if on else 0), "qc_timing_enable")


def timing_read(stage: int) -> tuple:
    """(summed device milliseconds, launch count) of one stage."""
    ms = ctypes.c_double(0.0)
    cnt = ctypes.c_int64(0)
    _check(lib().qc_timing_read(int(stage), ctypes.byref(ms), ctypes.byref(cnt)), "qc_timing_read")
    return float(ms.value), int(cnt.value)


def _stream_ptr(stream=None):
    import torch
    if stream is None:
        if not torch.cuda.is_available():
            return None  # default stream; the library reports QC_E_DEVICE itself
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Graph:
    """A graph handle: CSR uploaded once, distances/potentials resident."""

    def __init__(self, n: int, row_ptr, col, canonicalize: bool = False, directed: bool = False,
                 weights=None, stream=None):
        """CSR graph; `weights` (one integer 1..126 per CSR entry) makes the
        distances weighted shortest-path lengths (qc_graph_create_weighted)."""
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        c = np.ascontiguousarray(col, dtype=np.int32)
        self._rp, self._col = rp, c
        h = ctypes.c_void_p()
        flags = (GRAPH_CANONICALIZE if canonicalize else 0) | (GRAPH_DIRECTED if directed else 0)
        if weights is None:
            st = lib().qc_graph_create(
                int(n), int(c.shape[0]), rp.ctypes.data_as(ctypes.c_void_p),
                c.ctypes.data_as(ctypes.c_void_p), flags, _stream_ptr(stream), ctypes.byref(h))
            _check(st, "qc_graph_create")
        else:
            w = np.ascontiguousarray(weights, dtype=np.uint8)
            if w.shape != c.shape:
                raise ValueError("one weight per CSR entry")
            self._w = w
            st = lib().qc_graph_create_weighted(
                int(n), int(c.shape[0]), rp.ctypes.data_as(ctypes.c_void_p),
                c.ctypes.data_as(ctypes.c_void_p), w.ctypes.data_as(ctypes.c_void_p), flags,
                _stream_ptr(stream), ctypes.byref(h))
            _check(st, "qc_graph_create_weighted")
        self._h = h
        self.n = int(n)
        self.sigmas = None

    @classmethod
    def from_graph(cls, g, **kw):
        return cls(g.n, g.row_ptr, g.col, **kw)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().qc_graph_destroy(self._h)
            self._h = None
        self._dist_ref = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        n = ctypes.c_int32()
        nnz = ctypes.c_int64()
        dmax = ctypes.c_int32()
        comps = ctypes.c_int32()
        _check(lib().qc_graph_info(self._h, ctypes.byref(n), ctypes.byref(nnz),
                                   ctypes.byref(dmax), ctypes.byref(comps)), "qc_graph_info")
        return dict(n=n.value, nnz=nnz.value, dmax=dmax.value, n_components=comps.value)

    def bfs_plan(self) -> tuple:
        """(batch width, words per thread, planes, workgroup shape) of the BFS."""
        v = [ctypes.c_int32() for _ in range(4)]
        _check(lib().qc_graph_bfs_plan(self._h, *[ctypes.byref(x) for x in v]), "qc_graph_bfs_plan")
        return tuple(x.value for x in v)

    def distances(self, out=None, stream=None):
        """Hop-distance matrix (int8 [n, n], -1 = unreachable) into `out`
        (a CUDA int8 tensor) or kept resident when out is None. Returns dmax."""
        if out is not None:
            self._check_tensor(out, (self.n, self.n), "int8")
        dmax = ctypes.c_int32(-1)
        _check(lib().qc_distances(self._h, _dptr(out), ctypes.byref(dmax), _stream_ptr(stream)),
               "qc_distances")
        # the handle reads (and may rewrite) this buffer until the next
        # distances() call or close(): keep the caller's tensor alive
        self._dist_ref = out
        return int(dmax.value)

    def histograms_k(self) -> int:
        """Row length K of the resident histograms (a multiple of 32)."""
        k = ctypes.c_int32(0)
        _check(lib().qc_get_histograms(self._h, None, ctypes.byref(k), None), "qc_get_histograms")
        return int(k.value)

    def histograms(self, stream=None):
        import torch
        k = ctypes.c_int32(0)
        _check(lib().qc_get_histograms(self._h, None, ctypes.byref(k), _stream_ptr(stream)),
               "qc_get_histograms")
        out = torch.empty((self.n, k.value), dtype=torch.int32, device="cuda")
        _check(lib().qc_get_histograms(self._h, _dptr(out), ctypes.byref(k), _stream_ptr(stream)),
               "qc_get_histograms")
        return out

    def potential(self, sigmas, psi=None, v=None, precision=PREC_FP64ACC, stream=None):
        """psi and V [len(sigmas), n] (float32) for each sigma."""
        import torch
        sig = np.ascontiguousarray(np.asarray(sigmas, dtype=np.float64).reshape(-1))
        S = sig.shape[0]
        if psi is None:
            psi = torch.empty((S, self.n), dtype=torch.float32, device="cuda")
        if v is None:
            v = torch.empty((S, self.n), dtype=torch.float32, device="cuda")
        self._check_tensor(psi, (S, self.n), "float32")
        self._check_tensor(v, (S, self.n), "float32")
        _check(lib().qc_potential(self._h, sig.ctypes.data_as(ctypes.c_void_p), S, _dptr(psi),
                                  _dptr(v), int(precision), _stream_ptr(stream)), "qc_potential")
        self.sigmas = sig
        return psi, v

    def labels(self, sigma_index=0, tie_mode=TIE_STRICT, out=None, stream=None):
        """Graph Gradient Descent labels (int32 [n]) for one sigma."""
        import torch
        if out is None:
            out = torch.empty((self.n,), dtype=torch.int32, device="cuda")
        self._check_tensor(out, (self.n,), "int32")
        _check(lib().qc_ggd_labels(self._h, int(sigma_index), int(tie_mode), _dptr(out),
                                   _stream_ptr(stream)), "qc_ggd_labels")
        return out

    def potential64(self, stream=None):
        """The resident canonical FP64 V [n_sigmas, n] of the last potential."""
        import torch
        S = 0 if self.sigmas is None else self.sigmas.shape[0]
        out = torch.empty((max(S, 1), self.n), dtype=torch.float64, device="cuda")
        _check(lib().qc_get_potential64(self._h, _dptr(out), _stream_ptr(stream)),
               "qc_get_potential64")
        return out[:S]

    def recheck_count(self) -> int:
        c = ctypes.c_int64(0)
        _check(lib().qc_last_recheck_count(self._h, ctypes.byref(c)), "qc_last_recheck_count")
        return int(c.value)

    def sync(self, stream=None):
        _check(lib().qc_graph_sync(self._h, _stream_ptr(stream)), "qc_graph_sync")

    @staticmethod
    def _check_tensor(t, shape, dtype):
        import torch
        want = getattr(torch, dtype)
        if not t.is_cuda or t.dtype != want or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise ValueError(f"expected a contiguous CUDA {dtype} tensor of shape {shape}")


class Batch:
    """Many graphs x one sigma list in grouped launches (include/qc_batch.h)."""

    def __init__(self, graphs, sigmas, tie_mode=TIE_STRICT, hipgraph=True, fp32c=False,
                 autotune=False, serial=False, stream=None):
        self.graphs = list(graphs)          # keeps the Graph handles alive
        arr = (ctypes.c_void_p * len(self.graphs))(*[G.handle.value for G in self.graphs])
        sig = np.ascontiguousarray(np.asarray(sigmas, dtype=np.float64).reshape(-1))
        flags = ((BATCH_HIPGRAPH if hipgraph else 0) | (BATCH_FP32C if fp32c else 0)
                 | (BATCH_AUTOTUNE if autotune else 0) | (BATCH_SERIAL if serial else 0))
        h = ctypes.c_void_p()
        _check(lib().qc_batch_create(arr, len(self.graphs), sig.ctypes.data_as(ctypes.c_void_p),
                                     sig.shape[0], int(tie_mode), flags, _stream_ptr(stream),
                                     ctypes.byref(h)), "qc_batch_create")
        self._h = h
        self.sigmas = sig
        off = np.zeros(len(self.graphs) + 1, dtype=np.int64)
        _check(lib().qc_batch_node_offsets(h, off.ctypes.data_as(ctypes.c_void_p)),
               "qc_batch_node_offsets")
        self.offsets = off
        self.total = int(off[-1])

    def outputs(self):
        import torch
        S = self.sigmas.shape[0]
        psi = torch.empty((S, self.total), dtype=torch.float32, device="cuda")
        v = torch.empty((S, self.total), dtype=torch.float32, device="cuda")
        lab = torch.empty((S, self.total), dtype=torch.int32, device="cuda")
        return psi, v, lab

    def run(self, psi, v, labels, stream=None):
        _check(lib().qc_batch_run(self._h, _dptr(psi), _dptr(v), _dptr(labels),
                                  _stream_ptr(stream)), "qc_batch_run")

    def sweep_bf16(self, psi=None, v=None, stream=None):
        """Approximate psi/V of every (sigma, node) on the matrix cores
        (qc_batch_sweep_bf16): float32 [S, total] tensors, about 1e-3
        relative error; nothing resident changes."""
        import torch
        shape = (len(self.sigmas), self.total)
        if psi is None:
            psi = torch.empty(shape, dtype=torch.float32, device="cuda")
        if v is None:
            v = torch.empty(shape, dtype=torch.float32, device="cuda")
        Graph._check_tensor(psi, shape, "float32")
        Graph._check_tensor(v, shape, "float32")
        _check(lib().qc_batch_sweep_bf16(self._h, _dptr(psi), _dptr(v), _stream_ptr(stream)),
               "qc_batch_sweep_bf16")
        return psi, v

    def recheck_count(self) -> int:
        c = ctypes.c_int64(0)
        _check(lib().qc_batch_recheck_count(self._h, ctypes.byref(c)), "qc_batch_recheck_count")
        return int(c.value)

    def stage_tiles(self) -> dict:
        """Launch shapes of the stages: the BFS planning policy (widest batch,
        seen-in-registers shape first), the histogram pass (wavefronts per
        workgroup by row length), the pointer jumping (LDS or global) and
        which stages run beside the searches ("all", "histograms",
        "histograms and the tail": the other graphs' later stages beside the
        last search, or "none")."""
        bw, ff, j, ov = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
        w = (ctypes.c_int32 * 3)()
        _check(lib().qc_batch_stage_tiles(self._h, ctypes.byref(bw), ctypes.byref(ff), w,
                                          ctypes.byref(j), ctypes.byref(ov)), "qc_batch_stage_tiles")
        return {"bfs_widest": bw.value, "bfs_front_first": bool(ff.value),
                "hist_waves": {32: w[0], 64: w[1], 128: w[2]}, "jump": "global" if j.value else "lds",
                "overlap": {0: "none", 1: "histograms", 2: "all",
                            3: "histograms and the tail"}[ov.value]}

    def search_stats(self) -> tuple:
        """(edge visits, LDS bytes gathered) of the last run's searches."""
        v = ctypes.c_int64(0)
        b = ctypes.c_int64(0)
        _check(lib().qc_batch_search_stats(self._h, ctypes.byref(v), ctypes.byref(b)),
               "qc_batch_search_stats")
        return int(v.value), int(b.value)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().qc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def request_footprint(n: int, nnz: int, n_sigmas: int) -> int:
    return int(lib().qc_request_footprint(int(n), int(nnz), int(n_sigmas)))


class Server:
    """Continuous-batching request loop (include/qc_server.h)."""

    def __init__(self, max_slots=4, hbm_budget_bytes=16 << 30, tie_mode=TIE_STRICT,
                 want_potentials=False, queue_timeout_s=0.0, max_bypass=0):
        o = ServerOpts(int(max_slots), int(hbm_budget_bytes), int(tie_mode),
                       1 if want_potentials else 0, float(queue_timeout_s), int(max_bypass))
        h = ctypes.c_void_p()
        _check(lib().qc_server_create(ctypes.byref(o), ctypes.byref(h)), "qc_server_create")
        self._h = h
        self._meta = {}
        self.want_potentials = want_potentials

    def submit(self, n, row_ptr, col, sigmas) -> int:
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        c = np.ascontiguousarray(col, dtype=np.int32)
        sig = np.ascontiguousarray(np.asarray(sigmas, dtype=np.float64).reshape(-1))
        rid = ctypes.c_int64(0)
        _check(lib().qc_server_submit(self._h, int(n), int(c.shape[0]),
                                      rp.ctypes.data_as(ctypes.c_void_p),
                                      c.ctypes.data_as(ctypes.c_void_p),
                                      sig.ctypes.data_as(ctypes.c_void_p), sig.shape[0],
                                      ctypes.byref(rid)), "qc_server_submit")
        self._meta[rid.value] = (int(n), sig.shape[0])
        return int(rid.value)

    def poll(self, rid) -> bool:
        d = ctypes.c_int32(0)
        _check(lib().qc_server_poll(self._h, int(rid), ctypes.byref(d)), "qc_server_poll")
        return bool(d.value)

    def wait(self, rid):
        """(labels [S, n] int32, psi, V [S, n] float32 or None, info dict)."""
        n, S = self._meta.pop(rid)
        lab = np.empty((S, n), dtype=np.int32)
        psi = np.empty((S, n), dtype=np.float32) if self.want_potentials else None
        v = np.empty((S, n), dtype=np.float32) if self.want_potentials else None
        info = RequestInfo()
        st = lib().qc_server_wait(self._h, int(rid), lab.ctypes.data_as(ctypes.c_void_p),
                                  psi.ctypes.data_as(ctypes.c_void_p) if psi is not None else None,
                                  v.ctypes.data_as(ctypes.c_void_p) if v is not None else None,
                                  ctypes.byref(info))
        _check(st, f"request {rid}")
        d = {k: getattr(info, k) for k, _ in RequestInfo._fields_}
        return lab, psi, v, d

    def cancel(self, rid) -> int:
        """Withdraw a queued request; returns the library status (QC_OK when
        withdrawn, QC_E_BUSY when already running, QC_E_STATE when done)."""
        return int(lib().qc_server_cancel(self._h, int(rid)))

    def stats(self) -> dict:
        b = ctypes.c_int64(0)
        r = ctypes.c_int32(0)
        _check(lib().qc_server_stats(self._h, ctypes.byref(b), ctypes.byref(r)), "qc_server_stats")
        return {"peak_bytes_in_flight": int(b.value), "peak_requests_in_flight": int(r.value)}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().qc_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def potential_dense(dist, sigmas, n_cols=None, psi=None, v=None, stream=None):
    """Algorithm 1 on a dense float32 CUDA matrix of distances (rows = nodes;
    negative = no path). `dist` may be a row-strided view (stride(1) == 1);
    `n_cols` defaults to its width. Returns FP64 (psi, V), each [S, n_rows]."""
    import torch
    if not dist.is_cuda or dist.dtype != torch.float32 or dist.dim() != 2 or dist.stride(1) != 1:
        raise ValueError("expected a CUDA float32 matrix with unit column stride")
    n_rows, width = dist.shape
    n_cols = width if n_cols is None else int(n_cols)
    if not 0 <= n_cols <= width:
        raise ValueError("n_cols outside the matrix")
    sig = np.ascontiguousarray(sigmas, dtype=np.float64)
    shape = (sig.shape[0], n_rows)
    if psi is None:
        psi = torch.empty(shape, dtype=torch.float64, device=dist.device)
    if v is None:
        v = torch.empty(shape, dtype=torch.float64, device=dist.device)
    Graph._check_tensor(psi, shape, "float64")
    Graph._check_tensor(v, shape, "float64")
    ld = dist.stride(0) if n_rows > 1 else max(width, 1)
    st = lib().qc_potential_dense(_dptr(dist), int(n_rows), int(n_cols), int(ld),
                                  sig.ctypes.data_as(ctypes.c_void_p), int(sig.shape[0]),
                                  _dptr(psi), _dptr(v), _stream_ptr(stream))
    _check(st, "qc_potential_dense")
    return psi, v


def _cluster_args(n, row_ptr, col, sigmas, dist, psi, v, labels):
    import torch
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    c = np.ascontiguousarray(col, dtype=np.int32)
    sig = np.ascontiguousarray(np.asarray(sigmas, dtype=np.float64).reshape(-1))
    S = sig.shape[0]
    if labels is None:
        labels = torch.empty((S, n), dtype=torch.int32, device="cuda")
    Graph._check_tensor(labels, (S, n), "int32")
    if dist is not None:
        Graph._check_tensor(dist, (n, n), "int8")
    for t in (psi, v):
        if t is not None:
            Graph._check_tensor(t, (S, n), "float32")
    return rp, c, sig, labels


def cluster(n, row_ptr, col, sigmas, tie_mode=TIE_STRICT, dist=None, psi=None, v=None,
            labels=None, stream=None):
    """Algorithm 4 in one call (qc_cluster): labels [S, n] int32 on the GPU
    (and the optional dist / psi / v outputs filled)."""
    rp, c, sig, labels = _cluster_args(n, row_ptr, col, sigmas, dist, psi, v, labels)
    _check(lib().qc_cluster(int(n), int(c.shape[0]), rp.ctypes.data_as(ctypes.c_void_p),
                            c.ctypes.data_as(ctypes.c_void_p), sig.ctypes.data_as(ctypes.c_void_p),
                            sig.shape[0], int(tie_mode), _dptr(dist), _dptr(psi), _dptr(v),
                            _dptr(labels), _stream_ptr(stream)), "qc_cluster")
    return labels


def cluster_noalloc(n, row_ptr, col, sigmas, tie_mode=TIE_STRICT, dist=None, psi=None, v=None,
                    labels=None, stream=None):
    """qc_cluster_noalloc: as cluster(), with every device buffer besides the
    outputs carved from the library's fixed device scratch (no allocation;
    QC_E_TOO_LARGE when the problem does not fit it). Pass `labels` (and any
    other output) preallocated to keep the call free of allocations."""
    rp, c, sig, labels = _cluster_args(n, row_ptr, col, sigmas, dist, psi, v, labels)
    _check(lib().qc_cluster_noalloc(int(n), int(c.shape[0]), rp.ctypes.data_as(ctypes.c_void_p),
                                    c.ctypes.data_as(ctypes.c_void_p),
                                    sig.ctypes.data_as(ctypes.c_void_p), sig.shape[0],
                                    int(tie_mode), _dptr(dist), _dptr(psi), _dptr(v),
                                    _dptr(labels), _stream_ptr(stream)), "qc_cluster_noalloc")
    return labels


def _real_args(n, row_ptr, col, weights):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    c = np.ascontiguousarray(col, dtype=np.int32)
    w = np.ascontiguousarray(weights, dtype=np.float32)
    if w.shape != c.shape:
        raise ValueError("one weight per CSR entry")
    return rp, c, w


def distances_real(n, row_ptr, col, weights, directed=False, out=None, stream=None):
    """qc_distances_real: float32 [n, n] shortest-path lengths under positive
    real edge weights (one per CSR entry), +inf where unreachable."""
    import torch
    rp, c, w = _real_args(n, row_ptr, col, weights)
    if out is None:
        out = torch.empty((n, n), dtype=torch.float32, device="cuda")
    if not out.is_cuda or out.dtype != torch.float32 or out.dim() != 2 or out.stride(1) != 1 \
            or out.shape[0] != n or out.shape[1] < n:
        raise ValueError("expected a CUDA float32 [n, >= n] matrix with unit column stride")
    ld = out.stride(0) if n > 1 else max(out.shape[1], 1)
    _check(lib().qc_distances_real(int(n), int(c.shape[0]), rp.ctypes.data_as(ctypes.c_void_p),
                                   c.ctypes.data_as(ctypes.c_void_p),
                                   w.ctypes.data_as(ctypes.c_void_p),
                                   GRAPH_DIRECTED if directed else 0, _dptr(out), int(ld),
                                   _stream_ptr(stream)), "qc_distances_real")
    return out


def cluster_real(n, row_ptr, col, weights, sigmas, tie_mode=TIE_STRICT, directed=False, dist=None,
                 psi=None, v=None, labels=None, stream=None):
    """qc_cluster_real: labels [S, n] int32 of a graph with real edge weights
    (and the optional float32 dist [n, n], FP64 psi / v [S, n] filled)."""
    import torch
    rp, c, w = _real_args(n, row_ptr, col, weights)
    sig = np.ascontiguousarray(np.asarray(sigmas, dtype=np.float64).reshape(-1))
    S = sig.shape[0]
    if labels is None:
        labels = torch.empty((S, n), dtype=torch.int32, device="cuda")
    Graph._check_tensor(labels, (S, n), "int32")
    if dist is not None:
        Graph._check_tensor(dist, (n, n), "float32")
    for t in (psi, v):
        if t is not None:
            Graph._check_tensor(t, (S, n), "float64")
    _check(lib().qc_cluster_real(int(n), int(c.shape[0]), rp.ctypes.data_as(ctypes.c_void_p),
                                 c.ctypes.data_as(ctypes.c_void_p), w.ctypes.data_as(ctypes.c_void_p),
                                 GRAPH_DIRECTED if directed else 0,
                                 sig.ctypes.data_as(ctypes.c_void_p), S, int(tie_mode), _dptr(dist),
                                 _dptr(psi), _dptr(v), _dptr(labels), _stream_ptr(stream)),
           "qc_cluster_real")
    return labels
