"""C-ABI checks that need no GPU: the library loads, exports every symbol the
headers declare, and rejects invalid input on the host before any device work
(qc_graph_create validates first; on a machine without a gfx950 device a
valid graph is refused with QC_E_DEVICE)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2305_14641_amd import qc
from paper_2305_14641_amd import graphgen as gg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(inc, fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(qc_\w+)\s*\(", text, re.M):
            names.add(m.group(1))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = qc.lib()
    names = declared_symbols()
    assert "qc_graph_create" in names and "qc_potential" in names
    for name in names:
        assert hasattr(L, name), name
    assert set(qc.EXPORTED) <= set(names)


def test_status_strings():
    for s in range(10):
        assert qc.status_str(s).startswith("QC_")
    assert "unknown" in qc.status_str(99)


def create(n, rp, col, flags=0):
    h = ctypes.c_void_p()
    rp = np.ascontiguousarray(rp, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    st = qc.lib().qc_graph_create(n, col.shape[0], rp.ctypes.data_as(ctypes.c_void_p),
                                  col.ctypes.data_as(ctypes.c_void_p) if col.size else None,
                                  flags, None, ctypes.byref(h))
    if st == qc.QC_OK:
        qc.lib().qc_graph_destroy(h)
    return st


@pytest.mark.parametrize("case,want", [
    ((0, [0], []), qc.QC_E_INVAL),                          # n = 0
    ((70000, [0] * 70001, []), qc.QC_E_INVAL),              # n above 65536
    ((3, [0, 1, 2, 2], [1, 0, 0]), qc.QC_E_INVAL),          # row_ptr[n] != nnz... (3 entries, rp[3]=2)
    ((2, [0, 2, 1], [1, 0]), qc.QC_E_INVAL),                # decreasing row_ptr
    ((2, [0, 1, 2], [1, 5]), qc.QC_E_INVAL),                # column out of range
    ((2, [0, 1, 2], [1, 1]), qc.QC_E_NOT_SYMMETRIC),        # self-loop
    ((3, [0, 1, 1, 1], [1]), qc.QC_E_NOT_SYMMETRIC),        # (0,1) without (1,0)
    ((3, [0, 2, 3, 4], [2, 1, 0, 0]), qc.QC_E_NOT_SYMMETRIC),  # unsorted row
    ((3, [0, 2, 3, 4], [1, 1, 0, 0]), qc.QC_E_NOT_SYMMETRIC),  # duplicate entry
])
def test_invalid_csr_rejected_on_host(case, want):
    n, rp, col = case
    assert create(n, rp, col) == want


def test_edge_count_limit_checked_first():
    """nnz must stay below 2^29; the count is checked before the arrays are read."""
    L = qc.lib()
    h = ctypes.c_void_p()
    rp = np.array([0, 1, 2], np.int32)
    col = np.array([1, 0], np.int32)
    for nnz in (1 << 29, (1 << 31) - 1, -1):
        assert L.qc_graph_create(2, nnz, rp.ctypes.data_as(ctypes.c_void_p),
                                 col.ctypes.data_as(ctypes.c_void_p), 0, None,
                                 ctypes.byref(h)) == qc.QC_E_INVAL, nnz


def test_null_pointers_rejected():
    L = qc.lib()
    h = ctypes.c_void_p()
    assert L.qc_graph_create(2, 2, None, None, 0, None, ctypes.byref(h)) == qc.QC_E_INVAL
    rp = np.array([0, 1, 2], np.int32)
    col = np.array([1, 0], np.int32)
    assert L.qc_graph_create(2, 2, rp.ctypes.data_as(ctypes.c_void_p),
                             col.ctypes.data_as(ctypes.c_void_p), 0, None, None) == qc.QC_E_INVAL
    assert L.qc_graph_create(2, 2, rp.ctypes.data_as(ctypes.c_void_p),
                             col.ctypes.data_as(ctypes.c_void_p), 8, None,
                             ctypes.byref(h)) == qc.QC_E_INVAL  # unknown flag
    for fn, args in [("qc_graph_destroy", [None]), ("qc_distances", [None, None, None, None]),
                     ("qc_potential", [None, None, 1, None, None, 0, None]),
                     ("qc_ggd_labels", [None, 0, 0, None, None]),
                     ("qc_graph_info", [None, None, None, None, None]),
                     ("qc_graph_bfs_plan", [None, None, None, None, None]),
                     ("qc_graph_sync", [None, None]),
                     ("qc_last_recheck_count", [None, None]),
                     ("qc_get_histograms", [None, None, None, None])]:
        assert getattr(L, fn)(*args) == qc.QC_E_INVAL, fn


def test_request_footprint_host_only():
    n, nnz, S = 19717, 88726, 2
    fp = qc.request_footprint(n, nnz, S)
    # the request's own distance matrix has its rows on 128-byte lines
    ld = -(-n // 128) * 128
    assert fp >= n * ld + 4 * (n + 1) + 4 * nnz + 24 * n * S
    assert fp < n * n * 1.2
    # one node past a multiple of 128 pads every row by 127 bytes: from 1,024
    # to 1,025 nodes the matrix alone grows by 1025 * 1152 - 1024 * 1024
    # bytes (dense rows would add 2,049, the other buffers a few KB)
    grow = qc.request_footprint(1025, 4096, 1) - qc.request_footprint(1024, 4096, 1)
    assert grow >= 1025 * 1152 - 1024 * 1024
    assert qc.request_footprint(n, nnz, 3) > fp
    assert qc.request_footprint(0, 1, 1) == -1
    assert qc.request_footprint(10, 4, 0) == -1


def test_valid_graph_without_gpu_reports_device():
    if qc.device_count() > 0:
        pytest.skip("a gfx950 device is visible")
    g = gg.config1()
    assert create(g.n, g.row_ptr, g.col) == qc.QC_E_DEVICE
    # a non-canonical graph that canonicalises is also valid input
    assert create(3, [0, 2, 3, 4], [2, 1, 0, 0], flags=qc.GRAPH_CANONICALIZE) == qc.QC_E_DEVICE


def test_binding_refuses_missing_library(monkeypatch, tmp_path):
    monkeypatch.setattr(qc, "_lib", None)
    monkeypatch.setattr(qc, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        qc.lib()


def test_dense_potential_arguments_checked_on_host():
    """qc_potential_dense validates sizes and widths before touching a device."""
    L = qc.lib()
    sig = np.array([1.0], dtype=np.float64)
    sp = sig.ctypes.data_as(ctypes.c_void_p)
    fake = ctypes.c_void_p(4096)      # never dereferenced: every call below fails validation
    bad = [
        (fake, -1, 4, 4, sp, 1, fake, fake),       # negative rows
        (fake, 4, -1, 4, sp, 1, fake, fake),       # negative columns
        (fake, 4, 8, 4, sp, 1, fake, fake),        # ld < n_cols
        (fake, 4, 4, 4, None, 1, fake, fake),      # no sigmas
        (fake, 4, 4, 4, sp, 0, fake, fake),        # zero sigmas
        (None, 4, 4, 4, sp, 1, fake, fake),        # no matrix
        (fake, 4, 4, 4, sp, 1, None, fake),        # no psi
        (fake, 4, 4, 4, sp, 1, fake, None),        # no V
    ]
    for args in bad:
        assert L.qc_potential_dense(*args, None) == qc.QC_E_INVAL, args
    for s in (0.0, -1.0, float("nan"), float("inf"), 1e-101):
        sig[0] = s
        assert L.qc_potential_dense(fake, 4, 4, 4, sp, 1, fake, fake, None) == qc.QC_E_INVAL, s
    sig[0] = 1.0
    assert L.qc_potential_dense(None, 0, 4, 4, sp, 1, None, None, None) == qc.QC_OK   # no rows
    assert L.qc_potential_dense(fake, 4, 4, 4, sp, 1, fake, fake, None) == qc.QC_E_DEVICE


def test_directed_flag_validation_on_host():
    """QC_GRAPH_DIRECTED drops only the symmetry requirement; order,
    duplicates and self-loops are still checked (canonicalisation sorts and
    dedupes without symmetrising)."""
    D = qc.GRAPH_DIRECTED
    arc = (3, [0, 1, 2, 2], [1, 2])                   # 0->1, 1->2: not symmetric
    assert create(*arc) == qc.QC_E_NOT_SYMMETRIC
    ok = qc.QC_OK if qc.device_count() > 0 else qc.QC_E_DEVICE
    assert create(*arc, flags=D) == ok
    assert create(2, [0, 1, 1], [0], flags=D) == qc.QC_E_NOT_SYMMETRIC        # self-loop
    assert create(3, [0, 2, 2, 2], [2, 1], flags=D) == qc.QC_E_NOT_SYMMETRIC  # unsorted row
    assert create(3, [0, 2, 2, 2], [1, 1], flags=D) == qc.QC_E_NOT_SYMMETRIC  # duplicate arc
    assert create(3, [0, 3, 3, 3], [2, 1, 1], flags=D | qc.GRAPH_CANONICALIZE) == ok
    assert create(3, [0, 1, 2, 2], [1, 2], flags=4) == qc.QC_E_INVAL           # unknown flag


def test_weighted_graph_validation_on_host():
    """qc_graph_create_weighted checks weights before touching a device."""
    L = qc.lib()

    def create_w(n, rp, col, w, flags=0):
        h = ctypes.c_void_p()
        rp = np.ascontiguousarray(rp, dtype=np.int32)
        col = np.ascontiguousarray(col, dtype=np.int32)
        w = np.ascontiguousarray(w, dtype=np.uint8)
        st = L.qc_graph_create_weighted(n, col.shape[0], rp.ctypes.data_as(ctypes.c_void_p),
                                        col.ctypes.data_as(ctypes.c_void_p) if col.size else None,
                                        w.ctypes.data_as(ctypes.c_void_p) if w.size else None,
                                        flags, None, ctypes.byref(h))
        if st == qc.QC_OK:
            L.qc_graph_destroy(h)
        return st

    ok = qc.QC_OK if qc.device_count() > 0 else qc.QC_E_DEVICE
    path = (3, [0, 1, 3, 4], [1, 0, 2, 1])              # 0-1-2
    assert create_w(*path, [2, 2, 5, 5]) == ok
    assert create_w(*path, [2, 3, 5, 5]) == qc.QC_E_NOT_SYMMETRIC   # the two entries differ
    assert create_w(*path, [0, 0, 5, 5]) == qc.QC_E_INVAL           # weight 0
    assert create_w(*path, [127, 127, 5, 5]) == qc.QC_E_INVAL       # above 126
    assert create_w(*path, [2, 2, 5, 5], flags=qc.GRAPH_CANONICALIZE) == qc.QC_E_INVAL
    assert create_w(3, [0, 1, 2, 2], [1, 2], [9, 4], flags=qc.GRAPH_DIRECTED) == ok
    # a star of 600 nodes whose 599 edges weigh 126 has 600 + 599 * 125 = 75,475
    # nodes once subdivided: too many; with weight 100, 59,901 nodes fit
    n = 600
    rows = np.concatenate([np.zeros(n - 1, dtype=np.int32), np.arange(1, n, dtype=np.int32)])
    cols = np.concatenate([np.arange(1, n, dtype=np.int32), np.zeros(n - 1, dtype=np.int32)])
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    rp = np.zeros(n + 1, dtype=np.int32)
    np.cumsum(np.bincount(rows, minlength=n), out=rp[1:])
    assert create_w(n, rp, cols, np.full(cols.shape[0], 126, dtype=np.uint8)) == qc.QC_E_INVAL
    assert create_w(n, rp, cols, np.full(cols.shape[0], 100, dtype=np.uint8)) == ok


def test_cluster_arguments_checked_on_host():
    """qc_cluster validates its arguments and the CSR before any device work."""
    L = qc.lib()
    g = gg.config1()
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    sig = np.array([1.0, 2.0])
    P = ctypes.c_void_p

    def call(n=g.n, rp_=rp, col_=col, sig_=sig, tie=0, dist=None, labels=P(64)):
        return L.qc_cluster(n, col_.shape[0], rp_.ctypes.data_as(P), col_.ctypes.data_as(P),
                            sig_.ctypes.data_as(P), sig_.shape[0], tie, dist, None, None,
                            labels, None)

    assert call(labels=None) == qc.QC_E_INVAL                 # labels are required
    assert call(tie=2) == qc.QC_E_INVAL
    assert call(dist=P(65)) == qc.QC_E_INVAL                  # distances not 16-byte aligned
    assert call(sig_=np.array([1.0, 0.0])) == qc.QC_E_INVAL
    bad = col.copy()
    bad[0], bad[1] = bad[1], bad[0]                           # an unsorted row
    if g.row_ptr[1] - g.row_ptr[0] >= 2:
        assert call(col_=bad) == qc.QC_E_NOT_SYMMETRIC
    if qc.device_count() == 0:
        assert call() == qc.QC_E_DEVICE


def test_real_weight_arguments_checked_on_host():
    """qc_distances_real and qc_cluster_real check the CSR, the weights and
    their own arguments before any device work."""
    L = qc.lib()
    P = ctypes.c_void_p
    path = (3, np.array([0, 1, 3, 4], dtype=np.int32), np.array([1, 0, 2, 1], dtype=np.int32))

    def dist(n, rp, col, w, flags=0, out=P(256), ld=None):
        w = np.ascontiguousarray(w, dtype=np.float32)
        return L.qc_distances_real(n, col.shape[0], rp.ctypes.data_as(P), col.ctypes.data_as(P),
                                   w.ctypes.data_as(P) if w.size else None, flags, out,
                                   n if ld is None else ld, None)

    def clus(n, rp, col, w, sig=(1.0,), tie=0, labels=P(256), flags=0):
        w = np.ascontiguousarray(w, dtype=np.float32)
        s_ = np.ascontiguousarray(sig, dtype=np.float64)
        return L.qc_cluster_real(n, col.shape[0], rp.ctypes.data_as(P), col.ctypes.data_as(P),
                                 w.ctypes.data_as(P) if w.size else None, flags,
                                 s_.ctypes.data_as(P), s_.shape[0], tie, None, None, None, labels,
                                 None)

    good = [0.5, 0.5, 2.25, 2.25]
    if qc.device_count() == 0:
        assert dist(*path, good) == qc.QC_E_DEVICE
        assert clus(*path, good) == qc.QC_E_DEVICE
    assert dist(*path, good, out=None) == qc.QC_E_INVAL               # no output
    assert dist(*path, good, ld=2) == qc.QC_E_INVAL                   # ld < n
    assert dist(*path, [0.5, 0.75, 2.25, 2.25]) == qc.QC_E_NOT_SYMMETRIC
    for bad in (0.0, -1.0, np.nan, np.inf, 1e-40):                    # 1e-40: subnormal
        assert dist(*path, [bad, bad, 2.25, 2.25]) == qc.QC_E_INVAL, bad
    assert dist(*path, good, flags=qc.GRAPH_CANONICALIZE) == qc.QC_E_INVAL
    assert dist(3, path[1], np.array([1, 0, 1, 2], dtype=np.int32), good) == qc.QC_E_NOT_SYMMETRIC
    big = 32769                                                       # above the LDS row
    assert dist(big, np.zeros(big + 1, dtype=np.int32), np.zeros(0, dtype=np.int32), []) \
        == qc.QC_E_INVAL
    assert clus(*path, good, labels=None) == qc.QC_E_INVAL
    assert clus(*path, good, tie=2) == qc.QC_E_INVAL
    assert clus(*path, good, sig=(1.0, 0.0)) == qc.QC_E_INVAL
    assert clus(*path, good, sig=(1e-200,)) == qc.QC_E_INVAL
    assert clus(*path, [0.5, 0.75, 2.25, 2.25]) == qc.QC_E_NOT_SYMMETRIC
    if qc.device_count() == 0:
        # directed: the weights need not match across directions
        assert dist(3, np.array([0, 1, 2, 2], dtype=np.int32), np.array([1, 2], dtype=np.int32),
                    [0.5, 3.0], flags=qc.GRAPH_DIRECTED) == qc.QC_E_DEVICE


def test_noalloc_arguments_and_size_checked_on_host():
    """qc_cluster_noalloc validates its arguments and refuses a problem beyond
    its fixed scratch (QC_E_TOO_LARGE) before touching any device."""
    L = qc.lib()
    P = ctypes.c_void_p
    sig = np.array([1.0])

    def call(g, sig_=sig, tie=0, dist=None, labels=P(64)):
        rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
        col = np.ascontiguousarray(g.col, dtype=np.int32)
        return L.qc_cluster_noalloc(g.n, col.shape[0], rp.ctypes.data_as(P), col.ctypes.data_as(P),
                                    sig_.ctypes.data_as(P), sig_.shape[0], tie, dist, None, None,
                                    labels, None)

    small = gg.config1()
    assert call(small, labels=None) == qc.QC_E_INVAL
    assert call(small, tie=2) == qc.QC_E_INVAL
    assert call(small, dist=P(65)) == qc.QC_E_INVAL
    assert call(small, sig_=np.array([-1.0])) == qc.QC_E_INVAL
    big = gg.star_graph(8199)           # its 67 MB matrix alone exceeds the 64 MiB scratch
    assert big.n * big.n > qc.NOALLOC_SCRATCH_BYTES
    assert call(big) == qc.QC_E_TOO_LARGE
    assert L.qc_status_str(qc.QC_E_TOO_LARGE).startswith(b"QC_E_TOO_LARGE")
    if qc.device_count() == 0:
        assert call(small) == qc.QC_E_DEVICE
        assert call(big, dist=P(1 << 20)) == qc.QC_E_DEVICE   # fits once the caller holds the matrix


def test_hooks_and_new_entry_points_reject_bad_handles():
    L = qc.lib()
    live = ctypes.c_int64(-1)
    assert L.qc_debug_alloc_fault(-1, None) == qc.QC_E_INVAL
    assert L.qc_debug_alloc_fault(0, ctypes.byref(live)) == qc.QC_OK
    assert live.value >= 0
    assert L.qc_get_potential64(None, ctypes.c_void_p(64), None) == qc.QC_E_INVAL
    assert L.qc_batch_search_stats(None, None, None) == qc.QC_E_INVAL
    assert L.qc_batch_sweep_bf16(None, ctypes.c_void_p(64), ctypes.c_void_p(64), None) == qc.QC_E_INVAL
    assert L.qc_batch_stage_tiles(None, None, None, None, None, None) == qc.QC_E_INVAL
    assert L.qc_server_cancel(None, 1) == qc.QC_E_INVAL


@pytest.mark.parametrize("timeout,bypass", [(-1.0, 0), (float("nan"), 0), (0.0, -1),
                                            (0.0, 2_000_000)])
def test_server_options_checked_on_host(timeout, bypass):
    o = qc.ServerOpts(2, 1 << 20, 0, 0, timeout, bypass)
    h = ctypes.c_void_p()
    assert qc.lib().qc_server_create(ctypes.byref(o), ctypes.byref(h)) == qc.QC_E_INVAL
