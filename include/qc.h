/*
 * qc.h — C ABI of the MI355X (gfx950) graph Quantum Clustering library.
 *
 * The library computes, for an undirected graph, the quantities of Section 3.1
 * of Wang, He & Liu, "Graph Analysis Using a GPU-based Parallel Algorithm:
 * Quantum Clustering" (arXiv 2305.14641):
 *   - node-to-node distances (hop counts of shortest paths),
 *   - the wave function psi (Eq. 2) and the potential V (Eq. 7, approximate
 *     form, as computed by Algorithm 1) of every node for a list of widths
 *     sigma,
 *   - Graph Gradient Descent labels (Algorithms 2-4): each node descends to
 *     its lowest neighbour while that neighbour is strictly lower; the label
 *     is the id of the local minimum where the descent ends.
 *
 * Conventions shared by every entry point:
 *   - Every call returns a qc_status; nothing throws or aborts across the ABI.
 *   - Arguments are validated on the host before any device work; on an error
 *     status nothing has been written to any output.
 *   - Pointers documented as "device" are HIP device pointers (e.g. a torch
 *     tensor's data_ptr()); the caller owns them and keeps them alive until
 *     the stream has passed the call. Pointers documented as "host" are read
 *     (or written) before the call returns.
 *   - `stream` is a hipStream_t passed as void*; NULL means the default
 *     stream. Device work is ordered on that stream; device outputs are valid
 *     once the stream has reached the call (e.g. after qc_graph_sync).
 *   - Node ids are 0-based. Distances are int8: 0..126 for reachable pairs,
 *     -1 for unreachable pairs; a finite distance above 126 is an error
 *     (QC_E_OVERFLOW), never truncated.
 *   - One handle is used by one host thread at a time; distinct handles are
 *     independent.
 */
#ifndef QC_H_
#define QC_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t qc_status;

enum {
    QC_OK = 0,
    QC_E_INVAL = 1,         /* NULL pointer, size out of range, sigma <= 0 or not finite */
    QC_E_NOT_SYMMETRIC = 2, /* CSR not canonical: unsorted, duplicated, self-loops, or (undirected) asymmetric */
    QC_E_OOM = 3,           /* device or pinned-host allocation failed */
    QC_E_DEVICE = 4,        /* no gfx950 device visible, or a HIP call failed */
    QC_E_OVERFLOW = 5,      /* a finite hop distance above 126 */
    QC_E_STATE = 6,         /* call order violated (e.g. labels before potential) */
    QC_E_BUSY = 7,          /* serving: request does not fit the memory budget, or is already running */
    QC_E_TIMEOUT = 8,       /* serving: request not admitted before its queue deadline */
    QC_E_CANCELLED = 9,     /* serving: request withdrawn by qc_server_cancel */
    QC_E_TOO_LARGE = 10     /* qc_cluster_noalloc: the problem exceeds its fixed device scratch */
};

/* Tie rules of the descent (Algorithm 2 and the prose after Algorithm 4).
 * STRICT: a node moves to the lowest neighbour (equal neighbours -> smallest
 *         id) only if that neighbour's V is strictly lower than its own.
 * MERGE:  a node moves to the (V, id)-lexicographic minimum over itself and
 *         its neighbours, so equal-V neighbours join the smallest id. */
enum { QC_TIE_STRICT = 0, QC_TIE_MERGE = 1 };

/* Arithmetic of qc_potential (psi and V are always returned as FP32).
 * FP64ACC: histogram x weight products accumulated in FP64 (default).
 * FP32C:   FP32 with compensated (error-free transformation) sums.
 * BF16:    histograms and weights rounded to BF16, FP32 accumulation on the
 *          matrix cores; approximate (about 1e-3 relative) — qc_ggd_labels
 *          refuses potentials computed this way (QC_E_STATE). */
enum { QC_PREC_FP64ACC = 0, QC_PREC_FP32C = 1, QC_PREC_BF16 = 2 };

/* qc_graph_create flags. */
enum {
    QC_GRAPH_CANONICALIZE = 1u, /* sort, drop duplicates and self-loops (and, undirected, symmetrise) first */
    QC_GRAPH_DIRECTED = 2u      /* rows are out-neighbours; distances follow edge direction */
};

typedef struct qc_graph_s *qc_graph;

/* Human-readable name of a status code (static string, never NULL). */
const char *qc_status_str(qc_status s);

/* Number of visible gfx950 devices (0 when none); does not touch any handle. */
qc_status qc_device_count(int32_t *count_out);

/*
 * Create a graph handle from a CSR adjacency (the adjacency matrix of
 * Algorithm 1's input, stored sparsely).
 *   n        number of nodes, 1 <= n <= 65536
 *   nnz      number of stored entries (2 x undirected edges, or the directed
 *            edges), 0 <= nnz < 2^29
 *   row_ptr  host, int32[n+1], row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz
 *   col_idx  host, int32[nnz], neighbours of node i in row_ptr[i]..row_ptr[i+1]-1
 *   flags    0: the CSR must already be canonical (each row strictly
 *            increasing, no self-loop, (i,j) present iff (j,i) present),
 *            else QC_E_NOT_SYMMETRIC; QC_GRAPH_CANONICALIZE: the library
 *            canonicalises a copy first (the input is left unchanged).
 *            QC_GRAPH_DIRECTED: row i lists the heads of the edges leaving
 *            i (no symmetry required; canonical = sorted rows, no duplicate,
 *            no self-loop). Distances are then directed: d(i,j) is the
 *            length of a shortest path from i to j along edge directions,
 *            row i of the matrix holds the distances from i, and the descent
 *            moves a node only to one of its out-neighbours.
 *   stream   stream for the upload
 *   out      host, receives the handle (unchanged on error)
 * The library copies the CSR; the caller keeps ownership of its arrays.
 */
qc_status qc_graph_create(int32_t n, int64_t nnz, const int32_t *row_ptr,
                          const int32_t *col_idx, uint32_t flags, void *stream,
                          qc_graph *out);

/*
 * A graph handle whose distances are shortest-path lengths under positive
 * integer edge weights (Section 3.1: a path's length is the sum of its
 * edges' weights), for the same histogram, potential and descent path.
 *   weights  host, uint8[nnz], 1..126, one per CSR entry; for an undirected
 *            graph both entries of an edge must carry the same weight
 *   flags    0 or QC_GRAPH_DIRECTED (the CSR must be canonical: no
 *            QC_GRAPH_CANONICALIZE, since the weights follow its entries)
 * Internally an edge of weight w is walked as w unit steps, through w - 1
 * extra nodes, so n + sum over edges of (w - 1) must not exceed 65536 and
 * the entries of the subdivided graph must stay below 2^29 (else
 * QC_E_INVAL), and qc_distances reports QC_E_OVERFLOW when any of
 * those steps lies farther than 126 from a source (so distances up to 126
 * minus half the heaviest weight are always representable). The descent uses
 * the graph's own edges. Other arguments and errors as qc_graph_create;
 * QC_E_NOT_SYMMETRIC also when the two weights of an undirected edge differ.
 */
qc_status qc_graph_create_weighted(int32_t n, int64_t nnz, const int32_t *row_ptr,
                                   const int32_t *col_idx, const uint8_t *weights, uint32_t flags,
                                   void *stream, qc_graph *out);

/* Release a handle and all device memory it owns (waits for its work). */
qc_status qc_graph_destroy(qc_graph g);

/* The handle's current multi-source BFS launch plan (Algorithm 1's distances
 * are computed in batches of `batch` sources): batch width, 32-bit words per
 * thread and bit-field, distance bit-planes, workgroup shape (0: three
 * fields x 1024 threads, 1: two fields x 512 threads, 2: two fields x 1024
 * threads, 3: two fields x 1024 threads with the third in registers). Any
 * output pointer may be NULL. Host only. */
qc_status qc_graph_bfs_plan(qc_graph g, int32_t *batch, int32_t *words, int32_t *planes,
                            int32_t *shape);

/* Sizes of a handle: any output pointer may be NULL. dmax is -1 until the
 * first qc_distances / qc_potential has run. n_components counts connected
 * components (weakly connected ones for a directed graph). */
qc_status qc_graph_info(qc_graph g, int32_t *n, int64_t *nnz, int32_t *dmax,
                        int32_t *n_components);

/*
 * Hop distances between all pairs of nodes (Section 3.1: the distance the
 * potential is built from, read as the length of a shortest path) and the
 * per-node distance histograms h[i][k] = #{j : d(i,j) = k} that Algorithm 1's
 * sums regroup into.
 *   dist_out  device, int8[n*n] row-major (dist_out[i*n + j] = d(i,j)), 16-byte
 *             aligned (else QC_E_INVAL), or
 *             NULL to keep the matrix in a library-owned device buffer
 *             (its rows start on 128-byte lines, so the search writes whole
 *             lines: the faster form when the caller does not read the
 *             matrix itself).
 *             A non-NULL buffer is also remembered as the resident matrix
 *             and must stay alive while the handle may read it (until the
 *             next qc_distances call or qc_graph_destroy).
 *   dmax_out  host, may be NULL: largest finite distance. The first call on a
 *             handle always waits for the stream (it needs dmax to size the
 *             histograms); later calls return the cached value.
 * Errors: QC_E_OVERFLOW if some finite distance exceeds 126.
 */
qc_status qc_distances(qc_graph g, int8_t *dist_out, int32_t *dmax_out, void *stream);

/*
 * Copy the resident histograms to the caller.
 *   hist_out  device, int32[n * K] row-major, or NULL (then only k_out is set)
 *   k_out     host, receives K (the row length, >= dmax + 1, a multiple of 32)
 * Errors: QC_E_STATE before qc_distances / qc_potential.
 */
qc_status qc_get_histograms(qc_graph g, int32_t *hist_out, int32_t *k_out, void *stream);

/*
 * psi (Eq. 2) and V (Algorithm 1: (1/(2 sigma^2)) sum_j d^2 e^{-d^2/2sigma^2}
 * / sum_j e^{-d^2/2sigma^2}, self term included, unreachable j skipped) of
 * every node for each width in `sigmas`.
 *   sigmas     host, double[n_sigmas], each finite and > 0
 *   n_sigmas   1 <= n_sigmas <= 1024
 *   psi_out    device, float[n_sigmas][n], or NULL
 *   v_out      device, float[n_sigmas][n], or NULL
 *   precision  QC_PREC_* (see above)
 * Runs qc_distances first (with a library-owned matrix) if it has not run.
 * The values are kept resident for qc_ggd_labels; `sigma_index` there indexes
 * this list. Relative error of psi and V vs an FP64 evaluation: <= 1e-6 for
 * FP64ACC and FP32C.
 */
qc_status qc_potential(qc_graph g, const double *sigmas, int32_t n_sigmas,
                       float *psi_out, float *v_out, uint32_t precision, void *stream);

/*
 * Graph Gradient Descent labels for one width of the last qc_potential call
 * (Algorithms 2 and 3): labels_out[i] = id of the local minimum node i's
 * descent ends at. Comparisons whose FP32 gap is within the FP32 error bound
 * are re-decided with the canonical FP64 potential (h_k times exp weights
 * summed in ascending k, no fused multiply-add), so labels do not depend on
 * FP32 rounding.
 *   sigma_index  0 <= sigma_index < n_sigmas of the last qc_potential
 *   tie_mode     QC_TIE_STRICT or QC_TIE_MERGE
 *   labels_out   device, int32[n]
 * Errors: QC_E_STATE before qc_potential, or after a QC_PREC_BF16 potential.
 */
qc_status qc_ggd_labels(qc_graph g, int32_t sigma_index, uint32_t tie_mode,
                        int32_t *labels_out, void *stream);

/*
 * Algorithm 1 on a dense matrix of real-valued distances supplied by the
 * caller: the fully connected workload of the paper's GPU experiment
 * (Section 3.2, Fig. 3), and Section 3.1's distance read literally (an
 * edge's weight for an edge, a cap above every weight for a missing edge)
 * once the caller has written it out densely. Needs no graph handle.
 *   dist      device, float[n_rows * ld] row-major; row i holds d(i, j) for
 *             j < n_cols. Finite entries >= 0 are distances; any other
 *             entry (negative, NaN, infinite) means "no path" and is skipped.
 *             The self distance must be present (normally 0) if it is to be
 *             counted, as in Eq. 2. Rows whose start is 16-byte aligned
 *             (aligned `dist`, ld % 4 == 0) are read with 16-byte loads.
 *   n_rows    0 <= n_rows (0: nothing to do); n_cols >= 0; ld >= n_cols
 *   sigmas    host, double[n_sigmas], each finite and >= 1e-100;
 *             1 <= n_sigmas <= 1024
 *   psi_out   device, double[n_sigmas][n_rows]: psi_i = sum_j e^{-d_ij^2/2 sigma^2}
 *   v_out     device, double[n_sigmas][n_rows]: V_i of Algorithm 1
 * Sums are accumulated in FP64; each exponential is evaluated to about one
 * FP32 ulp, so psi and V are within 1e-6 relative of an FP64 evaluation.
 * A row with no counted entry gives psi = 0 and V = NaN (0/0).
 * The matrix is streamed once per group of up to 8 widths.
 * Errors: QC_E_INVAL for a NULL pointer with n_rows > 0, negative sizes,
 * ld < n_cols, or an invalid sigma; QC_E_DEVICE for a launch failure (or
 * when no gfx950 device is current).
 */
qc_status qc_potential_dense(const float *dist, int64_t n_rows, int64_t n_cols, int64_t ld,
                             const double *sigmas, int32_t n_sigmas, double *psi_out,
                             double *v_out, void *stream);

/*
 * Copy the resident canonical FP64 potential of the last qc_potential call
 * (or batch run) to the caller: the values on which the descent re-decides
 * near ties. V = (1/a) (S1/S2) with a = (2 sigma) sigma, S2 = sum_k h_k w_k,
 * S1 = sum_k (k^2 h_k) w_k, w_k = exp(-k^2/a) from the host C library, both
 * sums in ascending k from +0.0 with every product and sum rounded on its own
 * (Algorithm 1 regrouped by distance value; Eq. 7's approximate form).
 *   v64_out  device, double[n_sigmas][n], node order
 * Errors: QC_E_INVAL for a NULL pointer; QC_E_STATE before qc_potential, or
 * when the last potential was not QC_PREC_FP64ACC (the other precisions keep
 * no FP64 values).
 */
qc_status qc_get_potential64(qc_graph g, double *v64_out, void *stream);

/*
 * Shortest-path lengths of every ordered pair under positive real edge
 * weights (Section 3.1: a path's length is the sum of its edges' weights).
 * A path's length is summed in binary32 from its source outward, every
 * partial sum rounded to nearest, and d(i, j) is the least such sum over the
 * paths from i to j; +infinity when j is unreachable. (Row i holds the sums
 * from i, so under rounding d(i, j) and d(j, i) of an undirected graph can
 * differ in the last bit.)
 *   n, nnz, row_ptr, col_idx  host CSR as for qc_graph_create, canonical
 *             (sorted rows, no duplicates or self-loops; undirected:
 *             symmetric); 1 <= n <= 32768
 *   weights   host, float[nnz], one per CSR entry, each finite and at least
 *             FLT_MIN (normal, > 0); for an undirected graph both entries of
 *             an edge must carry the same weight
 *   flags     0 or QC_GRAPH_DIRECTED (row i lists i's out-neighbours and
 *             d(i, j) follows the edge directions)
 *   dist_out  device, float[n * ld] row-major
 *   ld        row stride in floats, ld >= n
 * One workgroup per source keeps that source's tentative lengths in LDS and
 * relaxes them in rounds from the nodes whose length dropped. The call waits
 * for `stream` and returns when the matrix is written; the caller keeps
 * ownership of every array.
 * Errors: QC_E_INVAL (NULL pointers, sizes, n > 32768, ld < n, a weight that
 * is not a normal positive float, unknown flags), QC_E_NOT_SYMMETRIC (CSR
 * not canonical, or the two weights of an undirected edge differ), QC_E_OOM,
 * QC_E_DEVICE.
 */
qc_status qc_distances_real(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                            const float *weights, uint32_t flags, float *dist_out, int64_t ld,
                            void *stream);

/*
 * Algorithm 4 on a graph with real edge weights, in one call: the distances
 * of qc_distances_real, psi and V of every width by Algorithm 1 on them (as
 * qc_potential_dense: FP64 sums, every exponential to about one FP32 ulp),
 * then the descent along the graph's own edges (Algorithms 2-3, as
 * qc_ggd_labels: FP32 comparisons, near ties re-decided on these FP64 V) and
 * pointer jumping.
 *   n, nnz, row_ptr, col_idx, weights, flags  as qc_distances_real
 *   sigmas, n_sigmas  host, as for qc_potential_dense (each finite and
 *                >= 1e-100, 1..1024 of them)
 *   tie_mode     QC_TIE_STRICT or QC_TIE_MERGE
 *   dist_out     device, float[n*n] row-major, or NULL (the library then
 *                uses a matrix of its own for the call)
 *   psi_out, v_out  device, double[n_sigmas][n], or NULL: the potentials the
 *                labels were decided on
 *   labels_out   device, int32[n_sigmas][n] (sigma-major), required
 * The call waits for `stream`. Errors as qc_distances_real, plus QC_E_INVAL
 * for a bad sigma list, tie mode or a NULL labels_out.
 */
qc_status qc_cluster_real(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                          const float *weights, uint32_t flags, const double *sigmas,
                          int32_t n_sigmas, uint32_t tie_mode, float *dist_out, double *psi_out,
                          double *v_out, int32_t *labels_out, void *stream);

/*
 * Algorithm 4 in one call, on a temporary handle released before the call
 * returns (the call waits for `stream`): hop distances, psi and V (Eq. 2,
 * Algorithm 1) for every width, and the descent's labels (Algorithms 2-3)
 * for every width. A problem that fits QC_NOALLOC_SCRATCH_BYTES runs in the
 * library's fixed device scratch, as qc_cluster_noalloc (no device
 * allocation; such calls on one device take turns), a larger one on
 * buffers allocated for the call.
 *   n, nnz, row_ptr, col_idx  host CSR as for qc_graph_create with flags 0
 *                (canonical and undirected, else QC_E_NOT_SYMMETRIC)
 *   sigmas, n_sigmas          host, as for qc_potential
 *   tie_mode     QC_TIE_STRICT or QC_TIE_MERGE
 *   dist_out     device, int8[n*n] row-major, 16-byte aligned, or NULL (the
 *                library then uses a matrix of its own for the call)
 *   psi_out, v_out  device, float[n_sigmas][n], or NULL
 *   labels_out   device, int32[n_sigmas][n] (sigma-major), required
 * Potentials are accumulated in FP64 (QC_PREC_FP64ACC). On QC_E_OVERFLOW the
 * outputs are undefined. Other errors as the calls it makes.
 */
qc_status qc_cluster(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                     const double *sigmas, int32_t n_sigmas, uint32_t tie_mode, int8_t *dist_out,
                     float *psi_out, float *v_out, int32_t *labels_out, void *stream);

/*
 * qc_cluster without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc). Same arguments, outputs and errors as qc_cluster; the caller
 * still provides the output buffers. Every buffer the call needs besides
 * them (CSR, packed edges, histograms, resident potentials, parents, weight
 * tables, job tables, status words, and the distance matrix when dist_out is
 * NULL) is carved from one fixed array of QC_NOALLOC_SCRATCH_BYTES of device
 * memory, a static device symbol of the library: each device the call runs
 * on holds its own copy until the process ends. The call never calls
 * hipMalloc or hipFree, and no stage timing is recorded for it.
 *   Size limit: the bytes it needs (about 4(n+1) + 4 nnz for the CSR, a
 *   sliced copy of the neighbour lists, 4 n K with K = 128 for histograms,
 *   20 n S for potentials and parents, plus n*n when dist_out is NULL) must
 *   not exceed QC_NOALLOC_SCRATCH_BYTES, else QC_E_TOO_LARGE before any
 *   device work (e.g. n = 19,717 with 88,726 entries and one width fits only
 *   with a caller's dist_out).
 *   Sharing: every call on one device uses that device's array, which keeps
 *   the last call's contents (the call initialises whatever it reads). Calls
 *   in one process on one device are serialised by a host lock, and the call
 *   waits for `stream` before it returns, so the next call finds the array
 *   free; work the caller enqueues on other streams never touches it.
 */
#define QC_NOALLOC_SCRATCH_BYTES (64ll * 1024 * 1024)
qc_status qc_cluster_noalloc(int32_t n, int64_t nnz, const int32_t *row_ptr,
                             const int32_t *col_idx, const double *sigmas, int32_t n_sigmas,
                             uint32_t tie_mode, int8_t *dist_out, float *psi_out, float *v_out,
                             int32_t *labels_out, void *stream);

/* Number of node decisions the last qc_ggd_labels call (or batch run)
 * re-decided in FP64 (waits for the stream). */
qc_status qc_last_recheck_count(qc_graph g, int64_t *count_out);

/* Wait for all work issued on `stream` and return any error the device
 * latched since the last check: QC_E_OVERFLOW for a finite distance above
 * 126, QC_E_DEVICE for a search level beyond the handle's distance planes. */
qc_status qc_graph_sync(qc_graph g, void *stream);

/*
 * Testing hook for out-of-memory handling; not meant for production use.
 * After this call the fail_at-th device allocation the library attempts
 * (counted from 1, in any thread; every buffer a serving request carves from
 * the server's arena counts as one) fails with QC_E_OOM, and later ones
 * succeed again;
 * fail_at = 0 disarms it.
 *   live_out  host, may be NULL: receives the number of device-allocator
 *             blocks the library holds at this moment (allocated and not yet
 *             freed), so a test can check that a failed call released what
 *             it had taken.
 * Process-wide. Errors: QC_E_INVAL for fail_at < 0.
 */
qc_status qc_debug_alloc_fault(int64_t fail_at, int64_t *live_out);

/*
 * Kernel timing, for benchmarks (process-wide). While enabled, the library
 * brackets every kernel launch of each stage with a pair of HIP events
 * recorded on the launch stream (never while that stream is being captured
 * into a HIP graph). qc_timing_read waits for the recorded events and returns
 * the summed device time and the number of launches of one stage.
 *   stage  QC_STAGE_*;  total_ms, launches: host, may be NULL
 */
enum {
    QC_STAGE_BFS = 0,        /* multi-source BFS (distances) */
    QC_STAGE_HIST = 1,       /* distance histograms */
    QC_STAGE_POTENTIAL = 2,  /* psi / V */
    QC_STAGE_GGD = 3,        /* descent parents (with FP64 re-check) */
    QC_STAGE_JUMP = 4,       /* pointer jumping to labels */
    QC_STAGE_DENSE = 5,      /* qc_potential_dense */
    QC_STAGE_SSSP = 6,       /* real-weighted shortest paths (qc_distances_real) */
    QC_N_STAGES = 7
};
qc_status qc_timing_enable(int32_t on);  /* on = 1 also clears earlier records */
qc_status qc_timing_read(int32_t stage, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* QC_H_ */
