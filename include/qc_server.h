/*
 * qc_server.h — serving form: a request loop that runs Algorithm 4 of
 * Wang, He & Liu (arXiv 2305.14641) — distances, potentials (Eq. 2, Eq. 7 /
 * Algorithm 1), Graph Gradient Descent labels (Algorithms 2-3) — for graph
 * clustering requests of mixed sizes.
 *
 * Continuous batching: up to `max_slots` requests are on the GPU at once,
 * each on its own stream, and a queued request is admitted as soon as a slot
 * is free and its device-memory footprint fits what is left of the budget
 * (oldest first; see max_bypass for passing a request that does not fit).
 * Device memory is one arena reserved when the server is created and
 * sub-allocated per request, so serving itself never calls the device
 * allocator. A request's results are bitwise identical to the plain
 * per-graph calls of qc.h.
 *
 * Robustness: a request that cannot be admitted before its queue deadline
 * completes with QC_E_TIMEOUT, a queued request can be withdrawn
 * (qc_server_cancel), and a request that fails (e.g. QC_E_OOM) releases its
 * arena region and slot, so later requests are served normally. A request
 * that has started is never interrupted: every kernel of the path ends on
 * its own (a search ends after at most 127 levels).
 */
#ifndef QC_SERVER_H_
#define QC_SERVER_H_

#include "qc.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qc_server_s *qc_server;

typedef struct {
    int32_t max_slots;          /* requests on the GPU at once, 1..64 */
    int64_t hbm_budget_bytes;   /* device arena for request state, > 0 */
    uint32_t tie_mode;          /* QC_TIE_STRICT or QC_TIE_MERGE */
    int32_t want_potentials;    /* 1: also keep psi and V for qc_server_wait */
    double queue_timeout_s;     /* > 0: a request still queued this many seconds after its
                                   submission completes with QC_E_TIMEOUT without running;
                                   0: no deadline (finite, >= 0) */
    int32_t max_bypass;         /* 0: strict first-in first-out admission. k > 0: when the
                                   oldest queued request does not fit, younger ones that fit
                                   may be admitted before it, but each request can be passed
                                   at most k times; after that nothing is admitted before it
                                   (0..1000000) */
} qc_server_opts;

typedef struct {
    int64_t id;
    double t_submit, t_admit, t_done;  /* seconds on the server's monotonic clock */
    int64_t footprint_bytes;           /* arena bytes the request reserved */
    int32_t n, n_sigmas, dmax;
    int32_t slot;                      /* slot (stream) that ran it */
    qc_status status;                  /* QC_OK or the error of its calls */
} qc_request_info;

/* Device bytes one request of n nodes, nnz CSR entries and n_sigmas widths
 * reserves (CSR, packed edges, N*N int8 distances, histograms, psi / V /
 * FP64 V / parents / labels per sigma, tables). Pure host computation;
 * returns -1 for out-of-range arguments. */
int64_t qc_request_footprint(int32_t n, int64_t nnz, int32_t n_sigmas);

/* Start a server (reserves the arena, creates the slot streams and threads).
 * Errors: QC_E_INVAL (options), QC_E_DEVICE, QC_E_OOM (arena). */
qc_status qc_server_create(const qc_server_opts *opts, qc_server *out);

/*
 * Queue one request; returns at once with its id.
 *   row_ptr, col_idx  host CSR as for qc_graph_create (validated here; the
 *                     server copies it)
 *   sigmas            host, double[n_sigmas] (1..1024, finite, > 0)
 * Errors: QC_E_INVAL / QC_E_NOT_SYMMETRIC (validation), QC_E_BUSY (the
 * request's footprint exceeds the whole budget, so it can never be admitted).
 */
qc_status qc_server_submit(qc_server s, int32_t n, int64_t nnz, const int32_t *row_ptr,
                           const int32_t *col_idx, const double *sigmas, int32_t n_sigmas,
                           int64_t *id_out);

/* Non-blocking: *done_out = 1 once the request has finished. */
qc_status qc_server_poll(qc_server s, int64_t id, int32_t *done_out);

/*
 * Wait for a request and collect its results (then the id is released).
 *   labels_out  host, int32[n_sigmas][n], or NULL
 *   psi_out, v_out  host, float[n_sigmas][n], or NULL (need want_potentials)
 *   info        host, or NULL
 * Returns the request's own status (e.g. QC_E_OVERFLOW) or QC_E_INVAL for an
 * unknown id.
 */
qc_status qc_server_wait(qc_server s, int64_t id, int32_t *labels_out, float *psi_out,
                         float *v_out, qc_request_info *info);

/*
 * Withdraw a request that is still queued: it completes with QC_E_CANCELLED
 * (collect it with qc_server_wait as any other). Returns QC_OK when it was
 * withdrawn, QC_E_BUSY when it has already been admitted (it then runs to
 * completion), QC_E_STATE when it has already completed, QC_E_INVAL for an
 * unknown id.
 */
qc_status qc_server_cancel(qc_server s, int64_t id);

/* Largest arena bytes and number of requests in flight at the same time so far. */
qc_status qc_server_stats(qc_server s, int64_t *peak_bytes_out, int32_t *peak_requests_out);

/* Finish every queued request, stop the threads, release the arena. */
qc_status qc_server_destroy(qc_server s);

#ifdef __cplusplus
}
#endif

#endif /* QC_SERVER_H_ */
