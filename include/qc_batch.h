/*
 * qc_batch.h — batched form: many graphs of uneven size and many widths
 * sigma in a handful of grouped launches, optionally replayed as one HIP graph.
 *
 * A batch runs Algorithm 4 of Wang, He & Liu (arXiv 2305.14641) — distances,
 * potentials (Eq. 2, Eq. 7 / Algorithm 1), Graph Gradient Descent labels
 * (Algorithms 2-3) — for every (graph, sigma) pair of the batch. Every result
 * is bitwise identical to what the plain per-graph calls of qc.h return.
 */
#ifndef QC_BATCH_H_
#define QC_BATCH_H_

#include "qc.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qc_batch_s *qc_batch;

enum {
    QC_BATCH_HIPGRAPH = 1u, /* capture the launch sequence once, replay it afterwards */
    QC_BATCH_FP32C = 2u,    /* potentials in compensated FP32 instead of FP64 accumulation */
    QC_BATCH_AUTOTUNE = 4u  /* time the candidate BFS launch shapes of every graph, keep the fastest */
};

/*
 * Plan a batch.
 *   graphs     host, qc_graph[n_graphs] created with qc_graph_create; the batch
 *              uses their resident buffers (distance matrix, histograms,
 *              potentials, weights), so a graph must not be used elsewhere
 *              while a batch run is in flight, and must outlive the batch.
 *              A graph appears at most once. The batch computes each
 *              graph's distances into a matrix the graph's handle owns
 *              (allocated here when the handle has none), never into a
 *              caller's buffer an earlier qc_distances call was given; that
 *              owned matrix becomes the graph's resident matrix.
 *   n_graphs   1 <= n_graphs <= 65536
 *   sigmas     host, double[n_sigmas], each finite and > 0 (1..1024 values),
 *              shared by every graph
 *   tie_mode   QC_TIE_STRICT or QC_TIE_MERGE
 *   flags      any of QC_BATCH_HIPGRAPH, QC_BATCH_FP32C, QC_BATCH_AUTOTUNE
 *              (AUTOTUNE: at set-up every graph's search runs once per
 *              candidate launch shape, timed with events on `stream`; the
 *              fastest becomes the graph's plan, for this batch and for the
 *              graph's own later calls. The outputs do not depend on it.)
 *   stream     stream for any set-up work (graphs whose largest distance is
 *              not yet known run their distances once here, synchronously)
 *   out        host, receives the batch handle
 * Errors: QC_E_INVAL, QC_E_OVERFLOW (from a set-up distance pass), QC_E_OOM.
 */
qc_status qc_batch_create(const qc_graph *graphs, int32_t n_graphs, const double *sigmas,
                          int32_t n_sigmas, uint32_t tie_mode, uint32_t flags, void *stream,
                          qc_batch *out);

/* Node offsets of each graph in the concatenated output layout:
 * offsets host int64[n_graphs + 1]; offsets[n_graphs] = total nodes. */
qc_status qc_batch_node_offsets(qc_batch b, int64_t *offsets);

/*
 * Run the whole path for every (graph, sigma).
 *   psi_out, v_out  device, float[n_sigmas][total_nodes] (graph g's node i of
 *                   sigma s at [s*total + offsets[g] + i]), or NULL
 *   labels_out      device, int32[n_sigmas][total_nodes], same layout, required
 * With QC_BATCH_HIPGRAPH the first run captures the launches on `stream`
 * and every later run with the same output pointers replays that graph.
 */
qc_status qc_batch_run(qc_batch b, float *psi_out, float *v_out, int32_t *labels_out,
                       void *stream);

/*
 * Approximate sigma sweep on the matrix cores: psi (Eq. 2) and V
 * (Algorithm 1, regrouped by distance value) for every (graph, sigma) of
 * the batch from the graphs' resident distance histograms, as the product
 * [weights x bins] . [bins x nodes] with both factors rounded to BF16 and
 * FP32 accumulation (QC_PREC_BF16 of qc_potential, one grouped launch per
 * histogram row length). BF16 keeps 8 significant bits: expect about 1e-3
 * relative error against FP64. Nothing resident changes: these potentials
 * never reach the descent, and a later qc_batch_run is unaffected.
 *   psi_out, v_out  device, float[n_sigmas][total_nodes] (layout as for
 *                   qc_batch_run), both required
 * Errors: QC_E_INVAL for a NULL batch or output; QC_E_DEVICE for a launch
 * failure.
 */
qc_status qc_batch_sweep_bf16(qc_batch b, float *psi_out, float *v_out, void *stream);

/* Number of node decisions re-decided in FP64 by the last run (waits). */
qc_status qc_batch_recheck_count(qc_batch b, int64_t *count_out);

/*
 * Work of the last run's multi-source searches (waits for the device), as
 * counted by the search kernel: edge_visits = sum over the batches of
 * sources of (levels pulled over the whole edge list x edge entries + the
 * sources' row entries pushed at level 1); lds_bytes = the bytes of bit
 * field those visits gathered from LDS (4 or 8 per visit, by batch width).
 * Either pointer (host) may be NULL.
 */
qc_status qc_batch_search_stats(qc_batch b, int64_t *edge_visits, int64_t *lds_bytes);

/* Release the batch (the graphs stay valid). */
qc_status qc_batch_destroy(qc_batch b);

#ifdef __cplusplus
}
#endif

#endif /* QC_BATCH_H_ */
