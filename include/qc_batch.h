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
    QC_BATCH_AUTOTUNE = 4u, /* time the candidate launch shapes (BFS planning policy, histogram pass,
                               pointer jumping, each over the whole batch), keep the fastest */
    QC_BATCH_SERIAL = 8u    /* run every stage in stream order on the caller's stream (see below) */
};

/*
 * Plan a batch.
 *   graphs     host, qc_graph[n_graphs] created with qc_graph_create; the batch
 *              uses their resident buffers (distance matrix, histograms,
 *              potentials, weights), so a graph must not be used elsewhere
 *              while a batch run is in flight, and must outlive the batch.
 *              A graph may be in several batches, used one after another:
 *              a later batch's planning can give it another BFS launch
 *              shape, and a run (of any batch, or a plain call) that finds
 *              the graph's packed edges in another shape's form waits for
 *              the device to drain and uploads them again (host to device,
 *              once per switch).
 *              A graph appears at most once. The batch computes each
 *              graph's distances into a matrix the graph's handle owns
 *              (allocated here when the handle has none), never into a
 *              caller's buffer an earlier qc_distances call was given; that
 *              owned matrix becomes the graph's resident matrix.
 *   n_graphs   1 <= n_graphs <= 65536
 *   sigmas     host, double[n_sigmas], each finite and > 0 (1..1024 values),
 *              shared by every graph
 *   tie_mode   QC_TIE_STRICT or QC_TIE_MERGE
 *   flags      any of QC_BATCH_HIPGRAPH, QC_BATCH_FP32C, QC_BATCH_AUTOTUNE,
 *              QC_BATCH_SERIAL
 *              (AUTOTUNE: at set-up the batch's searches run under each
 *              candidate planning policy, timed with events on `stream`;
 *              the fastest policy's plans stay with the graphs, for this
 *              batch and for their own later calls; then the whole path runs
 *              once and the histogram and pointer-jumping shapes are timed,
 *              see qc_batch_stage_tiles. The outputs do not depend on it.)
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
 * When the searches take more than one launch (graphs of different launch
 * shapes), the launches, largest first, run on `stream` and a stream the
 * batch owns, each on the one with the least estimated search work so far.
 * The distance histograms of the graphs one search launch
 * covers run on another stream the batch owns as soon as that launch has
 * finished, beside the following searches, and the potentials (Eq. 2 /
 * Eq. 7) and Algorithms 2-3 of the graphs of all but the last few launches
 * follow them there, beside those last launches; the last launches' graphs
 * take their histograms and later stages on `stream` once every search is
 * done. `stream` waits for the other streams before the run ends, so the run
 * is ordered on `stream` like any other work (and a captured graph holds
 * every branch). QC_BATCH_SERIAL keeps every launch on `stream`, in stream
 * order (timing one stage at a time). The outputs are the same either way.
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

/*
 * The launch shapes the batch's stages run with (set by QC_BATCH_AUTOTUNE,
 * else the defaults); every output pointer is host memory or NULL:
 *   bfs_widest_out, bfs_front_first_out  the BFS planning policy the graphs'
 *                    plans follow: the widest batch of sources (16, 32 or
 *                    64) and whether the seen-in-registers workgroup shape
 *                    comes first (1) or only the other shapes are used (0);
 *                    default 32 and 1. Each graph's plan: qc_graph_bfs_plan
 *   hist_waves_out   host, int32[3] or NULL: wavefronts per workgroup of the
 *                    histogram pass for row lengths 32, 64 and 128 (0: no
 *                    graph of that row length); each workgroup counts 32 rows
 *   jump_global_out  host or NULL: 1 when the pointer jumping runs in global
 *                    memory, 0 when it runs in LDS
 *   overlap_out      host or NULL: 3 when the histograms and the later
 *                    stages of the first launches' graphs run beside the
 *                    searches (see qc_batch_run), 0 when every stage runs in
 *                    stream order (1: the histograms only, 2: every stage
 *                    after the search beside the searches, measurement
 *                    switches)
 * The autotuner times the whole BFS stage of the batch under each planning
 * policy (widest batch 32, 64 or 16 with the seen-in-registers shape first,
 * and 32 without it); then, after one run of the whole path, it times whole
 * steps with the histogram pass in three shapes (the default wavefront
 * count, half and twice) and with the pointer jumping in LDS and in global
 * memory (in interleaved rounds, each variant's best round). Each default
 * (the first policy, the first variant) stays unless an alternative is
 * faster by 2 % (policies) or 1 % (variants); a later batch of the same
 * class (row length, rows, largest graph) in the process reuses the two
 * stage choices without timing. The outputs do not depend on any of these
 * choices.
 */
qc_status qc_batch_stage_tiles(qc_batch b, int32_t *bfs_widest_out, int32_t *bfs_front_first_out,
                               int32_t *hist_waves_out, int32_t *jump_global_out, int32_t *overlap_out);

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
