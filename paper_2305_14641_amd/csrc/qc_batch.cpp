// Batched form (include/qc_batch.h): grouped launches over many graphs and
// sigmas, optionally captured once into a HIP graph and replayed.
#include <hip/hip_runtime.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <map>
#include <mutex>
#include <set>
#include <tuple>
#include <utility>
#include <vector>

#include "qc_batch.h"
#include "qc_handle.h"

using namespace qc;

struct BfsGroup {
    int bw = 0, nw = 0, planes = 7;
    int shape = 0;
    int bias = 0;              // the row bias its graphs' edges carry (bfs_row_bias)
    BfsJob *d_jobs = nullptr;
    int n_jobs = 0;
    std::vector<int> graphs;   // the batch's graphs whose searches this launch runs
    double rows_bytes = 0.0;   // their distance matrices' bytes (sum of n^2)
    double cost = 0.0;         // their searches' estimated work (batches x levels x edges)
    int stream = 0;            // the search stream it runs on (0: the caller's)
};
struct KGroup {
    int K = 0;
    NodeJob *d_jobs = nullptr;
    int n_jobs = 0;
    int variant = 0;   // histogram workgroup shape (launch_hist)
};
// The stages after the search for a set of the batch's graphs: histograms,
// then (unless `rest` is false) potentials, descent and pointer jumping.
struct Stages {
    int bfs_group = -1;        // the BFS launch whose matrices it reads (-1: all of them;
                               // -2: the last launch's, on the caller's stream, beside the side stream)
    bool rest = true;
    std::vector<KGroup> hist, pot;
    NodeJob *d_ggd_jobs = nullptr;
    int n_ggd_jobs = 0;
    NodeJob *d_jump_jobs = nullptr;
    int n_jump_jobs = 0;
    int max_n = 0;             // largest node count among the graphs
};

struct qc_batch_s {
    std::vector<qc_graph> graphs;
    std::vector<double> sigmas;
    std::vector<int64_t> offsets;  // [n_graphs + 1]
    uint32_t tie = 0;
    uint32_t flags = 0;
    int precision = QC_PREC_FP64ACC;

    GraphDev *d_descs = nullptr;
    // [3] counters of the last run, cleared together at its start: the FP64
    // re-decisions, then the BFS edge visits and LDS bytes gathered
    unsigned long long *d_counters = nullptr;
    unsigned long long *d_recheck = nullptr;  // d_counters
    unsigned long long *d_visits = nullptr;   // d_counters + 1
    std::vector<BfsGroup> bfs;
    // Stage sets in launch order. Serial form: one over every graph, on the
    // caller's stream after the last search. Overlapped forms: one per BFS
    // launch on `side`, started by that launch's event ev_bfs[i] so that it
    // runs beside the next searches (histograms only, followed by one set of
    // the remaining stages over every graph on the caller's stream; or every
    // stage; or, by default, histograms for all but the last k launches, then
    // one set of the remaining stages of those launches' graphs on `side`,
    // and the last k launches' graphs on the caller's stream, bfs_group -2);
    // the caller's stream waits for ev_join.
    int overlap = 0;   // 0 serial, 1 histograms overlapped, 2 every stage overlapped,
                       // 3 histograms and the first launches' later stages overlapped
    std::vector<Stages> stages;
    std::vector<KGroup> pot_all;   // potential jobs of every graph by bin count (BF16 sweep)
    hipStream_t side = nullptr;
    std::vector<hipEvent_t> ev_bfs;
    hipEvent_t ev_join = nullptr;
    // The search launches themselves run on the caller's stream and these
    // (each launch on the one with the least estimated work so far), forked
    // after the counters are cleared (ev_fork) and joined back after the
    // last search (ev_search_join), so that one launch's last workgroups run
    // beside the next launch's first.
    std::vector<hipStream_t> search_side;
    hipEvent_t ev_fork = nullptr;
    std::vector<hipEvent_t> ev_search_join;
    int jump_variant = 0;   // pointer jumping in LDS when it fits (0) or in global memory (1)
    int bfs_policy = 0;     // the BFS planning policy the autotuner kept (0: the planner's)

    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    float *cap_psi = nullptr, *cap_v = nullptr;
    int32_t *cap_labels = nullptr;
    hipStream_t cap_stream = nullptr;
};

namespace {

void free_batch(qc_batch b)
{
    if (!b) return;
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    dfree(b->d_descs);
    dfree(b->d_counters);
    for (auto &g : b->bfs) dfree(g.d_jobs);
    for (auto &c : b->stages) {
        for (auto &g : c.hist) dfree(g.d_jobs);
        for (auto &g : c.pot) dfree(g.d_jobs);
        dfree(c.d_ggd_jobs);
        dfree(c.d_jump_jobs);
    }
    for (auto &g : b->pot_all) dfree(g.d_jobs);
    for (hipEvent_t e : b->ev_bfs) (void)hipEventDestroy(e);
    if (b->ev_join) (void)hipEventDestroy(b->ev_join);
    if (b->side) (void)hipStreamDestroy(b->side);
    for (hipEvent_t e : b->ev_search_join) (void)hipEventDestroy(e);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    for (hipStream_t x : b->search_side) (void)hipStreamDestroy(x);
    delete b;
}

template <class J>
qc_status upload_jobs(J **d, const std::vector<J> &h)
{
    QC_TRY(dalloc(d, h.size()));
    return upload(*d, h);
}

// Order jobs so that consecutive workgroups of one XCD (workgroups are handed
// to the 8 XCDs round-robin by index) stay on the same graph: each graph's
// jobs are dealt to one XCD list (the least loaded), and the lists are then
// interleaved. The graphs' CSR and LDS-resident state thus stay in fewer L2s.
template <class J>
std::vector<J> xcd_order(const std::vector<std::vector<J>> &per_graph, const std::vector<double> &cost)
{
    constexpr int kXcd = 8;
    std::vector<std::vector<J>> lanes(kXcd);
    std::vector<double> load(kXcd, 0.0);
    std::vector<int> order(per_graph.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    for (int gi : order) {
        if (per_graph[gi].empty()) continue;
        // big graphs are spread over every XCD; small ones stay on one
        const double share = cost[gi] / kXcd;
        const bool spread = per_graph[gi].size() >= (size_t)(4 * kXcd);
        if (spread) {
            for (size_t j = 0; j < per_graph[gi].size(); ++j) {
                int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                lanes[x].push_back(per_graph[gi][j]);
                load[x] += cost[gi] / per_graph[gi].size();
            }
        } else {
            int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            for (auto &j : per_graph[gi]) lanes[x].push_back(j);
            load[x] += cost[gi];
        }
        (void)share;
    }
    std::vector<J> out;
    size_t longest = 0;
    for (auto &l : lanes) longest = std::max(longest, l.size());
    for (size_t r = 0; r < longest; ++r)
        for (int x = 0; x < kXcd; ++x)
            if (r < lanes[x].size()) out.push_back(lanes[x][r]);
    return out;
}

// Descent jobs pinned to XCDs: every graph's jobs go to one XCD (largest
// graphs first, each to the least loaded XCD), and the eight lists are padded
// to one length with no-op jobs (first node past the graph's end) before they
// are interleaved. With a multiple of 8 jobs per sigma row of the grid, job k
// runs on XCD k % 8 for every sigma, so an XCD's L2 only ever holds the V
// planes and neighbour lists of its own graphs. Returns an empty list when
// the graphs cannot be balanced this way (too few, or one too large).
std::vector<NodeJob> xcd_pinned_node_jobs(const std::vector<qc_graph> &graphs)
{
    constexpr int kXcd = 8;
    const int ng = (int)graphs.size();
    std::vector<double> cost(ng);
    double total = 0.0, largest = 0.0;
    for (int i = 0; i < ng; ++i) {
        cost[i] = (double)graphs[i]->n + (double)graphs[i]->nnz;
        total += cost[i];
        largest = std::max(largest, cost[i]);
    }
    if (ng < 2 * kXcd || largest > total / kXcd) return {};
    std::vector<int> order(ng);
    for (int i = 0; i < ng; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    std::vector<std::vector<NodeJob>> lanes(kXcd);
    std::vector<double> load(kXcd, 0.0);
    for (int gi : order) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        for (int r = 0; r < graphs[gi]->n; r += kNodesPerJob) lanes[x].push_back(NodeJob{gi, r, 0});
        load[x] += cost[gi];
    }
    size_t longest = 0;
    for (auto &l : lanes) longest = std::max(longest, l.size());
    std::vector<NodeJob> out;
    out.reserve(longest * kXcd);
    for (size_t r = 0; r < longest; ++r)
        for (int x = 0; x < kXcd; ++x)
            out.push_back(r < lanes[x].size() ? lanes[x][r] : NodeJob{0, graphs[0]->n, 0});
    return out;
}

constexpr int kTuneReps = 2;
// Rounds over a stage's variants: each round times every variant once, in
// turn, and a variant's time is its best round, so that a drift over the
// tuning (clocks settling) does not favour the variants timed last.
constexpr int kTuneRounds = 3;
// How much faster than the default an alternative must be to replace it
// (half of it for the stage variants, which take their best of the rounds).
constexpr float kTuneMargin = 0.02f;

// BFS launch groups of the graphs' current plans: jobs grouped by launch
// shape (batch width, words per thread, planes, shape), each group's jobs in
// XCD order. Groups are appended to `out` before their tables are allocated,
// so on failure the caller frees whatever was allocated.
qc_status build_bfs_groups(const std::vector<qc_graph> &graphs, std::vector<BfsGroup> &out)
{
    std::map<std::tuple<int, int, int, int>, std::vector<int>> by_class;
    for (size_t i = 0; i < graphs.size(); ++i) {
        QC_TRY(check_edges(graphs[i]));
        const BfsPlan &p = graphs[i]->plan;
        by_class[std::make_tuple(p.bw, p.nw, p.planes,
                                 p.shape | (graphs[i]->weighted ? kBfsWeighted : 0))]
            .push_back((int)i);
    }
    for (auto &kv : by_class) {
        std::vector<std::vector<BfsJob>> per;
        std::vector<double> cost;
        for (int gi : kv.second) {
            qc_graph g = graphs[gi];
            // last batch first: the source order puts the farthest-reaching
            // sources (the longest searches) at the end
            std::vector<BfsJob> js;
            for (int bidx = g->plan.n_batches - 1; bidx >= 0; --bidx)
                js.push_back(BfsJob{gi, bidx * g->plan.bw,
                                    batch_target(g, bidx * g->plan.bw, g->plan.bw), 0u});
            per.push_back(js);
            cost.push_back((double)g->plan.n_batches * (double)(g->nnz + g->n) * (g->dmax + 2));
        }
        std::vector<BfsJob> jobs = xcd_order(per, cost);
        BfsGroup grp;
        grp.bw = std::get<0>(kv.first);
        grp.nw = std::get<1>(kv.first);
        grp.planes = std::get<2>(kv.first);
        grp.shape = std::get<3>(kv.first);
        const BfsPlan &p0 = graphs[kv.second[0]]->plan;
        grp.bias = bfs_row_bias(p0.bw, p0.nw, p0.shape);
        grp.n_jobs = (int)jobs.size();
        grp.graphs = kv.second;
        for (int gi : kv.second) grp.rows_bytes += (double)graphs[gi]->n * graphs[gi]->n;
        for (double c : cost) grp.cost += c;
        out.push_back(grp);
        QC_TRY(upload_jobs(&out.back().d_jobs, jobs));
    }
    return QC_OK;
}

void free_bfs_groups(std::vector<BfsGroup> &gs)
{
    for (auto &g : gs) dfree(g.d_jobs);
    gs.clear();
}

// One stage set on stream `st`.
qc_status run_stages(qc_batch b, const Stages &c, float *psi_out, float *v_out, int32_t *labels_out,
                     hipStream_t st)
{
    const int S = (int)b->sigmas.size();
    const int64_t total = b->offsets.back();
    for (auto &g : c.hist) {
        StageTimer t(QC_STAGE_HIST, st);
        QC_HIP(launch_hist(g.K, b->d_descs, g.d_jobs, g.n_jobs, st, g.variant));
    }
    if (!c.rest) return QC_OK;
    for (auto &g : c.pot) {
        StageTimer t(QC_STAGE_POTENTIAL, st);
        QC_HIP(launch_potential(b->precision, g.K, b->d_descs, g.d_jobs, g.n_jobs, psi_out, v_out,
                                total, st));
    }
    {
        StageTimer t(QC_STAGE_GGD, st);
        QC_HIP(launch_ggd_parent((int)b->tie, b->d_descs, c.d_ggd_jobs, c.n_ggd_jobs, 0, S, st));
    }
    {
        StageTimer t(QC_STAGE_JUMP, st);
        QC_HIP(launch_pointer_jump(b->d_descs, c.d_jump_jobs, c.n_jump_jobs, 0, S, labels_out, total,
                                   c.max_n, st, b->jump_variant));
    }
    return QC_OK;
}

qc_status enqueue(qc_batch b, float *psi_out, float *v_out, int32_t *labels_out, hipStream_t st)
{
    QC_HIP(launch_fill_u64(b->d_counters, 3, st));
    const size_t k = b->search_side.size() + 1;   // streams the searches take turns on
    if (k > 1) {
        QC_HIP(hipEventRecord(b->ev_fork, st));
        for (hipStream_t x : b->search_side) QC_HIP(hipStreamWaitEvent(x, b->ev_fork, 0));
    }
    for (size_t i = 0; i < b->bfs.size(); ++i) {
        const BfsGroup &g = b->bfs[i];
        hipStream_t bs = g.stream ? b->search_side[g.stream - 1] : st;
        {
            StageTimer t(QC_STAGE_BFS, bs);
            QC_HIP(launch_bfs(g.bw, g.nw, g.planes, g.shape, b->d_descs, g.d_jobs, g.n_jobs, bs));
        }
        if (b->overlap) QC_HIP(hipEventRecord(b->ev_bfs[i], bs));
    }
    for (size_t j = 0; j + 1 < k; ++j) {
        QC_HIP(hipEventRecord(b->ev_search_join[j], b->search_side[j]));
        QC_HIP(hipStreamWaitEvent(st, b->ev_search_join[j], 0));
    }
    bool forked = false;
    for (const Stages &c : b->stages) {
        if (c.bfs_group == -2) {
            // the last launch's graphs: on the caller's stream, beside the side stream
            QC_TRY(run_stages(b, c, psi_out, v_out, labels_out, st));
        } else if (c.bfs_group < 0) {
            // after every search: on the caller's stream, joined with the side stream first
            if (forked) {
                QC_HIP(hipEventRecord(b->ev_join, b->side));
                QC_HIP(hipStreamWaitEvent(st, b->ev_join, 0));
                forked = false;
            }
            QC_TRY(run_stages(b, c, psi_out, v_out, labels_out, st));
        } else {
            QC_HIP(hipStreamWaitEvent(b->side, b->ev_bfs[c.bfs_group], 0));
            forked = true;
            QC_TRY(run_stages(b, c, psi_out, v_out, labels_out, b->side));
        }
    }
    if (forked) {
        QC_HIP(hipEventRecord(b->ev_join, b->side));
        QC_HIP(hipStreamWaitEvent(st, b->ev_join, 0));
    }
    return QC_OK;
}

int batch_max_n(qc_batch b)
{
    int m = 0;
    for (qc_graph g : b->graphs) m = std::max(m, (int)g->n);
    return m;
}

int log2_bucket(double x)
{
    int k = 0;
    while (x >= 2.0 && k < 62) {
        x *= 0.5;
        ++k;
    }
    return k;
}

// Mean time of kTuneReps launches of `launch` (after one untimed), with
// HIP events on st; a negative value on failure.
template <class F>
float time_launches(F launch, hipStream_t st)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1.0f;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1.0f;
    }
    float ms = -1.0f;
    hipError_t e = launch();
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int r = 0; r < kTuneReps && e == hipSuccess; ++r) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) ms /= kTuneReps;
    else ms = -1.0f;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms;
}

// The stage tiles the autotuner chose, process-wide, by workload class:
// (stage, overlapped form, log2 of the batch's nodes, log2 of the largest
// graph); a batch of the same class reuses the choice.
std::mutex g_tiles_mu;
std::map<std::tuple<int, int, int, int>, int> g_tiles;

// The autotuner's second part: after one eager run of the whole path (so the
// matrices, histograms and parents are the batch's own and re-running a
// stage rewrites identical values), time whole steps with the histogram pass
// in each of its three workgroup shapes, then with pointer jumping in LDS and
// in global memory (interleaved rounds, each variant's best round); keep the
// fastest, and remember it for the class. Whole
// steps, because in the overlapped forms a stage's best shape is the one
// that shares the GPU best with the searches beside it.
qc_status autotune_stages(qc_batch b, hipStream_t st)
{
    StageTimingOff quiet;
    const int S = (int)b->sigmas.size();
    const int64_t total = b->offsets.back();
    const int max_n = batch_max_n(b);
    int32_t *labels = nullptr;
    QC_TRY(dalloc(&labels, (size_t)S * total));
    qc_status s = enqueue(b, nullptr, nullptr, labels, st);
    auto step = [&] {
        const qc_status r = enqueue(b, nullptr, nullptr, labels, st);
        return r == QC_OK ? hipSuccess : hipErrorUnknown;
    };
    auto set_hist = [&](int v) {
        for (auto &c : b->stages)
            for (auto &g : c.hist) g.variant = v;
    };
    auto tune = [&](int stage, int n_variants, const std::function<void(int)> &apply) {
        const auto key = std::make_tuple(stage, b->overlap, log2_bucket((double)total), log2_bucket(max_n));
        {
            std::lock_guard<std::mutex> lk(g_tiles_mu);
            auto it = g_tiles.find(key);
            if (it != g_tiles.end()) {
                apply(it->second);
                return;
            }
        }
        std::vector<float> best((size_t)n_variants, 1e30f);
        for (int r = 0; r < kTuneRounds && s == QC_OK; ++r)
            for (int v = 0; v < n_variants && s == QC_OK; ++v) {
                apply(v);
                const float ms = time_launches(step, st);
                if (ms < 0.0f) s = QC_E_DEVICE;
                else best[(size_t)v] = std::min(best[(size_t)v], ms);
            }
        // the default (variant 0) stays unless another is clearly faster
        int chosen = (int)(std::min_element(best.begin(), best.end()) - best.begin());
        if (chosen != 0 && best[(size_t)chosen] > best[0] * (1.0f - kTuneMargin / 2)) chosen = 0;
        apply(chosen);
        std::lock_guard<std::mutex> lk(g_tiles_mu);
        if (s == QC_OK) g_tiles[key] = chosen;
    };
    if (s == QC_OK) tune(0, 3, set_hist);
    if (s == QC_OK && max_n <= 40704) tune(1, 2, [&](int v) { b->jump_variant = v; });
    (void)hipStreamSynchronize(st);
    dfree(labels);
    return s;
}

// The BFS part of the autotuner, for the whole batch at once: the planner's
// rule under a few policies (widest batch 32, 64 or 16 sources with the
// seen-in-registers shape first; 32 without it) gives every graph a plan;
// each policy's launch groups run the whole BFS stage of the batch, one
// untimed and kTuneReps timed times (all in the plain edge order, so that no
// policy starts with an order chosen for it), and the fastest policy's
// plans stay with the graphs (with their edge order). Timing the stage as
// the batch runs it counts what timing one graph alone misses: how the
// graphs' jobs share the GPU.
struct BfsPolicy { int max_bw; bool front_first; };
constexpr BfsPolicy kBfsPolicies[] = {{kBfsFullWidth, true}, {64, true}, {16, true},
                                      {kBfsFullWidth, false}};

qc_status autotune_bfs_batch(qc_batch b, hipStream_t st, int *chosen)
{
    *chosen = 0;
    for (qc_graph g : b->graphs) QC_TRY(plain_edges(g));
    float best = 1e30f;
    qc_status s = QC_OK;
    int pi = 0;
    for (const BfsPolicy &pol : kBfsPolicies) {
        for (qc_graph g : b->graphs) {
            if (s == QC_OK) s = set_plan(g, plan_bfs_policy(g->n_bfs, g->dmax_bfs, pol.max_bw, pol.front_first), false);
        }
        std::vector<BfsGroup> groups;
        if (s == QC_OK) s = build_bfs_groups(b->graphs, groups);
        if (s == QC_OK) {
            const float ms = time_launches(
                [&] {
                    hipError_t e = hipSuccess;
                    for (auto &g : groups) {
                        e = launch_bfs(g.bw, g.nw, g.planes, g.shape, b->d_descs, g.d_jobs, g.n_jobs, st);
                        if (e != hipSuccess) break;
                    }
                    return e;
                },
                st);
            // the planner's policy (the first) stays unless another is
            // clearly faster: the policies' times are close on graphs the
            // planner was tuned on, and a close call is noise
            if (ms < 0.0f) s = QC_E_DEVICE;
            else if (pi == 0 || ms < best * (pi > 0 && *chosen == 0 ? 1.0f - kTuneMargin : 1.0f)) {
                best = ms;
                *chosen = pi;
            }
        }
        free_bfs_groups(groups);
        if (s != QC_OK) break;
        ++pi;
    }
    // the chosen plans, now with their edge order (even after a failure the
    // graphs keep valid plans)
    const BfsPolicy &pol = kBfsPolicies[*chosen];
    for (qc_graph g : b->graphs) {
        const qc_status r = set_plan(g, plan_bfs_policy(g->n_bfs, g->dmax_bfs, pol.max_bw, pol.front_first), true);
        if (s == QC_OK) s = r;
    }
    return s;
}

}  // namespace

extern "C" {

qc_status qc_batch_create(const qc_graph *graphs, int32_t n_graphs, const double *sigmas,
                          int32_t n_sigmas, uint32_t tie_mode, uint32_t flags, void *stream,
                          qc_batch *out)
{
    if (!graphs || !out || n_graphs < 1 || n_graphs > 65536) return QC_E_INVAL;
    if (tie_mode > QC_TIE_MERGE) return QC_E_INVAL;
    if (flags & ~(uint32_t)(QC_BATCH_HIPGRAPH | QC_BATCH_FP32C | QC_BATCH_AUTOTUNE | QC_BATCH_SERIAL))
        return QC_E_INVAL;
    QC_TRY(validate_sigmas(sigmas, n_sigmas));
    std::set<qc_graph> seen;
    for (int i = 0; i < n_graphs; ++i) {
        if (!graphs[i] || !seen.insert(graphs[i]).second) return QC_E_INVAL;
    }
    hipStream_t st = as_stream(stream);

    qc_batch b = new qc_batch_s();
    b->graphs.assign(graphs, graphs + n_graphs);
    b->sigmas.assign(sigmas, sigmas + n_sigmas);
    b->tie = tie_mode;
    b->flags = flags;
    b->precision = (flags & QC_BATCH_FP32C) ? QC_PREC_FP32C : QC_PREC_FP64ACC;
    auto fail = [&](qc_status s) { free_batch(b); return s; };

    // Per-graph set-up: resident matrix, largest distance, sigma tables.
    b->offsets.assign(n_graphs + 1, 0);
    for (int i = 0; i < n_graphs; ++i) {
        qc_graph g = graphs[i];
        // the batch writes distances only into a matrix the handle owns,
        // never into a caller's buffer an earlier qc_distances was given
        if (!g->d_dist_owned) {
            qc_status s = galloc(g, &g->d_dist_owned, (size_t)(g->n * owned_ld(g->n) + 16));
            if (s) return fail(s);
        }
        g->d_dist = g->d_dist_owned;
        g->d_ld = owned_ld(g->n);
        if (g->dmax < 0) {
            qc_status s = run_distances(g, st);
            if (s) return fail(s);
        }
        // the graph's potentials are the batch's once a run has computed them
        g->have_pot = false;
        qc_status s = load_sigmas(g, sigmas, n_sigmas, st);
        if (s) return fail(s);
        g->pot_precision = (uint32_t)b->precision;
        b->offsets[i + 1] = b->offsets[i] + g->n;
    }
    if (hipStreamSynchronize(st) != hipSuccess) return fail(QC_E_DEVICE);

    qc_status s;
    if ((s = dalloc(&b->d_counters, 3)) || (s = dalloc(&b->d_descs, (size_t)n_graphs))) return fail(s);
    b->d_recheck = b->d_counters;
    b->d_visits = b->d_counters + 1;
    std::vector<GraphDev> descs(n_graphs);
    for (int i = 0; i < n_graphs; ++i) {
        descs[i] = graphs[i]->desc();
        descs[i].recheck = b->d_recheck;
        descs[i].visits = b->d_visits;
    }
    if ((s = upload(b->d_descs, descs))) return fail(s);

    // BFS jobs grouped by launch shape, in XCD order (with AUTOTUNE, of the
    // policy that ran the batch's searches fastest)
    if ((flags & QC_BATCH_AUTOTUNE) && (s = autotune_bfs_batch(b, st, &b->bfs_policy)))
        return fail(s);
    if ((s = build_bfs_groups(b->graphs, b->bfs))) return fail(s);
    // When the searches take more than one launch, the histograms of each
    // launch's graphs run beside the later searches, and the potentials,
    // descent and jumping of the graphs of all but the last k launches run
    // beside those k launches (the tail, mode 3); the last launches' graphs
    // take theirs on the caller's stream once the searches are done.
    // QC_BATCH_OVERLAP=1 keeps every stage after the histograms for the end,
    // 2 runs every stage after the search per search launch, 0 none
    // (switches for measurements and tests). Every stage per launch
    // measured slower: the descent and jumping of one launch's few graphs
    // are latency-bound chains that, queued behind one another on the side
    // stream, outlast the searches.
    {
        const char *ov = getenv("QC_BATCH_OVERLAP");
        const int want = (ov && atoi(ov) >= 0 && atoi(ov) <= 3) ? atoi(ov) : 3;
        b->overlap = (b->bfs.size() > 1 && !(flags & QC_BATCH_SERIAL)) ? want : 0;
    }
    if (b->overlap) {
        // the launch with the fewest matrix bytes last: its stages are the
        // only ones no search runs beside
        std::stable_sort(b->bfs.begin(), b->bfs.end(), [](const BfsGroup &x, const BfsGroup &y) {
            return x.rows_bytes > y.rows_bytes;
        });

        if (hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) != hipSuccess) {
            b->side = nullptr;
            return fail(QC_E_DEVICE);
        }
        for (size_t i = 0; i <= b->bfs.size(); ++i) {
            hipEvent_t e = nullptr;
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return fail(QC_E_DEVICE);
            if (i < b->bfs.size()) b->ev_bfs.push_back(e);
            else b->ev_join = e;
        }
        // the searches on two streams (QC_BATCH_BFS_STREAMS=1..4, a switch
        // for measurements and tests)
        const char *ks = getenv("QC_BATCH_BFS_STREAMS");
        int k = (ks && atoi(ks) >= 1 && atoi(ks) <= 4) ? atoi(ks) : 2;
        k = std::min<int>(k, (int)b->bfs.size());
        if (k > 1 && hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess) {
            b->ev_fork = nullptr;
            return fail(QC_E_DEVICE);
        }
        for (int j = 1; j < k; ++j) {
            hipStream_t x = nullptr;
            if (hipStreamCreateWithFlags(&x, hipStreamNonBlocking) != hipSuccess) return fail(QC_E_DEVICE);
            b->search_side.push_back(x);
            hipEvent_t e = nullptr;
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return fail(QC_E_DEVICE);
            b->ev_search_join.push_back(e);
        }
        // each launch, in order, on the search stream with the least
        // estimated work so far (QC_BATCH_BFS_ASSIGN=turns: in turn, a
        // switch for measurements)
        const char *as = getenv("QC_BATCH_BFS_ASSIGN");
        const bool turns = as && strcmp(as, "turns") == 0;
        std::vector<double> load((size_t)k, 0.0);
        for (size_t i = 0; i < b->bfs.size(); ++i) {
            BfsGroup &g = b->bfs[i];
            g.stream = turns ? (int)(i % k) : (int)(std::min_element(load.begin(), load.end()) - load.begin());
            load[(size_t)g.stream] += g.cost;
        }
    }
    // One stage set over graphs `gis`: histogram and potential jobs grouped
    // by bin count, descent jobs (pinned to XCDs when the graphs allow it),
    // one jumping job per graph. Appended before its tables are allocated,
    // so a failure leaves nothing unowned.
    auto add_stages = [&](const std::vector<int> &gis, int bfs_group, bool with_hist, bool rest) -> qc_status {
        b->stages.emplace_back();
        Stages &c = b->stages.back();
        c.bfs_group = bfs_group;
        c.rest = rest;
        std::map<int, std::vector<int>> by_k;
        for (int gi : gis) {
            by_k[graphs[gi]->K].push_back(gi);
            c.max_n = std::max(c.max_n, (int)graphs[gi]->n);
        }
        for (auto &kv : by_k) {
            const int K = kv.first;
            std::vector<NodeJob> hj, pj;
            for (int gi : kv.second) {
                const int n = graphs[gi]->n;
                if (with_hist)
                    for (int r = 0; r < n; r += hist_rows_per_job(K)) hj.push_back(NodeJob{gi, r, 0});
                if (rest)
                    for (int r = 0; r < n; r += kNodesPerJob) pj.push_back(NodeJob{gi, r, b->offsets[gi]});
            }
            if (with_hist) {
                KGroup h;
                h.K = K;
                h.n_jobs = (int)hj.size();
                h.variant = 0;
                c.hist.push_back(h);
                QC_TRY(upload_jobs(&c.hist.back().d_jobs, hj));
            }
            if (rest) {
                KGroup pg;
                pg.K = K;
                pg.n_jobs = (int)pj.size();
                c.pot.push_back(pg);
                QC_TRY(upload_jobs(&c.pot.back().d_jobs, pj));
            }
        }
        if (!rest) return QC_OK;
        std::vector<qc_graph> gv;
        for (int gi : gis) gv.push_back(graphs[gi]);
        std::vector<NodeJob> gj = xcd_pinned_node_jobs(gv), jj;
        // pinned jobs index gv; the kernels index the batch's descriptors
        for (auto &j : gj) j.g = gis[j.g];
        const bool pinned = !gj.empty();
        for (int gi : gis) {
            if (!pinned)
                for (int r = 0; r < graphs[gi]->n; r += kNodesPerJob) gj.push_back(NodeJob{gi, r, 0});
            jj.push_back(NodeJob{gi, 0, b->offsets[gi]});
        }
        c.n_ggd_jobs = (int)gj.size();
        c.n_jump_jobs = (int)jj.size();
        QC_TRY(upload_jobs(&c.d_ggd_jobs, gj));
        return upload_jobs(&c.d_jump_jobs, jj);
    };
    std::vector<int> all(n_graphs);
    for (int i = 0; i < n_graphs; ++i) all[i] = i;
    {
        std::map<int, std::vector<int>> by_k;
        for (int gi : all) by_k[graphs[gi]->K].push_back(gi);
        for (auto &kv : by_k) {
            std::vector<NodeJob> pj;
            for (int gi : kv.second)
                for (int r = 0; r < graphs[gi]->n; r += kNodesPerJob) pj.push_back(NodeJob{gi, r, b->offsets[gi]});
            KGroup pg;
            pg.K = kv.first;
            pg.n_jobs = (int)pj.size();
            b->pot_all.push_back(pg);
            if ((s = upload_jobs(&b->pot_all.back().d_jobs, pj))) return fail(s);
        }
    }
    if (b->overlap == 0) {
        if ((s = add_stages(all, -1, true, true))) return fail(s);
    } else {
        const int G = (int)b->bfs.size();
        // mode 3: the later stages of the graphs of the first G - k launches
        // run beside the last k launches, the fewest that hold a tenth of
        // the batch's matrix bytes (the launches go largest first), so that
        // their searches last about as long as those stages
        // (QC_BATCH_TAIL_LAUNCHES=k sets k, a switch for measurements and tests)
        int k = 1;
        {
            double all_bytes = 0.0, last_bytes = 0.0;
            for (const BfsGroup &g : b->bfs) all_bytes += g.rows_bytes;
            while (k < G - 1 && (last_bytes += b->bfs[G - k].rows_bytes) < 0.1 * all_bytes) ++k;
        }
        if (const char *tl = getenv("QC_BATCH_TAIL_LAUNCHES")) k = atoi(tl);
        k = std::max(1, std::min(k, G - 1));
        for (int i = 0; i < G; ++i)
            if (b->overlap != 3 || i < G - k)
                if ((s = add_stages(b->bfs[i].graphs, i, true, b->overlap == 2))) return fail(s);
        if (b->overlap == 1 && (s = add_stages(all, -1, false, true))) return fail(s);
        if (b->overlap == 3) {
            std::vector<int> early, late;
            for (int i = 0; i < G; ++i) {
                std::vector<int> &to = (i < G - k) ? early : late;
                to.insert(to.end(), b->bfs[i].graphs.begin(), b->bfs[i].graphs.end());
            }
            if ((s = add_stages(early, G - k - 1, false, true))) return fail(s);
            if ((s = add_stages(late, -2, true, true))) return fail(s);
        }
    }
    // Each graph's own descriptor now reflects the batch's sigma list.
    for (int i = 0; i < n_graphs; ++i)
        if ((s = push_desc(graphs[i], st))) return fail(s);
    if (hipStreamSynchronize(st) != hipSuccess) return fail(QC_E_DEVICE);
    if (flags & QC_BATCH_AUTOTUNE) {
        if ((s = autotune_stages(b, st))) return fail(s);
    } else {
        // QC_HIST_VARIANT / QC_JUMP_VARIANT (switches for measurements and
        // tests): a fixed histogram shape (0-2) and jumping variant (0-1)
        const char *hv = getenv("QC_HIST_VARIANT"), *jv = getenv("QC_JUMP_VARIANT");
        if (hv && atoi(hv) >= 0 && atoi(hv) <= 2)
            for (auto &c : b->stages)
                for (auto &g : c.hist) g.variant = atoi(hv);
        if (jv && (atoi(jv) == 0 || atoi(jv) == 1)) b->jump_variant = atoi(jv);
    }
    *out = b;
    return QC_OK;
}

qc_status qc_batch_stage_tiles(qc_batch b, int32_t *bfs_widest_out, int32_t *bfs_front_first_out,
                               int32_t *hist_waves_out, int32_t *jump_global_out, int32_t *overlap_out)
{
    if (!b) return QC_E_INVAL;
    if (bfs_widest_out) *bfs_widest_out = kBfsPolicies[b->bfs_policy].max_bw;
    if (bfs_front_first_out) *bfs_front_first_out = kBfsPolicies[b->bfs_policy].front_first ? 1 : 0;
    if (hist_waves_out) {
        for (int i = 0; i < 3; ++i) hist_waves_out[i] = 0;
        for (auto &c : b->stages)
            for (auto &g : c.hist) {
                const int slot = g.K == 32 ? 0 : g.K == 64 ? 1 : 2;
                hist_waves_out[slot] = hist_waves(g.K, g.variant);
            }
    }
    if (jump_global_out) *jump_global_out = (b->jump_variant == 1 || batch_max_n(b) > 40704) ? 1 : 0;
    if (overlap_out) *overlap_out = b->overlap;
    return QC_OK;
}

qc_status qc_batch_node_offsets(qc_batch b, int64_t *offsets)
{
    if (!b || !offsets) return QC_E_INVAL;
    std::copy(b->offsets.begin(), b->offsets.end(), offsets);
    return QC_OK;
}

qc_status qc_batch_run(qc_batch b, float *psi_out, float *v_out, int32_t *labels_out, void *stream)
{
    if (!b || !labels_out) return QC_E_INVAL;
    hipStream_t st = as_stream(stream);
    // a graph that is also in another batch, or searched alone since, may
    // hold its edges in the form another launch shape reads
    for (const BfsGroup &grp : b->bfs)
        for (int gi : grp.graphs) QC_TRY(ensure_edges(b->graphs[gi], grp.bias));
    const bool use_graph = (b->flags & QC_BATCH_HIPGRAPH) && st != nullptr;
    if (!use_graph) {
        QC_TRY(enqueue(b, psi_out, v_out, labels_out, st));
        for (qc_graph g : b->graphs) g->have_pot = true;
        return QC_OK;
    }

    const bool same = b->exec && b->cap_psi == psi_out && b->cap_v == v_out &&
                      b->cap_labels == labels_out && b->cap_stream == st;
    if (!same) {
        if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
        if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
        QC_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        qc_status s = enqueue(b, psi_out, v_out, labels_out, st);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(st, &graph);
        if (s != QC_OK) { if (graph) (void)hipGraphDestroy(graph); return s; }
        QC_HIP(e);
        b->graph = graph;
        QC_HIP(hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0));
        b->cap_psi = psi_out;
        b->cap_v = v_out;
        b->cap_labels = labels_out;
        b->cap_stream = st;
    }
    QC_HIP(hipGraphLaunch(b->exec, st));
    for (qc_graph g : b->graphs) g->have_pot = true;
    return QC_OK;
}

qc_status qc_batch_sweep_bf16(qc_batch b, float *psi_out, float *v_out, void *stream)
{
    if (!b || !psi_out || !v_out) return QC_E_INVAL;
    hipStream_t st = as_stream(stream);
    const int64_t total = b->offsets.back();
    for (auto &g : b->pot_all) {
        StageTimer t(QC_STAGE_POTENTIAL, st);
        QC_HIP(launch_potential(QC_PREC_BF16, g.K, b->d_descs, g.d_jobs, g.n_jobs, psi_out, v_out,
                                total, st));
    }
    return QC_OK;
}

qc_status qc_batch_recheck_count(qc_batch b, int64_t *count_out)
{
    if (!b || !count_out) return QC_E_INVAL;
    unsigned long long c = 0;
    QC_HIP(hipDeviceSynchronize());
    QC_HIP(hipMemcpy(&c, b->d_recheck, sizeof c, hipMemcpyDeviceToHost));
    *count_out = (int64_t)c;
    return QC_OK;
}

qc_status qc_batch_search_stats(qc_batch b, int64_t *edge_visits, int64_t *lds_bytes)
{
    if (!b) return QC_E_INVAL;
    unsigned long long c[2] = {0, 0};
    QC_HIP(hipDeviceSynchronize());
    QC_HIP(hipMemcpy(c, b->d_visits, sizeof c, hipMemcpyDeviceToHost));
    if (edge_visits) *edge_visits = (int64_t)c[0];
    if (lds_bytes) *lds_bytes = (int64_t)c[1];
    return QC_OK;
}

qc_status qc_batch_destroy(qc_batch b)
{
    if (!b) return QC_E_INVAL;
    free_batch(b);
    return QC_OK;
}

}  // extern "C"
