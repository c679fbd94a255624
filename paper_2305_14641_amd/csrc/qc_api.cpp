// C ABI of the library (include/qc.h): graph handles, resident device state,
// and the launch sequence of each call.
#include <hip/hip_runtime.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <algorithm>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "qc.h"
#include "qc_host.h"
#include "qc_internal.h"
#include "qc_handle.h"

using namespace qc;

namespace qc {

qc_status from_hip(hipError_t e)
{
    if (e == hipSuccess) return QC_OK;
    if (e == hipErrorOutOfMemory) return QC_E_OOM;
    return QC_E_DEVICE;
}

// Out-of-memory injection: allocations left before the one that fails
// (0: disarmed), and the device allocator blocks currently held.
static std::atomic<int64_t> g_fault_countdown{0};
static std::atomic<int64_t> g_live_allocs{0};

bool alloc_fault_now()
{
    int64_t c = g_fault_countdown.load(std::memory_order_relaxed);
    while (c > 0) {
        if (g_fault_countdown.compare_exchange_weak(c, c - 1, std::memory_order_relaxed))
            return c == 1;
    }
    return false;
}

void note_device_alloc(int delta) { g_live_allocs.fetch_add(delta, std::memory_order_relaxed); }

qc_status check_device(int *dev_out)
{
    // The architecture of each device is looked up once (device properties
    // are slow to query) and cached; 0 unknown, 1 gfx950, 2 other.
    constexpr int kMaxDevices = 64;
    static std::atomic<int> arch[kMaxDevices];
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
        (void)hipGetLastError();
        return QC_E_DEVICE;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return QC_E_DEVICE;
    int a = arch[dev].load(std::memory_order_relaxed);
    if (a == 0) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return QC_E_DEVICE;
        a = strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : 2;
        arch[dev].store(a, std::memory_order_relaxed);
    }
    if (a != 1) return QC_E_DEVICE;
    *dev_out = dev;
    return QC_OK;
}

qc_status upload_group(qc_graph g, std::vector<HostSpan> spans)
{
    // large arrays go straight (a staging copy would only add host work);
    // the small ones are what costs a copy call each
    constexpr size_t kLarge = 64 * 1024;
    for (const HostSpan &x : spans)
        if (x.bytes >= kLarge) QC_HIP(hipMemcpy(x.dst, x.src, x.bytes, hipMemcpyHostToDevice));
    spans.erase(std::remove_if(spans.begin(), spans.end(),
                               [](const HostSpan &x) { return x.bytes == 0 || x.bytes >= kLarge; }),
                spans.end());
    std::sort(spans.begin(), spans.end(),
              [](const HostSpan &a, const HostSpan &b) { return (char *)a.dst < (char *)b.dst; });
    for (size_t i = 0; i < spans.size();) {
        char *const lo = (char *)spans[i].dst;
        char *hi = lo + spans[i].bytes;
        size_t j = i + 1;
        while (g->bump_base && j < spans.size() && (char *)spans[j].dst >= hi &&
               (char *)spans[j].dst - hi < 256) {
            hi = (char *)spans[j].dst + spans[j].bytes;
            ++j;
        }
        if (j == i + 1) {
            QC_HIP(hipMemcpy(spans[i].dst, spans[i].src, spans[i].bytes, hipMemcpyHostToDevice));
        } else {
            std::vector<char> stage((size_t)(hi - lo), 0);
            for (size_t k = i; k < j; ++k)
                memcpy(stage.data() + ((char *)spans[k].dst - lo), spans[k].src, spans[k].bytes);
            QC_HIP(hipMemcpy(lo, stage.data(), stage.size(), hipMemcpyHostToDevice));
        }
        i = j;
    }
    return QC_OK;
}

qc_status push_desc(qc_graph g, hipStream_t st)
{
    return from_hip(launch_set_desc(g->d_desc, g->desc(), st));
}

uint32_t batch_target(qc_graph g, int s0, int bw)
{
    uint64_t t = 0;
    for (int s = s0; s < s0 + bw && s < g->n; ++s) t += (uint64_t)g->comp_size[g->src_order[s]];
    return (uint32_t)t;
}

// LDS banks the order of the packed edges is chosen for (QC_EDGE_BANKS=0
// keeps rows-ascending order; a switch for measurements and tests).
static int edge_banks()
{
    const char *s = getenv("QC_EDGE_BANKS");
    if (!s) return 32;
    const int b = atoi(s);
    return (b == 0 || b == 16 || b == 32 || b == 64) ? b : 32;
}

// The packed edges with every row field raised by `bias` (bfs_row_bias).
static std::vector<uint32_t> biased_edges(const std::vector<uint32_t> &e, int bias)
{
    std::vector<uint32_t> out(e);
    if (bias)
        for (uint32_t &x : out) x += (uint32_t)bias << 16;
    return out;
}

// Upload the edges in the handle's current order with row bias `bias`; on a
// failure the device copy is unknown (a launch then refuses it).
static qc_status upload_edges(qc_graph g, int bias)
{
    const std::vector<uint32_t> &e = g->edges_bw ? g->edges_order : g->edges_host;
    g->edges_bias = -1;
    QC_TRY(bias ? upload(g->d_edges, biased_edges(e, bias)) : upload(g->d_edges, e));
    g->edges_bias = bias;
    return QC_OK;
}

// Upload the packed edges in the order that spreads the pull's gathers over
// the LDS banks for batches of `bw` sources.
static qc_status order_edges(qc_graph g, int bw, int bias)
{
    std::vector<uint32_t> e = g->edges_host;
    const int banks = edge_banks();
    if (banks > 0)
        spread_gather_banks(e, g->nnz_bfs, bw >= 32 ? 1 : 32 / bw, bw == 64 ? banks / 2 : banks);
    g->edges_order = std::move(e);
    g->edges_bw = bw;
    return upload_edges(g, bias);
}

qc_status plain_edges(qc_graph g)
{
    g->edges_bw = 0;
    g->edges_order.clear();
    return upload_edges(g, g->edges_bias < 0 ? 0 : g->edges_bias);
}

qc_status ensure_edges(qc_graph g, int bias)
{
    if (g->edges_bias == bias) return QC_OK;
    // the edges carry another launch shape's bias (the graph is also in a
    // batch that planned it otherwise, or a failed upload left them
    // unknown): nothing still in flight may read the old rows
    QC_HIP(hipDeviceSynchronize());
    return upload_edges(g, bias);
}

qc_status check_edges(qc_graph g)
{
    return ensure_edges(g, bfs_row_bias(g->plan.bw, g->plan.nw, g->plan.shape));
}

qc_status set_plan(qc_graph g, const BfsPlan &plan, bool reorder)
{
    if (plan.bw <= 0) return QC_E_INVAL;
    BfsPlan p = plan;
    p.n_batches = (g->n + p.bw - 1) / p.bw;   // sources are the graph's own nodes
    // the bank-aware order costs host time per edge that only repeated
    // searches repay: it is chosen once the largest distance (and so the
    // final batch width) is known, and never for serving requests, which
    // search once; and the rows carry the bias of the plan's launch shape.
    // The edges go up last, once nothing else can fail (a failed upload
    // leaves them unknown, and launches refuse them until a plan is set).
    const int bias = bfs_row_bias(p.bw, p.nw, p.shape);
    auto edges = [&]() -> qc_status {
        if (reorder && g->dmax >= 0 && !g->bump_base && p.bw != g->edges_bw)
            return order_edges(g, p.bw, bias);
        return bias != g->edges_bias ? upload_edges(g, bias) : QC_OK;
    };
    if (g->d_bfs_jobs && p.bw == g->plan.bw) {
        QC_TRY(edges());
        g->plan = p;
        return QC_OK;
    }
    // last batch first: the source order puts the farthest-reaching sources
    // (the longest searches) at the end
    std::vector<BfsJob> jobs(p.n_batches);
    for (int b = 0; b < p.n_batches; ++b) {
        const int s0 = (p.n_batches - 1 - b) * p.bw;
        jobs[b] = BfsJob{0, s0, batch_target(g, s0, p.bw), 0u};
    }
    // the new table replaces the old one only once it is in place, so a
    // failed allocation leaves the handle's plan and jobs as they were
    BfsJob *d_jobs = nullptr;
    QC_TRY(galloc(g, &d_jobs, jobs.size()));
    qc_status s = upload(d_jobs, jobs);
    if (s == QC_OK) s = edges();
    if (s != QC_OK) {
        gfree(g, d_jobs);
        return s;
    }
    gfree(g, g->d_bfs_jobs);
    g->d_bfs_jobs = d_jobs;
    g->plan = p;
    return QC_OK;
}

qc_status ensure_hist_jobs(qc_graph g)
{
    if (g->d_hist_jobs && g->hist_jobs_k == g->K) return QC_OK;
    const int rows = hist_rows_per_job(g->K);
    std::vector<NodeJob> jobs;
    for (int i = 0; i < g->n; i += rows) jobs.push_back(NodeJob{0, i, 0});
    NodeJob *d_jobs = nullptr;
    QC_TRY(galloc(g, &d_jobs, jobs.size()));
    const qc_status s = upload(d_jobs, jobs);
    if (s != QC_OK) {
        gfree(g, d_jobs);
        return s;
    }
    gfree(g, g->d_hist_jobs);
    g->d_hist_jobs = d_jobs;
    g->n_hist_jobs = (int)jobs.size();
    g->hist_jobs_k = g->K;
    return QC_OK;
}

// After the first search: the sources by their exact eccentricity, the last
// non-empty bin of their histogram row (ties keep the order of the bounds
// the host sweeps gave). A batch searches until its farthest source is
// done, so batches of sources with equal eccentricity pull the fewest
// levels; every later search of the handle (a batch, a sigma sweep, a
// second qc_distances) takes this order, and its batches' targets with it.
static qc_status exact_source_order(qc_graph g, hipStream_t st)
{
    std::vector<int32_t> h((size_t)g->n * g->K);
    QC_HIP(hipMemcpyAsync(h.data(), g->d_hist, h.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    QC_HIP(hipStreamSynchronize(st));
    std::vector<int32_t> ecc(g->n, 0);
    for (int32_t i = 0; i < g->n; ++i)
        for (int k = g->K - 1; k > 0; --k)
            if (h[(size_t)i * g->K + k]) {
                ecc[i] = k;
                break;
            }
    std::vector<int32_t> order = g->src_order;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return ecc[a] < ecc[b]; });
    const BfsPlan &p = g->plan;
    std::vector<BfsJob> jobs(p.n_batches);
    // the new tables replace the old ones only once both are in place
    int32_t *d_src = nullptr;
    BfsJob *d_jobs = nullptr;
    qc_status s = galloc(g, &d_src, order.size());
    if (s == QC_OK) s = galloc(g, &d_jobs, jobs.size());
    if (s == QC_OK) s = upload(d_src, order);
    if (s == QC_OK) {
        std::swap(g->src_order, order);
        for (int b = 0; b < p.n_batches; ++b) {
            const int s0 = (p.n_batches - 1 - b) * p.bw;   // last batch first, as in set_plan
            jobs[b] = BfsJob{0, s0, batch_target(g, s0, p.bw), 0u};
        }
        s = upload(d_jobs, jobs);
        if (s != QC_OK) std::swap(g->src_order, order);
    }
    if (s != QC_OK) {
        if (d_src) gfree(g, d_src);
        if (d_jobs) gfree(g, d_jobs);
        return s;
    }
    gfree(g, g->d_src);
    gfree(g, g->d_bfs_jobs);
    g->d_src = d_src;
    g->d_bfs_jobs = d_jobs;
    return push_desc(g, st);
}

// BFS into g->d_dist, then histograms. The first run waits to learn dmax.
qc_status run_distances(qc_graph g, hipStream_t st)
{
    QC_TRY(check_edges(g));
    QC_HIP(launch_fill_i32(g->d_status, 2, 0, st));
    QC_TRY(push_desc(g, st));
    {
        StageTimer t(QC_STAGE_BFS, st);
        QC_HIP(launch_bfs(g->plan.bw, g->plan.nw, g->plan.planes,
                          g->plan.shape | (g->weighted ? kBfsWeighted : 0), g->d_desc,
                          g->d_bfs_jobs, g->plan.n_batches, st));
    }
    const bool first = g->dmax < 0;
    if (first) {
        int32_t status[2];
        QC_HIP(hipMemcpyAsync(status, g->d_status, sizeof status, hipMemcpyDeviceToHost, st));
        QC_HIP(hipStreamSynchronize(st));
        if (status[1] & 1) return QC_E_OVERFLOW;
        // a level beyond the planes of a plan with fewer than 7 (cannot
        // happen: a first search with fewer planes was planned from an upper
        // bound on every distance)
        if (status[1] & 2) return QC_E_DEVICE;
        // the largest level the search reached; with weighted edges it can
        // be that of a node inside an edge, above the graph's own dmax
        const int old_k = g->K;
        g->dmax_bfs = status[0];
        g->dmax = status[0];
        g->K = bins_for(g->dmax);
        // a failed allocation leaves dmax unknown (the next call redoes this
        // step) with every buffer the handle had still in place
        int32_t *hist = nullptr;
        qc_status s = galloc(g, &hist, (size_t)g->n * g->K);
        // later runs need only enough planes for dmax: maybe a wider batch
        if (s == QC_OK) s = set_plan(g, plan_bfs(g->n_bfs, g->dmax_bfs));
        if (s == QC_OK) s = ensure_hist_jobs(g);
        if (s != QC_OK) {
            if (hist) gfree(g, hist);
            g->dmax = g->dmax_bfs = -1;
            g->K = old_k;
            return s;
        }
        gfree(g, g->d_hist);
        g->d_hist = hist;
        QC_TRY(push_desc(g, st));
    }
    {
        StageTimer t(QC_STAGE_HIST, st);
        QC_HIP(launch_hist(g->K, g->d_desc, g->d_hist_jobs, g->n_hist_jobs, st));
    }
    if (first && g->ecc_order) QC_TRY(exact_source_order(g, st));
    if (first && g->weighted) {
        // the graph's own largest finite distance: the last non-empty bin
        std::vector<int32_t> h((size_t)g->n * g->K);
        QC_HIP(hipMemcpyAsync(h.data(), g->d_hist, h.size() * sizeof(int32_t),
                              hipMemcpyDeviceToHost, st));
        QC_HIP(hipStreamSynchronize(st));
        int32_t dm = 0;
        for (size_t i = 0; i < h.size(); ++i)
            if (h[i] && (int32_t)(i % g->K) > dm) dm = (int32_t)(i % g->K);
        g->dmax = dm;
        QC_TRY(push_desc(g, st));
    }
    g->have_dist = true;
    return QC_OK;
}

qc_status ensure_sigma_buffers(qc_graph g, int S)
{
    // New buffers replace the old ones only once all of them are in place,
    // so a failed allocation leaves the handle's buffers as they were.
    if (S > g->pot_cap) {
        float *psi = nullptr, *v = nullptr;
        double *v64 = nullptr;
        int32_t *parent = nullptr;
        qc_status s = galloc(g, &psi, (size_t)S * g->n);
        if (s == QC_OK) s = galloc(g, &v, (size_t)v_floats(g->n, S));
        if (s == QC_OK) s = galloc(g, &v64, (size_t)S * g->n);
        if (s == QC_OK) s = galloc(g, &parent, (size_t)S * g->n);
        if (s != QC_OK) {
            gfree(g, psi);
            gfree(g, v);
            gfree(g, v64);
            gfree(g, parent);
            return s;
        }
        gfree(g, g->d_psi);
        gfree(g, g->d_v);
        gfree(g, g->d_v64);
        gfree(g, g->d_parent);
        g->d_psi = psi;
        g->d_v = v;
        g->d_v64 = v64;
        g->d_parent = parent;
        g->pot_cap = S;
    }
    if (S * g->K > g->w_cap) {
        double *w64 = nullptr, *u64 = nullptr, *inv_a = nullptr;
        float *w32c = nullptr;
        uint16_t *wbf16 = nullptr;
        qc_status s = galloc(g, &wbf16, (size_t)S * g->K * 2);
        if (s == QC_OK) s = galloc(g, &w64, (size_t)S * g->K);
        if (s == QC_OK) s = galloc(g, &u64, (size_t)S * g->K);
        if (s == QC_OK) s = galloc(g, &inv_a, (size_t)S);
        if (s == QC_OK) s = galloc(g, &w32c, (size_t)S * g->K * 4);
        if (s != QC_OK) {
            gfree(g, wbf16);
            gfree(g, w64);
            gfree(g, u64);
            gfree(g, inv_a);
            gfree(g, w32c);
            return s;
        }
        gfree(g, g->d_w64);
        gfree(g, g->d_u64);
        gfree(g, g->d_inv_a);
        gfree(g, g->d_w32c);
        gfree(g, g->d_wbf16);
        g->d_w64 = w64;
        g->d_u64 = u64;
        g->d_inv_a = inv_a;
        g->d_w32c = w32c;
        g->d_wbf16 = wbf16;
        g->w_cap = S * g->K;
    }
    return QC_OK;
}

qc_status load_sigmas(qc_graph g, const double *sigmas, int32_t n_sigmas, hipStream_t st)
{
    std::vector<double> sig(sigmas, sigmas + n_sigmas);
    if (sig != g->sigmas_loaded) {
        std::vector<double> w64, u64, inv_a;
        std::vector<float> w32c;
        std::vector<uint16_t> wbf16;
        weight_tables(sigmas, n_sigmas, g->K, w64, u64, inv_a, w32c, wbf16);
        QC_TRY(ensure_sigma_buffers(g, n_sigmas));
        // The weight tables are tiny; a synchronous upload keeps host buffers
        // safe. A repeated sigma list reuses the tables already on the device.
        QC_HIP(hipStreamSynchronize(st));
        QC_TRY(upload_group(g, {span_of(g->d_w64, w64), span_of(g->d_u64, u64), span_of(g->d_inv_a, inv_a),
                                span_of(g->d_w32c, w32c), span_of(g->d_wbf16, wbf16)}));
        g->sigmas_loaded = sig;
        g->n_sigmas = n_sigmas;
        QC_TRY(push_desc(g, st));
    }
    return QC_OK;
}

int64_t handle_footprint(int32_t n, int64_t nnz, int32_t n_sigmas, bool with_dist,
                         bool with_labels)
{
    if (n < 1 || n > kMaxNodes || nnz < 0 || nnz >= kMaxEdges || n_sigmas < 1 ||
        n_sigmas > 1024)
        return -1;
    const int64_t N = n, S = n_sigmas, K = 128;  // histogram bins: the largest row length
    const int64_t quads = (nnz + 3) / 4 * 4 + 4;
    int64_t b = 0;
    auto add = [&](int64_t bytes) { b += ((bytes > 0 ? bytes : 1) + 255) & ~(int64_t)255; };
    add(4 * (N + 1));                 // row_ptr
    add(4 * nnz);                     // col
    add(4 * N);                       // descent thread order
    add(4 * N + 4 * (N / 64 + 2));    // sliced neighbour lists: degrees, slice offsets
    {
        // and entries: within a window of degree-sorted nodes the padding
        // adds up to at most 63 times the window's largest degree
        const int64_t windows = (N + kOrderWindow - 1) / kOrderWindow;
        add(4 * (nnz + 63 * std::min<int64_t>(nnz, windows * (N - 1)) + 64 * kGgdPad));
    }
    add(4 * N);                       // BFS source order
    add(4 * quads);                   // packed edges
    add(8);                           // status
    add(8);                           // recheck counter
    add((int64_t)sizeof(GraphDev));   // descriptor
    add(16 * ((N + kNodesPerJob - 1) / kNodesPerJob));  // node jobs
    add(8 * N);                       // BFS jobs (first plan, <= one job per node)
    add(8 * N);                       // BFS jobs (plan after dmax is known)
    if (with_dist) add(N * owned_ld(n) + 16);   // distance matrix (rows on 128-byte lines)
    add(4 * N * K);                   // histograms
    add(16 * N);                      // histogram jobs
    add(4 * N * S);                   // psi
    add(4 * v_floats(n, n_sigmas));   // V (sigma groups rounded up)
    add(8 * N * S);                   // FP64 V
    add(4 * N * S);                   // parents
    add(8 * S * K);                   // w64
    add(8 * S * K);                   // u64
    add(8 * S);                       // 1/a
    add(16 * S * K);                  // FP32 split weights
    add(4 * S * K);                   // BF16 weights
    if (with_labels) add(4 * N * S);  // labels
    return b;
}

qc_status cluster_on_handle(qc_graph g, const double *sigmas, int32_t n_sigmas,
                            uint32_t tie_mode, int8_t *dist_out, float *psi_out, float *v_out,
                            int32_t *labels_out, hipStream_t st)
{
    void *stream = (void *)st;
    QC_TRY(qc_distances(g, dist_out, nullptr, stream));
    QC_TRY(qc_potential(g, sigmas, n_sigmas, psi_out, v_out, QC_PREC_FP64ACC, stream));
    for (int32_t k = 0; k < n_sigmas; ++k)
        QC_TRY(qc_ggd_labels(g, k, tie_mode, labels_out + (size_t)k * g->n, stream));
    return qc_graph_sync(g, stream);
}

void destroy(qc_graph g, bool sync)
{
    if (!g) return;
    if (sync) (void)hipDeviceSynchronize();
    gfree(g, g->d_row_ptr);
    gfree(g, g->d_col);
    gfree(g, g->d_order);
    gfree(g, g->d_sell_col);
    gfree(g, g->d_sell_off);
    gfree(g, g->d_sell_deg);
    gfree(g, g->d_src);
    gfree(g, g->d_bfs_row_ptr);
    gfree(g, g->d_bfs_col);
    gfree(g, g->d_edges);
    gfree(g, g->d_dist_owned);
    gfree(g, g->d_hist);
    gfree(g, g->d_psi);
    gfree(g, g->d_v);
    gfree(g, g->d_v64);
    gfree(g, g->d_parent);
    gfree(g, g->d_w64);
    gfree(g, g->d_u64);
    gfree(g, g->d_inv_a);
    gfree(g, g->d_w32c);
    gfree(g, g->d_wbf16);
    gfree(g, g->d_status);
    gfree(g, g->d_recheck);
    gfree(g, g->d_desc);
    gfree(g, g->d_bfs_jobs);
    gfree(g, g->d_node_jobs);
    gfree(g, g->d_hist_jobs);
    delete g;
}

}  // namespace qc

extern "C" {

const char *qc_status_str(qc_status s)
{
    switch (s) {
    case QC_OK: return "QC_OK";
    case QC_E_INVAL: return "QC_E_INVAL: invalid argument";
    case QC_E_NOT_SYMMETRIC: return "QC_E_NOT_SYMMETRIC: CSR is not a canonical adjacency";
    case QC_E_OOM: return "QC_E_OOM: out of device memory";
    case QC_E_DEVICE: return "QC_E_DEVICE: no gfx950 device or a HIP call failed";
    case QC_E_OVERFLOW: return "QC_E_OVERFLOW: a finite hop distance exceeds 126";
    case QC_E_STATE: return "QC_E_STATE: call order violated";
    case QC_E_BUSY: return "QC_E_BUSY: request does not fit the memory budget, or is running";
    case QC_E_TIMEOUT: return "QC_E_TIMEOUT: request not admitted before its queue deadline";
    case QC_E_CANCELLED: return "QC_E_CANCELLED: request withdrawn before it ran";
    case QC_E_TOO_LARGE: return "QC_E_TOO_LARGE: problem exceeds the fixed scratch of qc_cluster_noalloc";
    default: return "unknown qc_status";
    }
}

qc_status qc_device_count(int32_t *count_out)
{
    if (!count_out) return QC_E_INVAL;
    *count_out = 0;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess) {
        (void)hipGetLastError();
        return QC_OK;
    }
    int32_t c = 0;
    for (int d = 0; d < count; ++d) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, d) == hipSuccess &&
            strncmp(prop.gcnArchName, "gfx950", 6) == 0)
            ++c;
    }
    *count_out = c;
    return QC_OK;
}

qc_status qc_graph_create(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                          uint32_t flags, void *stream, qc_graph *out)
{
    return create_graph(n, nnz, row_ptr, col_idx, flags, as_stream(stream), nullptr, 0, out);
}

qc_status qc_graph_create_weighted(int32_t n, int64_t nnz, const int32_t *row_ptr,
                                   const int32_t *col_idx, const uint8_t *weights, uint32_t flags,
                                   void *stream, qc_graph *out)
{
    if (!weights && nnz > 0) return QC_E_INVAL;
    static const uint8_t kNone = 1;
    return create_graph(n, nnz, row_ptr, col_idx, flags, as_stream(stream), nullptr, 0, out,
                        weights ? weights : &kNone);
}

}  // extern "C"

namespace qc {

qc_status create_graph(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                       uint32_t flags, hipStream_t st, char *region, size_t region_bytes,
                       qc_graph *out, const uint8_t *weights, bool hop_search)
{
    if (!out) return QC_E_INVAL;
    if (flags & ~(uint32_t)(QC_GRAPH_CANONICALIZE | QC_GRAPH_DIRECTED)) return QC_E_INVAL;
    // weights follow the caller's CSR entries, so that CSR must be canonical
    if (weights && (flags & QC_GRAPH_CANONICALIZE)) return QC_E_INVAL;
    const bool directed = (flags & QC_GRAPH_DIRECTED) != 0;
    std::vector<int32_t> rp, col;
    QC_TRY(validate_csr(n, nnz, row_ptr, col_idx, (flags & QC_GRAPH_CANONICALIZE) != 0, rp, col,
                        directed));
    int32_t n_bfs = n;
    std::vector<int32_t> brp, bcol;
    if (weights) {
        QC_TRY(subdivide_weighted(n, rp, col, weights, directed, n_bfs, brp, bcol));
        if ((int64_t)bcol.size() >= kMaxEdges) return QC_E_INVAL;
    }
    int dev = 0;
    QC_TRY(check_device(&dev));

    qc_graph g = new qc_graph_s();
    g->device = dev;
    g->bump_base = region;
    g->bump_size = region_bytes;
    g->n = n;
    g->nnz = (int64_t)col.size();
    // (weakly) connected components: a source reaches at most its component,
    // exactly all of it when the graph is undirected (the BFS's stop target).
    // With weights they are taken in the graph the BFS walks, whose extra
    // nodes the search counts too (and whose components are the graph's).
    if (weights) {
        std::vector<int32_t> size_all;
        g->n_components = count_components(n_bfs, brp, bcol, &size_all);
        g->comp_size.assign(size_all.begin(), size_all.begin() + n);
    } else {
        g->n_components = count_components(n, rp, col, &g->comp_size);
    }

    g->n_bfs = n_bfs;
    g->nnz_bfs = weights ? (int64_t)bcol.size() : g->nnz;
    g->weighted = weights != nullptr;
    g->edges_host =
        weights ? pack_in_edges(n_bfs, brp, bcol, directed) : pack_in_edges(n, rp, col, directed);
    const std::vector<uint32_t> &edges = g->edges_host;
    // The descent gives one thread to each node, in this order: nodes sorted
    // by decreasing degree within windows of kOrderWindow consecutive nodes,
    // so a wavefront's neighbour loops have similar trip counts while the
    // scattered loads and stores of a window's jobs stay within a few KB.
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    for (int32_t i0 = 0; i0 < n; i0 += kOrderWindow)
        std::stable_sort(order.begin() + i0, order.begin() + std::min(n, i0 + kOrderWindow),
                         [&](int32_t a, int32_t b) { return rp[a + 1] - rp[a] > rp[b + 1] - rp[b]; });
    // ... and reads its node's neighbours from a sliced ELL copy of the CSR
    // in that order: 64 nodes (one wavefront) per slice, as wide as the
    // slice's largest degree, slot-major; unused entries hold node 0.
    const int32_t n_slices = (n + 63) / 64;
    std::vector<int32_t> sell_off(n_slices + 1, 0), sell_deg(n);
    for (int32_t t = 0; t < n; ++t) sell_deg[t] = rp[order[t] + 1] - rp[order[t]];
    for (int32_t w = 0; w < n_slices; ++w) {
        int32_t width = 0;
        for (int32_t t = 64 * w; t < std::min(n, 64 * w + 64); ++t) width = std::max(width, sell_deg[t]);
        sell_off[w + 1] = sell_off[w] + 64 * width;
    }
    std::vector<int32_t> sell_col((size_t)sell_off[n_slices] + 64 * kGgdPad, 0);
    for (int32_t t = 0; t < n; ++t) {
        const int32_t i = order[t], w = t / 64, lane = t % 64;
        for (int32_t k = 0; k < sell_deg[t]; ++k)
            sell_col[(size_t)sell_off[w] + 64 * k + lane] = col[rp[i] + k];
    }
    // BFS sources by estimated eccentricity (undirected graphs; a directed
    // graph keeps its node order, and so does a serving request: its one
    // search would not repay the host sweeps). QC_SOURCE_ORDER=identity keeps
    // the node order for every graph (a switch for measurements and tests).
    // The same sweeps bound every distance of an undirected graph (by the
    // largest eccentricity bound), so its first search can already run with
    // the distance planes and launch shape of a known largest distance
    // instead of 7 planes; a serving request, which searches once, takes one
    // sweep for this bound when the 7-plane plan would narrow its batches.
    const char *so = getenv("QC_SOURCE_ORDER");
    int32_t bound = -1;
    if (hop_search && !directed && !region && !(so && strcmp(so, "identity") == 0)) {
        g->src_order = weights ? source_order(n_bfs, brp, bcol, n, kSourceSweeps, &bound)
                               : source_order(n, rp, col, n, kSourceSweeps, &bound);
        g->ecc_order = !weights;
    } else {
        g->src_order.resize(n);
        std::iota(g->src_order.begin(), g->src_order.end(), 0);
        if (hop_search && !directed && plan_bfs(n_bfs, -1).bw < kBfsFullWidth) {
            if (weights)
                (void)source_order(n_bfs, brp, bcol, 0, 1, &bound);
            else
                (void)source_order(n, rp, col, 0, 1, &bound);
        }
    }
    // (a bound above 126 leaves the 7-plane plan, which detects overflow)
    if (bound > kMaxDist) bound = -1;
    std::vector<NodeJob> njobs;
    for (int i = 0; i < n; i += kNodesPerJob) njobs.push_back(NodeJob{0, i, 0});
    g->n_node_jobs = (int)njobs.size();

    qc_status st_ = QC_OK;
    auto fail = [&](qc_status s) { destroy(g, region == nullptr); return s; };
    if ((st_ = galloc(g, &g->d_row_ptr, rp.size())) || (st_ = galloc(g, &g->d_col, col.size())) ||
        (st_ = galloc(g, &g->d_order, order.size())) ||
        (st_ = galloc(g, &g->d_sell_col, sell_col.size())) ||
        (st_ = galloc(g, &g->d_sell_off, sell_off.size())) ||
        (st_ = galloc(g, &g->d_sell_deg, sell_deg.size())) ||
        (st_ = galloc(g, &g->d_src, g->src_order.size())) ||
        (weights && ((st_ = galloc(g, &g->d_bfs_row_ptr, brp.size())) ||
                     (st_ = galloc(g, &g->d_bfs_col, bcol.size())))) ||
        (st_ = galloc(g, &g->d_edges, edges.size())) || (st_ = galloc(g, &g->d_status, 2)) ||
        (st_ = galloc(g, &g->d_recheck, 1)) || (st_ = galloc(g, &g->d_desc, 1)) ||
        (st_ = galloc(g, &g->d_node_jobs, njobs.size())))
        return fail(st_);
    // the edges go up with the row bias of the first plan's launch shape
    const BfsPlan plan0 = plan_bfs(n_bfs, bound);
    const int bias0 = plan0.bw > 0 ? bfs_row_bias(plan0.bw, plan0.nw, plan0.shape) : 0;
    const std::vector<uint32_t> edges0 = bias0 ? biased_edges(edges, bias0) : std::vector<uint32_t>();
    g->edges_bias = bias0;
    std::vector<HostSpan> spans = {span_of(g->d_row_ptr, rp),        span_of(g->d_col, col),
                                   span_of(g->d_order, order),        span_of(g->d_src, g->src_order),
                                   span_of(g->d_sell_col, sell_col),  span_of(g->d_sell_off, sell_off),
                                   span_of(g->d_sell_deg, sell_deg),  span_of(g->d_edges, bias0 ? edges0 : edges),
                                   span_of(g->d_node_jobs, njobs)};
    if (weights) {
        spans.push_back(span_of(g->d_bfs_row_ptr, brp));
        spans.push_back(span_of(g->d_bfs_col, bcol));
    }
    if ((st_ = upload_group(g, spans)) || (st_ = set_plan(g, plan0)))
        return fail(st_);
    if ((st_ = from_hip(launch_fill_u64(g->d_recheck, 1, st))) || (st_ = push_desc(g, st)))
        return fail(st_);
    *out = g;
    return QC_OK;
}

}  // namespace qc

extern "C" {

qc_status qc_graph_destroy(qc_graph g)
{
    if (!g) return QC_E_INVAL;
    destroy(g);
    return QC_OK;
}

qc_status qc_graph_bfs_plan(qc_graph g, int32_t *batch, int32_t *words, int32_t *planes,
                            int32_t *shape)
{
    if (!g) return QC_E_INVAL;
    if (batch) *batch = g->plan.bw;
    if (words) *words = g->plan.nw;
    if (planes) *planes = g->plan.planes;
    if (shape) *shape = g->plan.shape;
    return QC_OK;
}

qc_status qc_graph_info(qc_graph g, int32_t *n, int64_t *nnz, int32_t *dmax, int32_t *n_components)
{
    if (!g) return QC_E_INVAL;
    if (n) *n = g->n;
    if (nnz) *nnz = g->nnz;
    if (dmax) *dmax = g->dmax;
    if (n_components) *n_components = g->n_components;
    return QC_OK;
}

qc_status qc_distances(qc_graph g, int8_t *dist_out, int32_t *dmax_out, void *stream)
{
    if (!g) return QC_E_INVAL;
    hipStream_t st = as_stream(stream);
    if (dist_out) {
        if (((uintptr_t)dist_out) % 16) return QC_E_INVAL;  // rows are read in 16-byte chunks
        g->d_dist = dist_out;
        g->d_ld = g->n;
    } else {
        if (!g->d_dist_owned) QC_TRY(galloc(g, &g->d_dist_owned, (size_t)(g->n * owned_ld(g->n) + 16)));
        g->d_dist = g->d_dist_owned;
        g->d_ld = owned_ld(g->n);
    }
    QC_TRY(run_distances(g, st));
    if (dmax_out) *dmax_out = g->dmax;
    return QC_OK;
}

qc_status qc_get_histograms(qc_graph g, int32_t *hist_out, int32_t *k_out, void *stream)
{
    if (!g) return QC_E_INVAL;
    if (!g->have_dist) return QC_E_STATE;
    if (k_out) *k_out = g->K;
    if (hist_out)
        QC_HIP(hipMemcpyAsync(hist_out, g->d_hist, (size_t)g->n * g->K * sizeof(int32_t),
                              hipMemcpyDeviceToDevice, as_stream(stream)));
    return QC_OK;
}

qc_status qc_potential(qc_graph g, const double *sigmas, int32_t n_sigmas, float *psi_out,
                       float *v_out, uint32_t precision, void *stream)
{
    if (!g) return QC_E_INVAL;
    QC_TRY(validate_sigmas(sigmas, n_sigmas));
    if (precision > QC_PREC_BF16) return QC_E_INVAL;
    hipStream_t st = as_stream(stream);
    if (!g->have_dist) QC_TRY(qc_distances(g, nullptr, nullptr, stream));

    // until this call has succeeded the handle holds no potentials (the
    // descent refuses to run on a half-made set)
    g->have_pot = false;
    QC_TRY(load_sigmas(g, sigmas, n_sigmas, st));
    if (precision != g->pot_precision) {
        // the descriptor's FP64 table pointer depends on the precision
        g->pot_precision = precision;
        QC_TRY(push_desc(g, st));
    }
    {
        StageTimer t(QC_STAGE_POTENTIAL, st);
        QC_HIP(launch_potential((int)precision, g->K, g->d_desc, g->d_node_jobs, g->n_node_jobs,
                                psi_out, v_out, g->n, st));
    }
    g->have_pot = true;
    return QC_OK;
}

qc_status qc_ggd_labels(qc_graph g, int32_t sigma_index, uint32_t tie_mode, int32_t *labels_out,
                        void *stream)
{
    if (!g || !labels_out) return QC_E_INVAL;
    if (tie_mode > QC_TIE_MERGE) return QC_E_INVAL;
    if (!g->have_pot || g->pot_precision == QC_PREC_BF16) return QC_E_STATE;
    if (sigma_index < 0 || sigma_index >= g->n_sigmas) return QC_E_INVAL;
    hipStream_t st = as_stream(stream);
    QC_HIP(launch_fill_u64(g->d_recheck, 1, st));
    {
        StageTimer t(QC_STAGE_GGD, st);
        QC_HIP(launch_ggd_parent((int)tie_mode, g->d_desc, g->d_node_jobs, g->n_node_jobs,
                                 sigma_index, 1, st));
    }
    {
        StageTimer t(QC_STAGE_JUMP, st);
        QC_HIP(launch_pointer_jump(g->d_desc, g->d_node_jobs, 1, sigma_index, 1, labels_out, 0,
                                   g->n, st));
    }
    return QC_OK;
}

qc_status qc_get_potential64(qc_graph g, double *v64_out, void *stream)
{
    if (!g || !v64_out) return QC_E_INVAL;
    if (!g->have_pot || g->pot_precision != QC_PREC_FP64ACC) return QC_E_STATE;
    QC_HIP(hipMemcpyAsync(v64_out, g->d_v64, (size_t)g->n_sigmas * g->n * sizeof(double),
                          hipMemcpyDeviceToDevice, as_stream(stream)));
    return QC_OK;
}

qc_status qc_last_recheck_count(qc_graph g, int64_t *count_out)
{
    if (!g || !count_out) return QC_E_INVAL;
    unsigned long long c = 0;
    QC_HIP(hipDeviceSynchronize());
    QC_HIP(hipMemcpy(&c, g->d_recheck, sizeof c, hipMemcpyDeviceToHost));
    *count_out = (int64_t)c;
    return QC_OK;
}

qc_status qc_potential_dense(const float *dist, int64_t n_rows, int64_t n_cols, int64_t ld,
                             const double *sigmas, int32_t n_sigmas, double *psi_out,
                             double *v_out, void *stream)
{
    if (n_rows < 0 || n_cols < 0 || ld < n_cols) return QC_E_INVAL;
    QC_TRY(validate_sigmas(sigmas, n_sigmas));
    // below 1e-100, d^2 / (2 sigma^2) could overflow for the largest floats
    for (int32_t s = 0; s < n_sigmas; ++s)
        if (sigmas[s] < 1e-100) return QC_E_INVAL;
    if (n_rows == 0) return QC_OK;
    if (!psi_out || !v_out || (n_cols > 0 && !dist)) return QC_E_INVAL;
    // one workgroup per 4 rows: the grid's x dimension bounds the row count
    if ((n_rows + 3) / 4 > (int64_t)INT32_MAX) return QC_E_INVAL;
    int dev = 0;
    QC_TRY(check_device(&dev));
    QC_HIP(launch_dense(dist, n_rows, n_cols, ld, sigmas, n_sigmas, psi_out, v_out,
                        as_stream(stream)));
    return QC_OK;
}

qc_status qc_graph_sync(qc_graph g, void *stream)
{
    if (!g) return QC_E_INVAL;
    hipStream_t st = as_stream(stream);
    QC_HIP(hipStreamSynchronize(st));
    int32_t status[2] = {0, 0};
    QC_HIP(hipMemcpy(status, g->d_status, sizeof status, hipMemcpyDeviceToHost));
    if (status[1] & 1) return QC_E_OVERFLOW;
    if (status[1] & 2) return QC_E_DEVICE;
    return QC_OK;
}

qc_status qc_cluster(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                     const double *sigmas, int32_t n_sigmas, uint32_t tie_mode, int8_t *dist_out,
                     float *psi_out, float *v_out, int32_t *labels_out, void *stream)
{
    if (!labels_out || tie_mode > QC_TIE_MERGE) return QC_E_INVAL;
    if (dist_out && ((uintptr_t)dist_out) % 16) return QC_E_INVAL;
    QC_TRY(validate_sigmas(sigmas, n_sigmas));
    hipStream_t st = as_stream(stream);
    // a problem that fits the fixed scratch runs there, without the device
    // allocations (and frees) of a temporary handle
    const qc_status fit = cluster_scratch(n, nnz, row_ptr, col_idx, sigmas, n_sigmas, tie_mode, dist_out,
                                          psi_out, v_out, labels_out, st, true);
    if (fit != QC_E_TOO_LARGE) return fit;
    qc_graph g = nullptr;
    QC_TRY(create_graph(n, nnz, row_ptr, col_idx, 0, st, nullptr, 0, &g));
    const qc_status s =
        cluster_on_handle(g, sigmas, n_sigmas, tie_mode, dist_out, psi_out, v_out, labels_out, st);
    (void)hipStreamSynchronize(st);
    destroy(g, false);
    return s;
}

qc_status qc_debug_alloc_fault(int64_t fail_at, int64_t *live_out)
{
    if (fail_at < 0) return QC_E_INVAL;
    g_fault_countdown.store(fail_at, std::memory_order_relaxed);
    if (live_out) *live_out = g_live_allocs.load(std::memory_order_relaxed);
    return QC_OK;
}

}  // extern "C"
