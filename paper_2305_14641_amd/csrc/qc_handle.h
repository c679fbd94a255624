// The graph handle and the helpers the API, batch and serving code share.
#pragma once

#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "qc.h"
#include "qc_host.h"
#include "qc_internal.h"

using qc::BfsJob;
using qc::BfsPlan;
using qc::GraphDev;
using qc::NodeJob;

struct qc_graph_s {
    int device = 0;
    // When set, every device buffer of the handle is carved from this region
    // (a serving request's slice of the server arena) instead of hipMalloc.
    char *bump_base = nullptr;
    size_t bump_size = 0, bump_off = 0;
    int32_t n = 0;
    int64_t nnz = 0;
    int32_t n_components = 0;
    std::vector<int32_t> comp_size;   // size of each node's component (host)
    BfsPlan plan{};

    // device CSR
    int32_t *d_row_ptr = nullptr;
    int32_t *d_col = nullptr;
    int32_t *d_order = nullptr;       // descent thread order (see create_graph)
    int32_t *d_sell_col = nullptr;    // descent neighbour lists, sliced ELL (see GraphDev)
    int32_t *d_sell_off = nullptr;
    int32_t *d_sell_deg = nullptr;
    std::vector<int32_t> src_order;   // BFS sources in batch order (host copy)
    bool ecc_order = false;           // sources ordered by eccentricity (bounds, then exact)
    int32_t *d_src = nullptr;         // and on the device
    int32_t n_bfs = 0;                // nodes of the graph the BFS walks
    int64_t nnz_bfs = 0;              // and its edges
    int32_t *d_bfs_row_ptr = nullptr; // its CSR when edges are weighted (else null)
    int32_t *d_bfs_col = nullptr;
    bool weighted = false;
    uint32_t *d_edges = nullptr;
    std::vector<uint32_t> edges_host; // packed edges, rows ascending (host copy)
    int edges_bw = 0;                 // batch width d_edges' order was chosen for (0: rows ascending)
    std::vector<uint32_t> edges_order; // that order (edges_bw > 0), rows as in edges_host
    int edges_bias = 0;               // row bias of d_edges (bfs_row_bias of the plan; -1: unknown)

    // distances and histograms
    int8_t *d_dist_owned = nullptr;   // library-owned matrix (n rows of owned_ld(n), 16-byte padded)
    int8_t *d_dist = nullptr;         // current resident matrix (owned or caller's)
    int64_t d_ld = 0;                 // its row stride
    int32_t *d_hist = nullptr;
    int K = 0;
    int32_t dmax = -1;
    int32_t dmax_bfs = -1;            // largest level of the search (>= dmax when weighted)
    bool have_dist = false;

    // potentials
    int n_sigmas = 0;
    int pot_cap = 0;                  // sigmas the buffers below hold
    float *d_psi = nullptr, *d_v = nullptr;
    double *d_v64 = nullptr;          // canonical FP64 V [S][n] (FP64ACC potentials)
    int32_t *d_parent = nullptr;
    double *d_w64 = nullptr, *d_u64 = nullptr, *d_inv_a = nullptr;
    float *d_w32c = nullptr;
    uint16_t *d_wbf16 = nullptr;
    int w_cap = 0;                    // sigma*K entries the weight buffers hold
    bool have_pot = false;
    uint32_t pot_precision = 0;
    std::vector<double> sigmas_loaded;  // sigma list whose tables are on the device

    // status words, descriptor, job tables
    int32_t *d_status = nullptr;              // [2]
    unsigned long long *d_recheck = nullptr;  // [1]
    GraphDev *d_desc = nullptr;
    BfsJob *d_bfs_jobs = nullptr;
    NodeJob *d_node_jobs = nullptr;           // kNodesPerJob nodes each
    int n_node_jobs = 0;
    NodeJob *d_hist_jobs = nullptr;           // hist_rows_per_job(K) rows each
    int n_hist_jobs = 0;
    int hist_jobs_k = 0;

    GraphDev desc() const
    {
        GraphDev d;
        memset(&d, 0, sizeof d);
        d.n = n;
        d.K = K;
        d.dmax = dmax;
        d.n_sigmas = n_sigmas;
        d.nnz = nnz;
        d.row_ptr = d_row_ptr;
        d.col = d_col;
        d.order = d_order;
        d.sell_col = d_sell_col;
        d.sell_off = d_sell_off;
        d.sell_deg = d_sell_deg;
        d.src = d_src;
        d.n_bfs = n_bfs;
        d.nnz_bfs = nnz_bfs;
        d.bfs_row_ptr = d_bfs_row_ptr ? d_bfs_row_ptr : d_row_ptr;
        d.bfs_col = d_bfs_row_ptr ? d_bfs_col : d_col;
        d.edges = d_edges;
        d.dist = d_dist;
        d.ld = d_ld;
        d.hist = d_hist;
        d.psi = d_psi;
        d.v = d_v;
        d.v64 = (pot_precision == QC_PREC_FP64ACC) ? d_v64 : nullptr;
        d.w64 = d_w64;
        d.u64 = d_u64;
        d.inv_a = d_inv_a;
        d.w32c = d_w32c;
        d.wbf16 = d_wbf16;
        d.parent = d_parent;
        d.status = d_status;
        d.recheck = d_recheck;
        return d;
    }
};


namespace qc {

qc_status from_hip(hipError_t e);

#define QC_TRY(expr)                                  \
    do {                                              \
        qc_status _st = (expr);                       \
        if (_st != QC_OK) return _st;                 \
    } while (0)
#define QC_HIP(expr) QC_TRY(from_hip(expr))

// Out-of-memory injection (qc_debug_alloc_fault): true when the device
// allocation being attempted is the one the armed countdown selects. Every
// device allocation path of the library asks first (the device allocator
// and the carving of arena regions).
bool alloc_fault_now();
// Device allocator blocks the library holds (hipMalloc'd, not yet freed).
void note_device_alloc(int delta);

// The library's device allocator: every hipMalloc of the library goes here.
inline qc_status device_malloc(void **p, size_t bytes)
{
    *p = nullptr;
    if (alloc_fault_now()) return QC_E_OOM;
    hipError_t e = hipMalloc(p, bytes ? bytes : 1);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return e == hipErrorOutOfMemory ? QC_E_OOM : QC_E_DEVICE;
    }
    note_device_alloc(1);
    return QC_OK;
}

inline void device_free(void *p)
{
    if (!p) return;
    (void)hipFree(p);
    note_device_alloc(-1);
}

template <class T>
qc_status dalloc(T **p, size_t count)
{
    return device_malloc((void **)p, (count ? count : 1) * sizeof(T));
}

template <class T>
void dfree(T *&p)
{
    device_free((void *)p);
    p = nullptr;
}

// Device buffer of a graph handle: from its arena region when it has one.
template <class T>
qc_status galloc(qc_graph g, T **p, size_t count)
{
    if (!g->bump_base) return dalloc(p, count);
    const size_t bytes = (((count ? count : 1) * sizeof(T)) + 255) & ~(size_t)255;
    if (alloc_fault_now() || g->bump_off + bytes > g->bump_size) {
        *p = nullptr;
        return QC_E_OOM;
    }
    *p = (T *)(g->bump_base + g->bump_off);
    g->bump_off += bytes;
    return QC_OK;
}

template <class T>
void gfree(qc_graph g, T *&p)
{
    if (!g->bump_base) dfree(p);
    p = nullptr;
}

// Upload a small host array synchronously (set-up only, never in a timed path).
template <class T>
qc_status upload(T *dst, const std::vector<T> &src)
{
    if (src.empty()) return QC_OK;
    return from_hip(hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
}

// One host array bound for the device.
struct HostSpan {
    void *dst;
    const void *src;
    size_t bytes;
};
template <class T>
HostSpan span_of(T *dst, const std::vector<T> &src)
{
    return HostSpan{(void *)dst, (const void *)src.data(), src.size() * sizeof(T)};
}
// Upload several host arrays (set-up only). In a handle's arena region,
// small arrays whose buffers follow one another (separated only by the
// region's 256-byte alignment padding, which no buffer uses) go as one copy
// from a staging buffer; large arrays, and every array outside a region,
// are copies of their own.
qc_status upload_group(qc_graph g, std::vector<HostSpan> spans);

inline hipStream_t as_stream(void *s) { return (hipStream_t)s; }

qc_status check_device(int *dev_out);
qc_status push_desc(qc_graph g, hipStream_t st);
qc_status ensure_hist_jobs(qc_graph g);
// Make p g's BFS plan (job list); `reorder`: also put the edges into the
// bank-aware order for p's batch width (when the graph qualifies).
qc_status set_plan(qc_graph g, const BfsPlan &p, bool reorder = true);
// Put the graph's edges back into rows-ascending order.
qc_status plain_edges(qc_graph g);
// Make the device edges carry row bias `bias` (bfs_row_bias of the launch
// shape about to read them): a no-op when they do; else, after the device
// has drained, an upload of the handle's current edge order with that bias.
qc_status ensure_edges(qc_graph g, int bias);
// ensure_edges for the launch shape of the handle's own plan.
qc_status check_edges(qc_graph g);
// Reachable (source, node) pairs of the batch of sources at positions
// s0..s0+bw-1 of the source order.
uint32_t batch_target(qc_graph g, int s0, int bw);
qc_status run_distances(qc_graph g, hipStream_t st);
qc_status ensure_sigma_buffers(qc_graph g, int S);
// Load the weight tables of a sigma list into g (no-op if already loaded).
qc_status load_sigmas(qc_graph g, const double *sigmas, int32_t n_sigmas, hipStream_t st);
// Device bytes a handle of n nodes, nnz CSR entries and n_sigmas widths
// carves from an arena region for the whole path (histograms sized for the
// largest row length); with_dist: including the n*n distance matrix,
// with_labels: including an [n_sigmas][n] label buffer. -1 out of range.
int64_t handle_footprint(int32_t n, int64_t nnz, int32_t n_sigmas, bool with_dist,
                         bool with_labels);
// Algorithm 4 on a created handle: distances (into dist_out, or the handle's
// own matrix when null), FP64-accumulated potentials, labels of every width
// into labels_out [n_sigmas][n]; waits for st and returns any latched error.
qc_status cluster_on_handle(qc_graph g, const double *sigmas, int32_t n_sigmas,
                            uint32_t tie_mode, int8_t *dist_out, float *psi_out, float *v_out,
                            int32_t *labels_out, hipStream_t st);
// Algorithm 4 in one call with every device buffer carved from the library's
// fixed per-device scratch (qc_noalloc.hip; one call per device at a time):
// QC_E_TOO_LARGE when the problem does not fit it. `stage_events`: let the
// stage timers record (they create HIP events, an allocation).
qc_status cluster_scratch(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                          const double *sigmas, int32_t n_sigmas, uint32_t tie_mode, int8_t *dist_out,
                          float *psi_out, float *v_out, int32_t *labels_out, hipStream_t st,
                          bool stage_events);
// Release a handle; `sync` waits for the whole device first (handles that
// live in an arena region are released after their own stream has drained).
void destroy(qc_graph g, bool sync = true);
// qc_graph_create with an optional arena region for every device buffer.
// `weights` (host, one per CSR entry, or null): integer edge weights 1..126.
// `hop_search` false: the handle's hop distances will never be searched (the
// real-weight path uses only its descent), so the host sweeps that order
// the search's sources are skipped.
qc_status create_graph(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                       uint32_t flags, hipStream_t stream, char *region, size_t region_bytes,
                       qc_graph *out, const uint8_t *weights = nullptr, bool hop_search = true);

}  // namespace qc
