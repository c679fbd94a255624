// C ABI of the library (include/qc.h): graph handles, resident device state,
// and the launch sequence of each call.
#include <hip/hip_runtime.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "qc.h"
#include "qc_host.h"
#include "qc_internal.h"

using namespace qc;

struct qc_graph_s {
    int device = 0;
    int32_t n = 0;
    int64_t nnz = 0;
    int32_t n_components = 0;
    BfsPlan plan{};

    // device CSR
    int32_t *d_row_ptr = nullptr;
    int32_t *d_col = nullptr;
    uint32_t *d_edges = nullptr;

    // distances and histograms
    int8_t *d_dist_owned = nullptr;   // library-owned matrix (n*n, 16-byte padded)
    int8_t *d_dist = nullptr;         // current resident matrix (owned or caller's)
    int32_t *d_hist = nullptr;
    int K = 0;
    int32_t dmax = -1;
    bool have_dist = false;

    // potentials
    int n_sigmas = 0;
    int pot_cap = 0;                  // sigmas the buffers below hold
    float *d_psi = nullptr, *d_v = nullptr;
    int32_t *d_parent = nullptr;
    double *d_w64 = nullptr, *d_u64 = nullptr, *d_inv_a = nullptr;
    float *d_w32c = nullptr;
    int w_cap = 0;                    // sigma*K entries the weight buffers hold
    bool have_pot = false;
    uint32_t pot_precision = 0;

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
        d.edges = d_edges;
        d.dist = d_dist;
        d.hist = d_hist;
        d.psi = d_psi;
        d.v = d_v;
        d.w64 = d_w64;
        d.u64 = d_u64;
        d.inv_a = d_inv_a;
        d.w32c = d_w32c;
        d.parent = d_parent;
        d.status = d_status;
        d.recheck = d_recheck;
        return d;
    }
};

namespace {

qc_status from_hip(hipError_t e)
{
    if (e == hipSuccess) return QC_OK;
    if (e == hipErrorOutOfMemory) return QC_E_OOM;
    return QC_E_DEVICE;
}

#define QC_TRY(expr)                                  \
    do {                                              \
        qc_status _st = (expr);                       \
        if (_st != QC_OK) return _st;                 \
    } while (0)
#define QC_HIP(expr) QC_TRY(from_hip(expr))

template <class T>
qc_status dalloc(T **p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return e == hipErrorOutOfMemory ? QC_E_OOM : QC_E_DEVICE;
    }
    return QC_OK;
}

template <class T>
void dfree(T *&p)
{
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

qc_status check_device(int *dev_out)
{
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
        (void)hipGetLastError();
        return QC_E_DEVICE;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return QC_E_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return QC_E_DEVICE;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return QC_E_DEVICE;
    *dev_out = dev;
    return QC_OK;
}

hipStream_t as_stream(void *s) { return (hipStream_t)s; }

qc_status push_desc(qc_graph g, hipStream_t st)
{
    return from_hip(launch_set_desc(g->d_desc, g->desc(), st));
}

// Upload a small host array synchronously (set-up only, never in a timed path).
template <class T>
qc_status upload(T *dst, const std::vector<T> &src)
{
    if (src.empty()) return QC_OK;
    return from_hip(hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
}

qc_status ensure_hist_jobs(qc_graph g)
{
    if (g->d_hist_jobs && g->hist_jobs_k == g->K) return QC_OK;
    dfree(g->d_hist_jobs);
    const int rows = hist_rows_per_job(g->K);
    std::vector<NodeJob> jobs;
    for (int i = 0; i < g->n; i += rows) jobs.push_back(NodeJob{0, i, 0});
    QC_TRY(dalloc(&g->d_hist_jobs, jobs.size()));
    QC_TRY(upload(g->d_hist_jobs, jobs));
    g->n_hist_jobs = (int)jobs.size();
    g->hist_jobs_k = g->K;
    return QC_OK;
}

// BFS into g->d_dist, then histograms. The first run waits to learn dmax.
qc_status run_distances(qc_graph g, hipStream_t st)
{
    QC_HIP(launch_fill_i32(g->d_status, 2, 0, st));
    QC_TRY(push_desc(g, st));
    QC_HIP(launch_bfs(g->plan.bw, g->plan.nw, g->d_desc, g->d_bfs_jobs, g->plan.n_batches, st));
    if (g->dmax < 0) {
        int32_t status[2];
        QC_HIP(hipMemcpyAsync(status, g->d_status, sizeof status, hipMemcpyDeviceToHost, st));
        QC_HIP(hipStreamSynchronize(st));
        if (status[1]) return QC_E_OVERFLOW;
        g->dmax = status[0];
        g->K = bins_for(g->dmax);
        dfree(g->d_hist);
        QC_TRY(dalloc(&g->d_hist, (size_t)g->n * g->K));
        QC_TRY(ensure_hist_jobs(g));
        QC_TRY(push_desc(g, st));
    }
    QC_HIP(launch_hist(g->K, g->d_desc, g->d_hist_jobs, g->n_hist_jobs, st));
    g->have_dist = true;
    return QC_OK;
}

qc_status ensure_sigma_buffers(qc_graph g, int S)
{
    if (S > g->pot_cap) {
        dfree(g->d_psi);
        dfree(g->d_v);
        dfree(g->d_parent);
        QC_TRY(dalloc(&g->d_psi, (size_t)S * g->n));
        QC_TRY(dalloc(&g->d_v, (size_t)S * g->n));
        QC_TRY(dalloc(&g->d_parent, (size_t)S * g->n));
        g->pot_cap = S;
    }
    if (S * g->K > g->w_cap) {
        dfree(g->d_w64);
        dfree(g->d_u64);
        dfree(g->d_inv_a);
        dfree(g->d_w32c);
        QC_TRY(dalloc(&g->d_w64, (size_t)S * g->K));
        QC_TRY(dalloc(&g->d_u64, (size_t)S * g->K));
        QC_TRY(dalloc(&g->d_inv_a, (size_t)S));
        QC_TRY(dalloc(&g->d_w32c, (size_t)S * g->K * 4));
        g->w_cap = S * g->K;
    }
    return QC_OK;
}

void destroy(qc_graph g)
{
    if (!g) return;
    (void)hipDeviceSynchronize();
    dfree(g->d_row_ptr);
    dfree(g->d_col);
    dfree(g->d_edges);
    dfree(g->d_dist_owned);
    dfree(g->d_hist);
    dfree(g->d_psi);
    dfree(g->d_v);
    dfree(g->d_parent);
    dfree(g->d_w64);
    dfree(g->d_u64);
    dfree(g->d_inv_a);
    dfree(g->d_w32c);
    dfree(g->d_status);
    dfree(g->d_recheck);
    dfree(g->d_desc);
    dfree(g->d_bfs_jobs);
    dfree(g->d_node_jobs);
    dfree(g->d_hist_jobs);
    delete g;
}

}  // namespace

extern "C" {

const char *qc_status_str(qc_status s)
{
    switch (s) {
    case QC_OK: return "QC_OK";
    case QC_E_INVAL: return "QC_E_INVAL: invalid argument";
    case QC_E_NOT_SYMMETRIC: return "QC_E_NOT_SYMMETRIC: CSR is not a canonical undirected adjacency";
    case QC_E_OOM: return "QC_E_OOM: out of device memory";
    case QC_E_DEVICE: return "QC_E_DEVICE: no gfx950 device or a HIP call failed";
    case QC_E_OVERFLOW: return "QC_E_OVERFLOW: a finite hop distance exceeds 126";
    case QC_E_STATE: return "QC_E_STATE: call order violated";
    case QC_E_BUSY: return "QC_E_BUSY: request does not fit the memory budget now";
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
    if (!out) return QC_E_INVAL;
    if (flags & ~(uint32_t)QC_GRAPH_CANONICALIZE) return QC_E_INVAL;
    std::vector<int32_t> rp, col;
    QC_TRY(validate_csr(n, nnz, row_ptr, col_idx, (flags & QC_GRAPH_CANONICALIZE) != 0, rp, col));
    int dev = 0;
    QC_TRY(check_device(&dev));

    qc_graph g = new qc_graph_s();
    g->device = dev;
    g->n = n;
    g->nnz = (int64_t)col.size();
    g->n_components = count_components(n, rp, col);
    g->plan = plan_bfs(n);
    hipStream_t st = as_stream(stream);

    std::vector<uint32_t> edges(g->nnz);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e)
            edges[e] = ((uint32_t)i << 16) | (uint32_t)col[e];
    std::vector<BfsJob> bjobs(g->plan.n_batches);
    for (int b = 0; b < g->plan.n_batches; ++b) bjobs[b] = BfsJob{0, b * g->plan.bw};
    std::vector<NodeJob> njobs;
    for (int i = 0; i < n; i += kNodesPerJob) njobs.push_back(NodeJob{0, i, 0});
    g->n_node_jobs = (int)njobs.size();

    qc_status st_ = QC_OK;
    auto fail = [&](qc_status s) { destroy(g); return s; };
    if ((st_ = dalloc(&g->d_row_ptr, rp.size())) || (st_ = dalloc(&g->d_col, col.size())) ||
        (st_ = dalloc(&g->d_edges, edges.size())) || (st_ = dalloc(&g->d_status, 2)) ||
        (st_ = dalloc(&g->d_recheck, 1)) || (st_ = dalloc(&g->d_desc, 1)) ||
        (st_ = dalloc(&g->d_bfs_jobs, bjobs.size())) || (st_ = dalloc(&g->d_node_jobs, njobs.size())))
        return fail(st_);
    if ((st_ = upload(g->d_row_ptr, rp)) || (st_ = upload(g->d_col, col)) ||
        (st_ = upload(g->d_edges, edges)) || (st_ = upload(g->d_bfs_jobs, bjobs)) ||
        (st_ = upload(g->d_node_jobs, njobs)))
        return fail(st_);
    if ((st_ = from_hip(launch_fill_u64(g->d_recheck, 1, st))) || (st_ = push_desc(g, st)))
        return fail(st_);
    *out = g;
    return QC_OK;
}

qc_status qc_graph_destroy(qc_graph g)
{
    if (!g) return QC_E_INVAL;
    destroy(g);
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
    } else {
        if (!g->d_dist_owned) QC_TRY(dalloc(&g->d_dist_owned, (size_t)g->n * g->n + 16));
        g->d_dist = g->d_dist_owned;
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
    if (precision > QC_PREC_FP32C) return QC_E_INVAL;
    hipStream_t st = as_stream(stream);
    if (!g->have_dist) QC_TRY(qc_distances(g, nullptr, nullptr, stream));

    std::vector<double> w64, u64, inv_a;
    std::vector<float> w32c;
    weight_tables(sigmas, n_sigmas, g->K, w64, u64, inv_a, w32c);
    QC_TRY(ensure_sigma_buffers(g, n_sigmas));
    // The weight tables are tiny; a synchronous upload keeps host buffers safe.
    QC_HIP(hipStreamSynchronize(st));
    QC_TRY(upload(g->d_w64, w64));
    QC_TRY(upload(g->d_u64, u64));
    QC_TRY(upload(g->d_inv_a, inv_a));
    QC_TRY(upload(g->d_w32c, w32c));
    g->n_sigmas = n_sigmas;
    QC_TRY(push_desc(g, st));
    QC_HIP(launch_potential((int)precision, g->K, g->d_desc, g->d_node_jobs, g->n_node_jobs,
                            psi_out, v_out, g->n, st));
    g->have_pot = true;
    g->pot_precision = precision;
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
    QC_HIP(launch_ggd_parent((int)tie_mode, g->d_desc, g->d_node_jobs, g->n_node_jobs, sigma_index,
                             1, st));
    QC_HIP(launch_pointer_jump(g->d_desc, g->d_node_jobs, 1, sigma_index, 1, labels_out, 0, st));
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

qc_status qc_graph_sync(qc_graph g, void *stream)
{
    if (!g) return QC_E_INVAL;
    hipStream_t st = as_stream(stream);
    QC_HIP(hipStreamSynchronize(st));
    int32_t status[2] = {0, 0};
    QC_HIP(hipMemcpy(status, g->d_status, sizeof status, hipMemcpyDeviceToHost));
    if (status[1]) return QC_E_OVERFLOW;
    return QC_OK;
}

}  // extern "C"
