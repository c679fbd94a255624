// Real edge weights (include/qc.h: qc_distances_real, qc_cluster_real):
// shortest paths per source on the GPU, then Algorithm 1 on the dense
// lengths and the descent along the graph's own edges.
#include <float.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "qc_handle.h"

using namespace qc;

namespace {

// The CSR and its weights checked for qc_distances_real: a canonical CSR,
// every weight finite and normal (>= FLT_MIN), an undirected edge's two
// entries of equal weight.
qc_status validate_real(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                        const float *weights, uint32_t flags, std::vector<int32_t> &rp,
                        std::vector<int32_t> &col)
{
    if (flags & ~(uint32_t)QC_GRAPH_DIRECTED) return QC_E_INVAL;
    if (n < 1 || n > kSsspMaxNodes) return QC_E_INVAL;
    if (nnz > 0 && !weights) return QC_E_INVAL;
    const bool directed = (flags & QC_GRAPH_DIRECTED) != 0;
    QC_TRY(validate_csr(n, nnz, row_ptr, col_idx, false, rp, col, directed));
    for (int64_t e = 0; e < nnz; ++e)
        if (!(weights[e] >= FLT_MIN) || !std::isfinite(weights[e])) return QC_E_INVAL;
    if (!directed) {
        for (int32_t v = 0; v < n; ++v)
            for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
                const int32_t u = col[e];
                const int32_t *b = col.data() + rp[u], *f = col.data() + rp[u + 1];
                const int32_t *it = std::lower_bound(b, f, v);
                if (it == f || *it != v || weights[it - col.data()] != weights[e])
                    return QC_E_NOT_SYMMETRIC;
            }
    }
    return QC_OK;
}

// The distances into dist (stride ld), on st, from device copies of the CSR
// and weights made here; waits for st before freeing them.
qc_status real_distances(int32_t n, const std::vector<int32_t> &rp, const std::vector<int32_t> &col,
                         const float *weights, float *dist, int64_t ld, hipStream_t st)
{
    // each entry's column and weight bits side by side: one 8-byte load per edge
    std::vector<uint32_t> cw(2 * col.size());
    for (size_t e = 0; e < col.size(); ++e) {
        cw[2 * e] = (uint32_t)col[e];
        memcpy(&cw[2 * e + 1], &weights[e], sizeof(float));
    }
    int32_t *d_rp = nullptr;
    uint32_t *d_cw = nullptr;
    qc_status s = dalloc(&d_rp, rp.size());
    if (s == QC_OK) s = dalloc(&d_cw, cw.size());
    if (s == QC_OK) s = upload(d_rp, rp);
    if (s == QC_OK) s = upload(d_cw, cw);
    if (s == QC_OK) {
        StageTimer t(QC_STAGE_SSSP, st);
        s = from_hip(launch_sssp(n, d_rp, d_cw, dist, ld, 0, n, st));
    }
    if (s == QC_OK) s = from_hip(hipStreamSynchronize(st));
    dfree(d_rp);
    dfree(d_cw);
    return s;
}

}  // namespace

extern "C" {

qc_status qc_distances_real(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                            const float *weights, uint32_t flags, float *dist_out, int64_t ld,
                            void *stream)
{
    if (!dist_out || ld < n) return QC_E_INVAL;
    std::vector<int32_t> rp, col;
    QC_TRY(validate_real(n, nnz, row_ptr, col_idx, weights, flags, rp, col));
    int dev = 0;
    QC_TRY(check_device(&dev));
    return real_distances(n, rp, col, weights, dist_out, ld, as_stream(stream));
}

qc_status qc_cluster_real(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                          const float *weights, uint32_t flags, const double *sigmas,
                          int32_t n_sigmas, uint32_t tie_mode, float *dist_out, double *psi_out,
                          double *v_out, int32_t *labels_out, void *stream)
{
    if (!labels_out || tie_mode > QC_TIE_MERGE) return QC_E_INVAL;
    QC_TRY(validate_sigmas(sigmas, n_sigmas));
    for (int32_t s = 0; s < n_sigmas; ++s)
        if (sigmas[s] < 1e-100) return QC_E_INVAL;
    std::vector<int32_t> rp, col;
    QC_TRY(validate_real(n, nnz, row_ptr, col_idx, weights, flags, rp, col));
    hipStream_t st = as_stream(stream);

    // The handle carries the descent's neighbour lists and the resident
    // potentials; its hop distances are never computed.
    qc_graph g = nullptr;
    QC_TRY(create_graph(n, nnz, row_ptr, col_idx, flags, st, nullptr, 0, &g, nullptr, false));
    float *dist = dist_out;
    double *psi = psi_out;
    qc_status s = QC_OK;
    if (!dist) s = dalloc(&dist, (size_t)n * n);
    if (s == QC_OK && !psi) s = dalloc(&psi, (size_t)n_sigmas * n);
    if (s == QC_OK) s = real_distances(n, rp, col, weights, dist, n, st);
    // Algorithm 1 on the lengths: FP64 V straight into the handle's FP64 V
    // (the values the descent re-decides near ties on), its FP32 copy in the
    // resident layout
    if (s == QC_OK) s = ensure_sigma_buffers(g, n_sigmas);
    if (s == QC_OK) {
        g->n_sigmas = n_sigmas;
        g->pot_precision = QC_PREC_FP64ACC;
        g->sigmas_loaded.clear();   // the weight tables are not this sigma list's
        s = push_desc(g, st);
    }
    if (s == QC_OK) {
        StageTimer t(QC_STAGE_DENSE, st);
        s = from_hip(launch_dense(dist, n, n, n, sigmas, n_sigmas, psi, g->d_v64, st));
    }
    if (s == QC_OK) s = from_hip(launch_v_resident(g->d_v64, n, n_sigmas, g->d_v, st));
    if (s == QC_OK && v_out)
        s = from_hip(hipMemcpyAsync(v_out, g->d_v64, sizeof(double) * n_sigmas * n,
                                    hipMemcpyDeviceToDevice, st));
    if (s == QC_OK) {
        g->have_pot = true;
        for (int32_t k = 0; k < n_sigmas && s == QC_OK; ++k)
            s = qc_ggd_labels(g, k, tie_mode, labels_out + (size_t)k * n, stream);
    }
    const qc_status sync = from_hip(hipStreamSynchronize(st));
    if (s == QC_OK) s = sync;
    if (!dist_out) dfree(dist);
    if (!psi_out) dfree(psi);
    destroy(g, false);
    return s;
}

}  // extern "C"
