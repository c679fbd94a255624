// qc_cluster_noalloc (include/qc.h): Algorithm 4 in one call with every
// device buffer carved from one fixed array of device memory, for callers
// that cannot allocate (code under HIP graph capture, tight serving loops).
//
// The array below is a device symbol: its name in host code is a host-side
// stand-in, not a device address. Its device address is looked up once per
// device with hipGetSymbolAddress (with that device current) and only that
// address is ever handed to kernels or copies.
#include <hip/hip_runtime.h>

#include <mutex>
#include <optional>
#include <vector>

#include "qc.h"
#include "qc_handle.h"

using namespace qc;

namespace {

constexpr size_t kScratchBytes = (size_t)QC_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size must keep 256-byte carving aligned");

static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_dev_mu[kMaxDevices];   // one call at a time per device: they share its scratch
char *g_scratch[kMaxDevices];       // device address of `scratch` per device (set under g_dev_mu)

// The device address of this device's copy of `scratch` (looked up on the
// first call on the device; the caller holds g_dev_mu[dev]).
qc_status scratch_ptr(int dev, char **out)
{
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return QC_E_DEVICE;
        }
        g_scratch[dev] = (char *)p;
    }
    *out = g_scratch[dev];
    return QC_OK;
}

}  // namespace

namespace qc {

qc_status cluster_scratch(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                          const double *sigmas, int32_t n_sigmas, uint32_t tie_mode, int8_t *dist_out,
                          float *psi_out, float *v_out, int32_t *labels_out, hipStream_t st,
                          bool stage_events)
{
    if (!labels_out || tie_mode > QC_TIE_MERGE) return QC_E_INVAL;
    if (dist_out && ((uintptr_t)dist_out) % 16) return QC_E_INVAL;
    QC_TRY(validate_sigmas(sigmas, n_sigmas));
    // everything the call keeps on the device (the matrix only when the
    // caller passes none), sized as for a serving request's arena region
    const int64_t need = handle_footprint(n, nnz, n_sigmas, dist_out == nullptr, false);
    if (need < 0) return QC_E_INVAL;
    if (need > (int64_t)kScratchBytes) return QC_E_TOO_LARGE;
    {
        // the CSR is checked on the host before any device work
        std::vector<int32_t> rp, col;
        QC_TRY(validate_csr(n, nnz, row_ptr, col_idx, false, rp, col));
    }
    int dev = 0;
    QC_TRY(check_device(&dev));
    if (dev >= kMaxDevices) return QC_E_DEVICE;
    std::lock_guard<std::mutex> lk(g_dev_mu[dev]);
    char *base = nullptr;
    QC_TRY(scratch_ptr(dev, &base));
    // without allocation no stage timer may run (each creates HIP events)
    std::optional<StageTimingOff> no_events;
    if (!stage_events) no_events.emplace();
    qc_graph g = nullptr;
    QC_TRY(create_graph(n, nnz, row_ptr, col_idx, 0, st, base, kScratchBytes, &g));
    const qc_status s =
        cluster_on_handle(g, sigmas, n_sigmas, tie_mode, dist_out, psi_out, v_out, labels_out, st);
    // the scratch is free for the next call only once the stream has passed
    // this one
    (void)hipStreamSynchronize(st);
    destroy(g, false);
    return s;
}

}  // namespace qc

extern "C" qc_status qc_cluster_noalloc(int32_t n, int64_t nnz, const int32_t *row_ptr,
                                        const int32_t *col_idx, const double *sigmas,
                                        int32_t n_sigmas, uint32_t tie_mode, int8_t *dist_out,
                                        float *psi_out, float *v_out, int32_t *labels_out,
                                        void *stream)
{
    return cluster_scratch(n, nnz, row_ptr, col_idx, sigmas, n_sigmas, tie_mode, dist_out, psi_out,
                           v_out, labels_out, as_stream(stream), false);
}
