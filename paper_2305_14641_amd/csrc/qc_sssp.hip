// Shortest paths under real edge weights (Section 3.1: a path's length is the
// sum of its edges' weights), one source per workgroup, and the conversion
// of a dense FP64 potential into the resident layout the descent reads.
//
// A path's length is summed in binary32 from the source outward, each partial
// sum rounded to nearest, and d(s, v) is the least such sum over all paths.
// The workgroup keeps its source's row of tentative lengths in LDS (the bits
// of a non-negative float order like the float, so an unsigned LDS min is a
// float min) and relaxes in rounds: every node whose length dropped in the
// previous round (a bit in `cur`) offers d(v) + w to each out-neighbour u
// with one LDS min; a drop marks u in `nxt`. The search ends after a round in
// which nothing dropped. The least sum is what any such order reaches: a
// relaxation only ever produces the sum of an actual path, and once nothing
// drops, every node on a least path holds at most that path's partial sum
// (rounding is monotone), so the order of relaxations inside a round does not
// change the result.
#include <hip/hip_runtime.h>

#include "qc_internal.h"

namespace qc {

namespace {

constexpr uint32_t kInfBits = 0x7F800000u;   // +infinity: unreached

template <int MAXN, int T>
__global__ __launch_bounds__(T) void k_sssp(int n, const int32_t *__restrict__ row_ptr,
                                            const int32_t *__restrict__ col,
                                            const float *__restrict__ w, float *__restrict__ dist,
                                            int64_t ld, int src0)
{
    constexpr int kWords = MAXN / 32;
    __shared__ uint32_t d[MAXN];
    __shared__ uint32_t cur[kWords];
    __shared__ uint32_t nxt[kWords];
    const int s = src0 + (int)blockIdx.x;
    const int tid = (int)threadIdx.x;
    const int nw = (n + 31) / 32;
    for (int v = tid; v < n; v += T) d[v] = kInfBits;
    for (int i = tid; i < nw; i += T) {
        cur[i] = 0u;
        nxt[i] = 0u;
    }
    __syncthreads();
    if (tid == 0) {
        d[s] = 0u;
        cur[s >> 5] = 1u << (s & 31);
    }
    __syncthreads();
    for (;;) {
        for (int v = tid; v < n; v += T) {
            if (!((cur[v >> 5] >> (v & 31)) & 1u)) continue;
            // the length may drop again during the round (another node's
            // offer): reading either value is a valid path sum, and a drop
            // puts v into the next round anyway
            const float dv =
                __uint_as_float(__hip_atomic_load(&d[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
            const int e1 = row_ptr[v + 1];
            for (int e = row_ptr[v]; e < e1; ++e) {
                const int u = col[e];
                const uint32_t cand = __float_as_uint(dv + w[e]);
                const uint32_t old = __hip_atomic_fetch_min(&d[u], cand, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_WORKGROUP);
                if (cand < old)
                    __hip_atomic_fetch_or(&nxt[u >> 5], 1u << (u & 31), __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
        __syncthreads();
        int any = 0;
        for (int i = tid; i < nw; i += T) {
            const uint32_t x = nxt[i];
            cur[i] = x;
            nxt[i] = 0u;
            any |= (x != 0u);
        }
        if (!__syncthreads_or(any)) break;
    }
    float *__restrict__ row = dist + (int64_t)s * ld;
    for (int v = tid; v < n; v += T) row[v] = __uint_as_float(d[v]);
}

// v32[v_index(n, s, i)] = (float)v64[s * n + i]: the descent's FP32 copy of a
// potential, sigma groups of kVGroup interleaved by node.
__global__ __launch_bounds__(256) void k_v_resident(const double *__restrict__ v64, int n, int n_sigmas,
                                                    float *__restrict__ v32)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= (int64_t)n * n_sigmas) return;
    const int s = (int)(k / n), i = (int)(k % n);
    v32[v_index(n, s, i)] = (float)v64[k];
}

template <int MAXN, int T>
hipError_t launch_sssp_t(int n, const int32_t *row_ptr, const int32_t *col, const float *w,
                         float *dist, int64_t ld, int src0, int count, hipStream_t stream)
{
    hipLaunchKernelGGL((k_sssp<MAXN, T>), dim3(count), dim3(T), 0, stream, n, row_ptr, col, w, dist,
                       ld, src0);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sssp(int n, const int32_t *row_ptr, const int32_t *col, const float *w, float *dist,
                       int64_t ld, int src0, int count, hipStream_t stream)
{
    if (n < 1 || n > kSsspMaxNodes || src0 < 0 || count < 0 || src0 + count > n || ld < n)
        return hipErrorInvalidValue;
    if (count == 0) return hipSuccess;
    if (n <= 4096) return launch_sssp_t<4096, 256>(n, row_ptr, col, w, dist, ld, src0, count, stream);
    if (n <= 8192) return launch_sssp_t<8192, 512>(n, row_ptr, col, w, dist, ld, src0, count, stream);
    if (n <= 16384) return launch_sssp_t<16384, 1024>(n, row_ptr, col, w, dist, ld, src0, count, stream);
    return launch_sssp_t<32768, 1024>(n, row_ptr, col, w, dist, ld, src0, count, stream);
}

hipError_t launch_v_resident(const double *v64, int n, int n_sigmas, float *v32, hipStream_t stream)
{
    const int64_t total = (int64_t)n * n_sigmas;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_v_resident, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, v64, n,
                       n_sigmas, v32);
    return hipGetLastError();
}

}  // namespace qc
