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
// Out-edges a thread relaxes itself (more: a group of kSsspGroup lanes
// shares them).
constexpr int kSsspSmallDegree = 12;
// Lanes that share a queued node's edges (four nodes per wavefront at a time).
constexpr int kSsspGroup = 16;
// Edges whose loads a lane issues together.
constexpr int kSsspChunk = 4;
// Entries of the per-round queue of high-degree nodes (beyond it a node's
// thread relaxes its edges itself).
constexpr int kSsspQueue = 1024;

// Offer d(v) + w(e) for the edges e0 + k * stride < e1 (k = 0, 1, ...): a
// chunk's loads in flight together, then its LDS mins together, then a mark
// in `nxt` for every head whose length dropped.
__device__ __forceinline__ void relax_edges(float dv, int e0, int e1, int stride,
                                            const uint2 *__restrict__ cw, uint32_t *d, uint32_t *nxt,
                                            uint32_t *spare)
{
    for (int e = e0; e < e1; e += kSsspChunk * stride) {
        uint2 x[kSsspChunk];
#pragma unroll
        for (int k = 0; k < kSsspChunk; ++k)
            x[k] = (e + k * stride < e1) ? cw[e + k * stride] : make_uint2(0u, 0u);
        // a slot past the end offers 0xFFFFFFFF to the thread's own spare
        // word: an unsigned min with it changes nothing and never counts as a
        // drop, so the chunk's mins need no branches and are issued back to
        // back (and the lanes' spare words never collide)
        uint32_t cand[kSsspChunk], old[kSsspChunk];
        uint32_t *at[kSsspChunk];
#pragma unroll
        for (int k = 0; k < kSsspChunk; ++k) {
            const bool in = e + k * stride < e1;
            cand[k] = in ? __float_as_uint(dv + __uint_as_float(x[k].y)) : 0xFFFFFFFFu;
            at[k] = in ? &d[x[k].x] : spare;
        }
#pragma unroll
        for (int k = 0; k < kSsspChunk; ++k)
            old[k] = __hip_atomic_fetch_min(at[k], cand[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
        for (int k = 0; k < kSsspChunk; ++k)
            if (cand[k] < old[k])
                __hip_atomic_fetch_or(&nxt[x[k].x >> 5], 1u << (x[k].x & 31), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

template <int MAXN, int T>
__global__ __launch_bounds__(T) void k_sssp(int n, const int32_t *__restrict__ row_ptr,
                                            const uint2 *__restrict__ cw, float *__restrict__ dist,
                                            int64_t ld, int src0)
{
    constexpr int kWords = MAXN / 32;
    constexpr int kWaves = T / 64;
    __shared__ uint32_t d[MAXN];
    __shared__ uint32_t cur[kWords];
    __shared__ uint32_t nxt[kWords];
    __shared__ int32_t queue[kSsspQueue];
    __shared__ int32_t queued;
    __shared__ uint32_t spare[T];   // each thread's target for unused chunk slots
    const int s = src0 + (int)blockIdx.x;
    const int tid = (int)threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int nw = (n + 31) / 32;
    // thread tid owns nodes [v0, v1): consecutive, so a round reads the one
    // or two bitmap words that cover them
    const int per = (n + T - 1) / T;
    const int v0 = min(n, tid * per), v1 = min(n, v0 + per);
    for (int v = tid; v < n; v += T) d[v] = kInfBits;
    for (int i = tid; i < nw; i += T) {
        cur[i] = 0u;
        nxt[i] = 0u;
    }
    if (tid == 0) queued = 0;
    __syncthreads();
    if (tid == 0) {
        d[s] = 0u;
        cur[s >> 5] = 1u << (s & 31);
    }
    __syncthreads();
    for (;;) {
        // every node whose length dropped in the previous round offers it
        // along its out-edges (the length may drop again meanwhile: any
        // value read is a valid path sum, and a drop makes the node active
        // in the next round)
        for (int v = v0; v < v1;) {
            const uint32_t word = cur[v >> 5];
            const int top = min(v1, (v | 31) + 1);
            uint32_t bits = word >> (v & 31);
            if (top - v < 32) bits &= (1u << (top - v)) - 1u;
            while (bits) {
                // up to four active nodes at a time, their row bounds loaded together
                int u[4], e0[4], e1[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    u[k] = bits ? v + __builtin_ctz(bits) : -1;
                    bits &= bits - 1u;
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    e0[k] = u[k] >= 0 ? row_ptr[u[k]] : 0;
                    e1[k] = u[k] >= 0 ? row_ptr[u[k] + 1] : 0;
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (u[k] < 0) break;
                    if (e1[k] - e0[k] > kSsspSmallDegree) {
                        const int slot = __hip_atomic_fetch_add(&queued, 1, __ATOMIC_RELAXED,
                                                                __HIP_MEMORY_SCOPE_WORKGROUP);
                        if (slot < kSsspQueue) {
                            queue[slot] = u[k];
                            continue;
                        }
                    }
                    const float du = __uint_as_float(
                        __hip_atomic_load(&d[u[k]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
                    relax_edges(du, e0[k], e1[k], 1, cw, d, nxt, &spare[tid]);
                }
            }
            v = top;
        }
        __syncthreads();
        // the queued high-degree nodes: four per wavefront at a time, each
        // node's edges spread over a group of 16 lanes (most queued nodes
        // have fewer than 64 edges, which would leave a whole wavefront's
        // lanes idle)
        const int nq = min(queued, kSsspQueue);
        constexpr int kPerWave = 64 / kSsspGroup;
        for (int j = wave * kPerWave + lane / kSsspGroup; j < nq; j += kWaves * kPerWave) {
            const int u = queue[j];
            const int e0 = row_ptr[u], e1 = row_ptr[u + 1];
            const float du = __uint_as_float(
                __hip_atomic_load(&d[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
            relax_edges(du, e0 + lane % kSsspGroup, e1, kSsspGroup, cw, d, nxt, &spare[tid]);
        }
        __syncthreads();
        int any = 0;
        for (int i = tid; i < nw; i += T) {
            const uint32_t x = nxt[i];
            cur[i] = x;
            nxt[i] = 0u;
            any |= (x != 0u);
        }
        if (tid == 0) queued = 0;
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
hipError_t launch_sssp_t(int n, const int32_t *row_ptr, const uint2 *cw, float *dist, int64_t ld,
                         int src0, int count, hipStream_t stream)
{
    hipLaunchKernelGGL((k_sssp<MAXN, T>), dim3(count), dim3(T), 0, stream, n, row_ptr, cw, dist, ld,
                       src0);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sssp(int n, const int32_t *row_ptr, const uint32_t *col_w, float *dist, int64_t ld,
                       int src0, int count, hipStream_t stream)
{
    if (n < 1 || n > kSsspMaxNodes || src0 < 0 || count < 0 || src0 + count > n || ld < n)
        return hipErrorInvalidValue;
    if (count == 0) return hipSuccess;
    const uint2 *cw = (const uint2 *)col_w;
    if (n <= 4096) return launch_sssp_t<4096, 256>(n, row_ptr, cw, dist, ld, src0, count, stream);
    if (n <= 8192) return launch_sssp_t<8192, 512>(n, row_ptr, cw, dist, ld, src0, count, stream);
    if (n <= 16384) return launch_sssp_t<16384, 1024>(n, row_ptr, cw, dist, ld, src0, count, stream);
    return launch_sssp_t<32768, 1024>(n, row_ptr, cw, dist, ld, src0, count, stream);
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
