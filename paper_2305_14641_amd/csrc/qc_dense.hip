// Algorithm 1 over a caller-supplied dense distance matrix: the workload of
// the paper's GPU experiment (Section 3.2, Fig. 3: fully connected graphs
// whose distances d_ij are real numbers, so no integer histogram applies).
//
// The kernel streams the matrix once per chunk of up to eight widths. One
// wavefront owns one row: its 64 lanes read consecutive 16-byte quads (a
// 1 KB coalesced load per wavefront per step), evaluate the Gaussian weight
// of every element for each width of the chunk and accumulate
// S2 = sum_j e_j and S1 = sum_j d_j^2 e_j in FP64; a butterfly reduction ends
// the row. Rows are independent and read once, so the launch needs no
// cross-workgroup locality and no XCD-aware tile order.
#include <limits.h>

#include "qc_internal.h"

#include "qc.h"

namespace qc {
namespace {

constexpr int kDenseWaves = 4;          // rows (one per wavefront) per workgroup
constexpr int kDenseMaxChunk = 8;       // widths evaluated per pass over the matrix
constexpr int kDenseUnroll = 4;         // 16-byte loads in flight per lane

struct DenseCoef {
    double c[kDenseMaxChunk];      // -log2(e) / a, a = (2 sigma) sigma
    double inv_a[kDenseMaxChunk];  // 1 / a
};

// 2^y for y = dd * c <= 0 in FP64: y = k + f with k = rint(y), |f| <= 1/2. 2^f comes
// from the FP32 hardware exp2 and the scaling by 2^k is done in FP64, so
// nothing underflows before FP64 would. Relative error: the rounding of f to
// FP32 (at most 2^-26 absolute, about 1.1e-8 relative after exp2) plus the
// exp2 instruction's own error (about one FP32 ulp). A false `keep` replaces
// k by INT_MIN, which scales the weight to an exact zero. The product y is
// rounded before the split (no fused multiply-add): for |y| >= 2^52 the
// rounded y is an integer, so f = 0 and k saturates to an exact zero weight,
// where a fused dd * c - k would leave the product's rounding error in f.
__device__ __forceinline__ double exp2_split(double dd, double c, bool keep)
{
#pragma clang fp contract(off)
    const double y = dd * c;
    const double k = rint(y);
    const float f = (float)(y - k);
    const int ki = keep ? (int)k : INT_MIN;
    return ldexp((double)__builtin_amdgcn_exp2f(f), ki);
}

template <int C>
struct DenseAcc {
    double s1[C];
    double s2[C];

    __device__ __forceinline__ void zero()
    {
#pragma unroll
        for (int c = 0; c < C; ++c) s1[c] = s2[c] = 0.0;
    }

    // One matrix entry. Only finite entries >= 0 are distances; anything else
    // (negative, NaN, infinite) means "no path" and adds nothing. With
    // sigma >= 1e-100 every product d^2 * c below is finite.
    __device__ __forceinline__ void add(float d, const DenseCoef &k)
    {
        const bool ok = (d >= 0.0f) && (d <= 3.40282347e38f);
        const double dd = ok ? (double)d * (double)d : 0.0;   // exact: 24-bit mantissas
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const double e = exp2_split(dd, k.c[c], ok);
            s2[c] += e;
            s1[c] = fma(dd, e, s1[c]);
        }
    }
};

template <int C, bool VEC>
__global__ __launch_bounds__(64 * kDenseWaves) void k_dense(
    const float *__restrict__ dist, int64_t n_rows, int64_t n_cols, int64_t ld, DenseCoef coef,
    int n_out, double *__restrict__ psi, double *__restrict__ v, int64_t out_ld)
{
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * kDenseWaves + (threadIdx.x >> 6);
    if (row >= n_rows) return;
    const float *r = dist + row * ld;
    DenseAcc<C> acc;
    acc.zero();
    int64_t j0 = 0;
    if (VEC) {
        // the row starts on a 16-byte boundary (checked by the launcher)
        const int64_t nq = n_cols >> 2;
        global_u4 rq = (global_u4)(const void *)r;
        int64_t q = lane;
        for (; q + 64 * (kDenseUnroll - 1) < nq; q += 64 * kDenseUnroll) {
            u32x4 x[kDenseUnroll];
#pragma unroll
            for (int u = 0; u < kDenseUnroll; ++u) x[u] = rq[q + 64 * u];
#pragma unroll
            for (int u = 0; u < kDenseUnroll; ++u) {
#pragma unroll
                for (int t = 0; t < 4; ++t) acc.add(__uint_as_float(x[u][t]), coef);
            }
        }
        for (; q < nq; q += 64) {
            const u32x4 x = rq[q];
#pragma unroll
            for (int t = 0; t < 4; ++t) acc.add(__uint_as_float(x[t]), coef);
        }
        j0 = nq << 2;
    }
    for (int64_t j = j0 + lane; j < n_cols; j += 64) acc.add(r[j], coef);

#pragma unroll
    for (int c = 0; c < C; ++c) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            acc.s1[c] += __shfl_xor(acc.s1[c], off, 64);
            acc.s2[c] += __shfl_xor(acc.s2[c], off, 64);
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if (c < n_out) {
                psi[c * out_ld + row] = acc.s2[c];
                v[c * out_ld + row] = coef.inv_a[c] * (acc.s1[c] / acc.s2[c]);
            }
        }
    }
}

template <int C>
hipError_t launch_chunk(bool vec, const float *dist, int64_t n_rows, int64_t n_cols, int64_t ld,
                        const DenseCoef &k, int n_out, double *psi, double *v, hipStream_t st)
{
    const dim3 grid((unsigned)((n_rows + kDenseWaves - 1) / kDenseWaves));
    const dim3 block(64 * kDenseWaves);
    if (vec)
        hipLaunchKernelGGL((k_dense<C, true>), grid, block, 0, st, dist, n_rows, n_cols, ld, k,
                           n_out, psi, v, n_rows);
    else
        hipLaunchKernelGGL((k_dense<C, false>), grid, block, 0, st, dist, n_rows, n_cols, ld, k,
                           n_out, psi, v, n_rows);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_dense(const float *dist, int64_t n_rows, int64_t n_cols, int64_t ld,
                        const double *sigmas, int n_sigmas, double *psi, double *v,
                        hipStream_t st)
{
    const double log2e = 1.4426950408889634;  // log2(e) rounded to FP64
    const bool vec = ((uintptr_t)dist % 16 == 0) && (ld % 4 == 0);
    for (int s0 = 0; s0 < n_sigmas; s0 += kDenseMaxChunk) {
        const int cnt = n_sigmas - s0 < kDenseMaxChunk ? n_sigmas - s0 : kDenseMaxChunk;
        const int C = cnt <= 1 ? 1 : cnt <= 2 ? 2 : cnt <= 4 ? 4 : 8;
        DenseCoef k;
        for (int c = 0; c < kDenseMaxChunk; ++c) {
            const double sigma = sigmas[s0 + (c < cnt ? c : cnt - 1)];
            const double a = (2.0 * sigma) * sigma;
            k.c[c] = -log2e / a;
            k.inv_a[c] = 1.0 / a;
        }
        double *p = psi + (int64_t)s0 * n_rows;
        double *q = v + (int64_t)s0 * n_rows;
        StageTimer timer(QC_STAGE_DENSE, st);
        hipError_t e;
        switch (C) {
        case 1: e = launch_chunk<1>(vec, dist, n_rows, n_cols, ld, k, cnt, p, q, st); break;
        case 2: e = launch_chunk<2>(vec, dist, n_rows, n_cols, ld, k, cnt, p, q, st); break;
        case 4: e = launch_chunk<4>(vec, dist, n_rows, n_cols, ld, k, cnt, p, q, st); break;
        default: e = launch_chunk<8>(vec, dist, n_rows, n_cols, ld, k, cnt, p, q, st); break;
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace qc
