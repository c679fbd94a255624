// HIP kernels (gfx950) of the graph Quantum Clustering hot path:
//   k_bfs        all-pairs hop distances by bit-parallel multi-source BFS
//   k_hist       per-node distance histograms from the int8 distance rows
//   k_potential  psi (Eq. 2) and V (Algorithm 1) from histogram x exp weights
//   k_ggd_parent Graph Gradient Descent step (Algorithm 2) with FP64 re-check
//   k_jump       find the centre of every node (Algorithm 3) by pointer jumping
#include "qc_internal.h"

#include <float.h>

namespace qc {

hipError_t launch_bfs(int bw, int nw, int planes, int shape, const GraphDev *graphs,
                      const BfsJob *jobs, int n_jobs, hipStream_t stream)
{
    if (n_jobs <= 0) return hipSuccess;
    switch (bw) {
    case 4: return launch_bfs_bw<4>(nw, planes, shape, graphs, jobs, n_jobs, stream);
    case 8: return launch_bfs_bw<8>(nw, planes, shape, graphs, jobs, n_jobs, stream);
    case 16: return launch_bfs_bw<16>(nw, planes, shape, graphs, jobs, n_jobs, stream);
    case 32: return launch_bfs_bw<32>(nw, planes, shape, graphs, jobs, n_jobs, stream);
    case 64: return launch_bfs_bw<64>(nw, planes, shape, graphs, jobs, n_jobs, stream);
    default: return hipErrorInvalidValue;
    }
}

// ===========================================================================
// Distance histograms h[i][k] = #{j : d(i,j) = k} from resident int8 rows.
// One wavefront per row (RPW rows per wavefront per job). Every lane counts
// into its own LDS column (bins[k][lane]), so increments never collide, with
// one extra bin that absorbs unreachable entries (-1 read as 255), which keeps
// the per-byte work branch-free: extract and clamp the byte, form the bin's
// address, one no-return LDS add. The lanes then sum each bin over its 64
// columns with 16-byte reads and clear the bins for the next row. (Two bins
// per word as 16-bit halves would halve the LDS but double the per-byte ALU
// work.) Loads are aligned 16-byte chunks in two sets of kHistDepth per lane
// that take turns: one set is counted while the other's loads are in flight
// (sets of 2 / 3 / 4 / 6 chunks measured 1.18 / 1.19 / 1.23 / 1.32 ms per
// sweep step).
// ===========================================================================

#ifndef QC_HIST_DEPTH
#define QC_HIST_DEPTH 2
#endif
constexpr int kHistDepth = QC_HIST_DEPTH;

template <int K, int WAVES, int RPW>
__global__ __launch_bounds__(WAVES * 64) void k_hist(const GraphDev *__restrict__ graphs,
                                                     const NodeJob *__restrict__ jobs)
{
    __shared__ __attribute__((aligned(16))) uint32_t bins[WAVES][K + 1][64];
    const NodeJob job = jobs[blockIdx.x];
    const GraphDev &G = graphs[job.g];
    const int n = G.n;
    const int wave = threadIdx.x / 64;
    const int lane = threadIdx.x % 64;
    const int8_t *__restrict__ base = G.dist;
    // bytes up to the end of the last row (rows are G.ld apart)
    const int64_t total = (int64_t)(n - 1) * G.ld + n;
    const bool vec_ok = total >= 16;
    const int64_t last_whole = vec_ok ? ((total - 16) & ~(int64_t)15) : 0;
    constexpr int64_t kStep = 64 * 16;   // bytes one wavefront covers per chunk
    uint32_t *const col = &bins[wave][0][lane];
    // The bins are this wavefront's own, so its lanes only need ordering
    // among themselves (counts before the column sum, the sum's clears
    // before the next row's counts): a wavefront-scope fence, no workgroup
    // barrier, and the workgroup's wavefronts run their rows independently.
    auto wave_sync = [] {
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
    };
    // the wavefront's bins as 16-byte quads, 16 per bin row
    constexpr int kQuads = 16;
    uint4 *const quads = (uint4 *)&bins[wave][0][0];
    const uint4 zero4 = make_uint4(0u, 0u, 0u, 0u);
    for (int i = lane; i < (K + 1) * kQuads; i += 64) quads[i] = zero4;
    wave_sync();

    // bin min(u, K) of this lane: 256 bytes per bin row (one shift-add)
    auto count = [&](uint32_t u) {
        __hip_atomic_fetch_add((uint32_t *)((char *)col + (min(u, (uint32_t)K) << 8)), 1u,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };

    for (int rr = 0; rr < RPW; ++rr) {
        const int row = __builtin_amdgcn_readfirstlane(job.i0 + rr * WAVES + wave);
        const bool active = row < n;
        if (active && vec_ok) {
            const int64_t r0 = (int64_t)row * G.ld;
            const int64_t r1 = r0 + n;
            const int64_t wb0 = r0 & ~(int64_t)15;   // the wavefront's first chunk
            const int64_t first = wb0 + lane * 16;
            // Whole 16-byte chunks inside the row are counted in the loop; a
            // chunk cut by a row end has its bytes set to all ones, which the
            // clamp sends to the junk bin K, so the byte loop has no selects
            // or branches. Loads past the row's last chunk re-read that chunk
            // (an L2 hit); a whole chunk inside the row is never clamped.
            const int64_t last_c = min((r1 - 1) & ~(int64_t)15, last_whole);
            auto load = [&](u32x4 *set, int64_t c) {
#pragma unroll
                for (int u = 0; u < kHistDepth; ++u)
                    set[u] = *(global_u4)(base + min(c + u * kStep, last_c));
                // keeps the loads here: the compiler would otherwise sink them
                // past the exit test, next to their use
                asm volatile("" ::: "memory");
            };
            auto count_set = [&](const u32x4 *set, int64_t c) {
#pragma unroll
                for (int u = 0; u < kHistDepth; ++u) {
                    const int64_t cc = c + u * kStep;
                    const uint32_t jm = (cc >= r0 && cc + 16 <= r1) ? 0u : 0xFFFFFFFFu;
                    const uint32_t wv[4] = {set[u].x | jm, set[u].y | jm, set[u].z | jm,
                                            set[u].w | jm};
#pragma unroll
                    for (int p = 0; p < 16; ++p) count((wv[p / 4] >> (8 * (p % 4))) & 0xFFu);
                }
            };
            // Two register sets take turns: one is counted while the other's
            // loads are in flight (a copy from one to the other would make
            // the compiler wait for every load before the next round). The
            // exits test the wavefront's first chunk, so no set that starts
            // past the row is counted.
            constexpr int64_t kHalf = kHistDepth * kStep;
            u32x4 a[kHistDepth], b[kHistDepth];
            load(a, first);
            for (int64_t c = first, wb = wb0;; c += 2 * kHalf, wb += 2 * kHalf) {
                load(b, c + kHalf);
                count_set(a, c);
                if (wb + kHalf >= r1) break;
                load(a, c + 2 * kHalf);
                count_set(b, c + kHalf);
                if (wb + 2 * kHalf >= r1) break;
            }
            // the row's bytes outside whole chunks: at most 15 at each end
            const int64_t head_end = min(r1, (r0 + 15) & ~(int64_t)15);
            const int64_t tail_begin = max(r1 & ~(int64_t)15, head_end);
            const int64_t f = (lane < 16) ? r0 + lane : tail_begin + (lane - 16);
            if ((lane < 16 && f < head_end) || (lane >= 16 && lane < 32 && f < r1))
                count((uint32_t)(uint8_t)base[f]);
        } else if (active) {
            // a matrix of fewer than 16 bytes: byte loads
            const int64_t r0 = (int64_t)row * G.ld;
            for (int64_t f = r0 + lane; f < r0 + n; f += 64) count((uint32_t)(uint8_t)base[f]);
        }
        wave_sync();
        if (active) {
            // bin k = the sum of its 64 columns: kLanes lanes per bin each add
            // a share of its quads (rotated by lane, so the 16-byte reads of
            // eight consecutive lanes cover all banks) and clear them for the
            // next row; the next row's counts come after the fence below
            int32_t *__restrict__ h = G.hist + (int64_t)row * G.K;
            constexpr int kLanes = (K >= 64) ? 1 : 64 / K;
            constexpr int kShare = kQuads / kLanes;
            const int part = lane % kLanes;
            for (int k = lane / kLanes; k < K; k += 64 / kLanes) {
                uint32_t sum = 0;
#pragma unroll
                for (int i = 0; i < kShare; ++i) {
                    const int q = k * kQuads + part * kShare + (i + lane) % kShare;
                    const uint4 x = quads[q];
                    sum += x.x + x.y + x.z + x.w;
                    quads[q] = zero4;
                }
                if constexpr (kLanes == 2) sum += (uint32_t)__shfl_xor((int)sum, 1);
                if (part == 0) h[k] = (int32_t)sum;
            }
            for (int k = K + lane; k < G.K; k += 64) h[k] = 0;
        }
        wave_sync();
    }
}

// Workgroup shapes of the histogram pass per row length: the 32 rows of a
// job split over W wavefronts of 32 / W rows each (the LDS bins are
// W x (K + 1) x 256 bytes). Variant 0 is the default (about 66 KB of bins);
// 1 halves the wavefronts, 2 doubles them.
int hist_waves(int K, int variant)
{
    const int base = (K == 32) ? 8 : (K == 64) ? 4 : 2;
    return variant == 1 ? base / 2 : variant == 2 ? base * 2 : base;
}

template <int K, int W>
static void launch_hist_w(const GraphDev *graphs, const NodeJob *jobs, int n_jobs, hipStream_t stream)
{
    static_assert(W * (32 / W) == 32, "a job is 32 rows");
    hipLaunchKernelGGL((k_hist<K, W, 32 / W>), dim3(n_jobs), dim3(W * 64), 0, stream, graphs, jobs);
}

hipError_t launch_hist(int K, const GraphDev *graphs, const NodeJob *jobs, int n_jobs,
                       hipStream_t stream, int variant)
{
    if (n_jobs <= 0) return hipSuccess;
    if (variant < 0 || variant > 2) return hipErrorInvalidValue;
    const int w = hist_waves(K, variant);
    switch (K * 100 + w) {
    case 3204: launch_hist_w<32, 4>(graphs, jobs, n_jobs, stream); break;
    case 3208: launch_hist_w<32, 8>(graphs, jobs, n_jobs, stream); break;
    case 3216: launch_hist_w<32, 16>(graphs, jobs, n_jobs, stream); break;
    case 6402: launch_hist_w<64, 2>(graphs, jobs, n_jobs, stream); break;
    case 6404: launch_hist_w<64, 4>(graphs, jobs, n_jobs, stream); break;
    case 6408: launch_hist_w<64, 8>(graphs, jobs, n_jobs, stream); break;
    case 12801: launch_hist_w<128, 1>(graphs, jobs, n_jobs, stream); break;
    case 12802: launch_hist_w<128, 2>(graphs, jobs, n_jobs, stream); break;
    case 12804: launch_hist_w<128, 4>(graphs, jobs, n_jobs, stream); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ===========================================================================
// psi and V (Eq. 2; Algorithm 1 regrouped by distance value):
//   psi_i = sum_k h[i][k] w_k,  V_i = (1/a) sum_k k^2 h[i][k] w_k / psi_i,
//   w_k = exp(-k^2 / a),  a = 2 sigma^2.
// One thread per node, all sigmas of the graph; the histogram row stays in
// registers.
// FP64ACC: the canonical FP64 evaluation — S2 = sum h_k*w_k and
//   S1 = sum (k^2 h_k)*w_k in ascending k from +0.0, each product and sum
//   rounded separately (no contraction), V = (1/a)*(S1/S2). psi and V are
//   returned as the FP32 roundings of S2 and V; V itself stays resident in
//   FP64 for the descent's near-tie decisions. These are the IEEE operations,
//   in the same order, of the CPU oracle's canonical form.
// FP32C: FP32 only, error-free products (FMA) and TwoSum accumulation, the
//   weights split as hi + lo FP32 pairs.
// ===========================================================================

__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e)
{
    s = a + b;
    const float z = s - a;
    e = (a - (s - z)) + (b - z);
}

// A read-only table whose loads are all uniform: through the constant
// address space they become scalar loads into scalar registers, which
// leaves the vector registers to the counts and sums.
typedef const __attribute__((address_space(4))) double cdouble;

// A copy of a count the compiler cannot see through: its conversion to FP64
// is redone inside the loop over sigma groups instead of being hoisted out
// of it, where the 2 x K converted values (and their k^2 multiples) would
// hold most of the registers.
__device__ __forceinline__ int32_t fresh(int32_t x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// The canonical FP64 sums of Q consecutive sigmas from s, independent
// chains each in ascending k: S2 += h_k * w_k and S1 += (k^2 h_k) * w_k from
// +0.0, every product and sum rounded on its own. Bins go in chunks of 8 up
// to the largest distance (a uniform exit: every node of a job belongs to
// one graph) with a chunk's weights loaded together; bins of the last chunk
// past the largest distance hold a zero count, whose +0.0 terms leave the
// sums unchanged. w64 rows have K entries.
template <int K, int Q>
__device__ __forceinline__ void canonical_group(const int32_t (&h)[K], int kmax,
                                                const cdouble *w64, int s, double (&a2)[Q],
                                                double (&a1)[Q])
{
#pragma clang fp contract(off)
#pragma unroll
    for (int q = 0; q < Q; ++q) a2[q] = a1[q] = 0.0;
#pragma unroll
    for (int kc = 0; kc < K; kc += 8) {
        if (kc >= kmax) break;
        double w[8][Q];
#pragma unroll
        for (int j = 0; j < 8; ++j)
#pragma unroll
            for (int q = 0; q < Q; ++q) w[j][q] = w64[(int64_t)(s + q) * K + kc + j];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = kc + j;
            const double hk = (double)fresh(h[k]);
            const double kk = (double)(k * k) * hk;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                a2[q] = a2[q] + hk * w[j][q];
                a1[q] = a1[q] + kk * w[j][q];
            }
        }
    }
}

__device__ __forceinline__ double canonical_ratio(double s1, double s2, double inv_a)
{
#pragma clang fp contract(off)
    return inv_a * (s1 / s2);
}

constexpr int kPotSigmas = 4;

template <int K, int PREC>
__global__ __launch_bounds__(256) void k_potential(const GraphDev *__restrict__ graphs,
                                                   const NodeJob *__restrict__ jobs,
                                                   float *__restrict__ psi_out,
                                                   float *__restrict__ v_out, int64_t out_ld)
{
    const NodeJob job = jobs[blockIdx.x];
    const GraphDev &G = graphs[job.g];
    const int n = G.n;
    const int i = job.i0 + (int)threadIdx.x;
    if (i >= n) return;
    const int kmax = min(G.dmax + 1, K);
    const int32_t *__restrict__ hrow = G.hist + (int64_t)i * G.K;
    // the whole row (K == G.K: every graph of a launch has this row length)
    // in 16-byte loads, then the bins past the largest distance zeroed
    int32_t h[K];
#pragma unroll
    for (int c = 0; c < K / 4; ++c) {
        const u32x4 q = ((global_u4)hrow)[c];
        h[4 * c + 0] = (int32_t)q.x;
        h[4 * c + 1] = (int32_t)q.y;
        h[4 * c + 2] = (int32_t)q.z;
        h[4 * c + 3] = (int32_t)q.w;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) h[k] = (k < kmax) ? h[k] : 0;

    // one (node, sigma) result: FP32 psi and V for the caller (or resident
    // psi when the caller takes none), the resident V, and with FP64
    // accumulation the resident FP64 V
    auto store = [&](int s, float psi32, float v32) {
        const int64_t o = (int64_t)s * n + i;
        G.v[v_index(n, s, i)] = v32;
        const int64_t ou = job.out_off + (int64_t)s * out_ld + i;
        if (psi_out) psi_out[ou] = psi32;
        else G.psi[o] = psi32;
        if (v_out) v_out[ou] = v32;
    };
    int s = 0;
    if constexpr (PREC == 0) {
        // kPotSigmas sigmas at a time (rows of up to 64 bins): their sums
        // are independent chains (each in the canonical order), so the FP64
        // adds of one sigma wait on their predecessors while the others'
        // issue
        constexpr int Q = (K <= 64) ? kPotSigmas : 1;
        const cdouble *w64 = (const cdouble *)G.w64;
        for (; s + Q <= G.n_sigmas; s += Q) {
            double a2[Q], a1[Q];
            canonical_group<K, Q>(h, kmax, w64, s, a2, a1);
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const double v64 = canonical_ratio(a1[q], a2[q], G.inv_a[s + q]);
                G.v64[(int64_t)(s + q) * n + i] = v64;
                store(s + q, (float)a2[q], (float)v64);
            }
        }
        for (; s < G.n_sigmas; ++s) {
            double a2[1], a1[1];
            canonical_group<K, 1>(h, kmax, w64, s, a2, a1);
            const double v64 = canonical_ratio(a1[0], a2[0], G.inv_a[s]);
            G.v64[(int64_t)s * n + i] = v64;
            store(s, (float)a2[0], (float)v64);
        }
    } else {
        for (; s < G.n_sigmas; ++s) {
            const float *__restrict__ wt = G.w32c + (int64_t)s * G.K * 4;
            float ps = 0.f, pe = 0.f, qs = 0.f, qe = 0.f;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (k < kmax) {
                    const float hk = (float)h[k];   // exact: counts < 2^24
                    const float whi = wt[4 * k + 0], wlo = wt[4 * k + 1];
                    const float uhi = wt[4 * k + 2], ulo = wt[4 * k + 3];
                    // TwoProduct(hk, hi) + hk*lo, then TwoSum into (sum, err)
                    float t = hk * whi;
                    float te = __fmaf_rn(hk, whi, -t) + hk * wlo;
                    float s1, e1;
                    two_sum(ps, t, s1, e1);
                    ps = s1;
                    pe += e1 + te;
                    t = hk * uhi;
                    te = __fmaf_rn(hk, uhi, -t) + hk * ulo;
                    two_sum(qs, t, s1, e1);
                    qs = s1;
                    qe += e1 + te;
                }
            }
            const float p = ps + pe;
            const float q = qs + qe;
            store(s, p, __fdiv_rn(q, p));
        }
    }
}

// BF16 matrix-core variant: the product [weights x bins] . [bins x nodes]
// on v_mfma_f32_16x16x32_bf16, accumulated in FP32. For a tile of 16 nodes,
// A = 16 weight columns (8 sigmas x {psi weight w_k, V numerator weight
// k^2 w_k / a}) by 32 bins and B = the 16 histogram rows (32 bins each), both
// rounded to BF16. BF16 keeps 8 significant bits, so psi and V carry about
// 1e-3 relative error: an approximate sweep, never used for the descent.
// The weight fragments do not depend on the graph, so each workgroup builds
// them once in LDS (for 32 sigmas at a time: 16 bytes per lane and column
// block) and every tile reads them with one 16-byte LDS read per MFMA. The
// output layout puts one node per lane column: lane (row, quad) holds psi and
// the numerator of sigmas 2 quad and 2 quad + 1 of node row, so each store
// covers 16 consecutive nodes of 4 sigmas. One wavefront per 16-node tile;
// a job of kNodesPerJob nodes is 16 tiles for 4 wavefronts.
typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short f32_to_bf16(float f)
{
    // round to nearest even (counts and weights are finite and >= 0)
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

constexpr int kBf16SigmaGroup = 32;   // sigmas whose weight fragments sit in LDS at once

template <int K>
__global__ __launch_bounds__(256) void k_potential_bf16(const GraphDev *__restrict__ graphs,
                                                        const NodeJob *__restrict__ jobs,
                                                        float *__restrict__ psi_out,
                                                        float *__restrict__ v_out, int64_t out_ld)
{
    constexpr int KC = K / 32;                       // 32-bin chunks
    constexpr int CB = 2 * kBf16SigmaGroup / 16;     // 16-column blocks per sigma group
    __shared__ bf16x8 wfrag[KC][CB][64];             // K = 32: 4 KB
    const NodeJob job = jobs[blockIdx.x];
    const GraphDev &G = graphs[job.g];
    const int n = G.n;
    const int S = G.n_sigmas;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int row = lane % 16, quad = lane / 16;
    const int kmax = min(G.dmax + 1, K);             // bins past the largest distance count 0
    constexpr int kTiles = kNodesPerJob / 16 / 4;    // tiles per wavefront

    for (int sg = 0; sg < S; sg += kBf16SigmaGroup) {
        // A fragments of this sigma group: column c = 2 s + kind of the group
        __syncthreads();
        for (int f = threadIdx.x; f < KC * CB * 64; f += 256) {
            const int l = f % 64, cb = (f / 64) % CB, kc = f / (64 * CB);
            const int c = cb * 16 + l % 16, q = l / 16;
            const int sig = sg + c / 2, kind = c % 2;
            bf16x8 a;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = kc * 32 + q * 8 + e;
                a[e] = (sig < S) ? (short)G.wbf16[((int64_t)sig * G.K + k) * 2 + kind] : (short)0;
            }
            wfrag[kc][cb][l] = a;
        }
        __syncthreads();
#pragma unroll 1
        for (int t = 0; t < kTiles; ++t) {
            const int node0 = job.i0 + (wave + 4 * t) * 16;
            if (node0 >= n) break;
            const int node = node0 + row;
            // B fragments: lane holds bins 8 quad .. 8 quad + 7 of node
            // node0 + row, two 16-byte loads per chunk
            bf16x8 hb[KC];
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
                u32x4 lo = {0u, 0u, 0u, 0u}, hi = {0u, 0u, 0u, 0u};
                if (node < n) {
                    const global_u4 src =
                        (global_u4)(G.hist + (int64_t)node * G.K + kc * 32 + quad * 8);
                    lo = src[0];
                    hi = src[1];
                }
                const uint32_t h8[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    hb[kc][e] = (kc * 32 + quad * 8 + e < kmax) ? f32_to_bf16((float)h8[e]) : (short)0;
            }
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                if (sg + cb * 8 >= S) break;
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kc = 0; kc < KC; ++kc)
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wfrag[kc][cb][lane], hb[kc], acc,
                                                                  0, 0, 0);
                // acc[r] = column 4 quad + r of the block for node `row`:
                // sigma sg + 8 cb + 2 quad + r / 2, psi (r even) or numerator
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int sig = sg + cb * 8 + 2 * quad + j;
                    if (sig < S && node < n) {
                        const float psi = acc[2 * j], v = acc[2 * j + 1] / psi;
                        const int64_t ou = job.out_off + (int64_t)sig * out_ld + node;
                        if (psi_out) psi_out[ou] = psi;
                        else G.psi[(int64_t)sig * n + node] = psi;
                        if (v_out) v_out[ou] = v;
                        else G.v[v_index(n, sig, node)] = v;
                    }
                }
            }
        }
    }
}

hipError_t launch_potential(int precision, int K, const GraphDev *graphs, const NodeJob *jobs,
                            int n_jobs, float *psi_out, float *v_out, int64_t out_ld,
                            hipStream_t stream)
{
    if (n_jobs <= 0) return hipSuccess;
    const dim3 grid(n_jobs), block(256);
#define QC_POT_ARGS grid, block, 0, stream, graphs, jobs, psi_out, v_out, out_ld
    if (precision == 0) {
        switch (K) {
        case 32: hipLaunchKernelGGL((k_potential<32, 0>), QC_POT_ARGS); break;
        case 64: hipLaunchKernelGGL((k_potential<64, 0>), QC_POT_ARGS); break;
        case 128: hipLaunchKernelGGL((k_potential<128, 0>), QC_POT_ARGS); break;
        default: return hipErrorInvalidValue;
        }
    } else if (precision == 2) {
        switch (K) {
        case 32: hipLaunchKernelGGL((k_potential_bf16<32>), QC_POT_ARGS); break;
        case 64: hipLaunchKernelGGL((k_potential_bf16<64>), QC_POT_ARGS); break;
        case 128: hipLaunchKernelGGL((k_potential_bf16<128>), QC_POT_ARGS); break;
        default: return hipErrorInvalidValue;
        }
    } else if (precision == 1) {
        switch (K) {
        case 32: hipLaunchKernelGGL((k_potential<32, 1>), QC_POT_ARGS); break;
        case 64: hipLaunchKernelGGL((k_potential<64, 1>), QC_POT_ARGS); break;
        case 128: hipLaunchKernelGGL((k_potential<128, 1>), QC_POT_ARGS); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        return hipErrorInvalidValue;
    }
#undef QC_POT_ARGS
    return hipGetLastError();
}

// ===========================================================================
// Graph Gradient Descent, first half of Algorithm 2: every node picks the
// neighbour it descends to.
//
// FP32 pass: lowest and second-lowest neighbour V (the lowest keeps the
// smallest id, since neighbours are sorted). If both the argmin and the
// comparison with the node's own V are clear by more than the FP32 error
// bound, the FP32 order is the FP64 order and the decision is final.
// Otherwise the node is re-decided with the canonical FP64 potential of
// itself and of every neighbour within the bound of the lowest one. The
// canonical FP64 value sums h_k * w_k and (k^2 h_k) * w_k in ascending k from
// +0.0 with separate roundings (no contraction), then (1/a) * (S1/S2): the
// same IEEE operations in the same order as the CPU oracle, so both sides
// take identical decisions, exact ties included.
// ===========================================================================

// On-demand canonical FP64 V of one node (used when no FP64 table is resident).
__device__ __noinline__ double canonical_v(const int32_t *__restrict__ h, int kmax,
                                           const double *__restrict__ w, double inv_a)
{
#pragma clang fp contract(off)
    double s2 = 0.0, s1 = 0.0;
    for (int k = 0; k < kmax; ++k) {
        const double hk = (double)h[k];
        s2 = s2 + hk * w[k];
        s1 = s1 + ((double)(k * k) * hk) * w[k];
    }
    return inv_a * (s1 / s2);
}

__device__ __forceinline__ double fp64_v(const GraphDev &G, int s, int node)
{
    if (G.v64) return G.v64[(int64_t)s * G.n + node];
    return canonical_v(G.hist + (int64_t)node * G.K, G.dmax + 1, G.w64 + (int64_t)s * G.K,
                       G.inv_a[s]);
}

// The FP64 decision for node i (thread t of the descent's order) at sigma
// s: among the neighbours whose FP32 V lies within the bound of the lowest
// one (m1), the lowest canonical FP64 V, compared with the node's own. The
// neighbours come from the thread's sliced list in CSR order, kGgdPad per
// round with their loads in flight together (a hub re-deciding among many
// twin leaves would otherwise wait for two dependent loads per neighbour);
// the first of equal FP64 minima wins, as in a plain CSR scan.
__device__ __noinline__ int fp64_decide(int tie_mode, const GraphDev &G, int s, int t, int i,
                                        float m1)
{
    const int n = G.n;
    const float *__restrict__ V = G.v;
    const double vi64 = fp64_v(G, s, i);
    const int deg = G.sell_deg[t];
    const int32_t *__restrict__ sc = G.sell_col + G.sell_off[t >> 6] + (t & 63);
    double bv = DBL_MAX;
    int best = -1;
    for (int k = 0; k < deg; k += kGgdPad) {
        int j[kGgdPad];
        float vj[kGgdPad];
#pragma unroll
        for (int u = 0; u < kGgdPad; ++u) j[u] = sc[64 * (k + u)];
#pragma unroll
        for (int u = 0; u < kGgdPad; ++u) vj[u] = V[v_index(n, s, j[u])];
        double d[kGgdPad];
#pragma unroll
        for (int u = 0; u < kGgdPad; ++u)
            d[u] = (k + u < deg && vj[u] - m1 <= kTieTau * vj[u]) ? fp64_v(G, s, j[u]) : DBL_MAX;
#pragma unroll
        for (int u = 0; u < kGgdPad; ++u)
            if (d[u] < bv) {
                bv = d[u];
                best = j[u];
            }
    }
    if (tie_mode == 0) return (bv < vi64) ? best : i;
    return (bv < vi64 || (bv == vi64 && best < i)) ? best : i;
}

// One thread per node and KS consecutive sigmas: the node's order slot,
// degree and neighbour indices are loaded once and the V values of all KS
// sigmas are gathered together, so one chain of dependent loads serves KS
// decisions (the kernel is bound by memory latency, not by bandwidth).
template <int KS>
__global__ __launch_bounds__(256) void k_ggd_parent(int tie_mode, const GraphDev *__restrict__ graphs,
                                                    const NodeJob *__restrict__ jobs, int sigma_base,
                                                    int sigma_end)
{
    // blockIdx.y selects the sigmas: the blocks in flight share them, so the
    // gathered V values (one interleaved group of sigmas, a few MB for a
    // whole batch) stay in L2 while the neighbour lists stream past.
    const NodeJob job = jobs[blockIdx.x];
    const GraphDev &G = graphs[job.g];
    const int n = G.n;
    const int s0 = sigma_base + (int)blockIdx.y * KS;
    const int s_end = min(sigma_end, G.n_sigmas);
    const int t = job.i0 + (int)threadIdx.x;
    bool rechecked[KS];
#pragma unroll
    for (int q = 0; q < KS; ++q) rechecked[q] = false;
    if (t < n && s0 < s_end) {
        // within the job, threads take its nodes by decreasing degree, so the
        // neighbour loops of one wavefront have similar trip counts
        const int i = G.order[t];
        float vi[KS], m1[KS], m2[KS];
        int j1[KS];
        // V of node j for this thread's sigmas: with a whole, aligned group
        // of kVGroup sigmas one 16-byte load (the values of sigmas past the
        // end are padding and are never used), else one load per sigma
        auto load_v = [&](int j, float (&out)[KS]) {
            if constexpr (KS == kVGroup) {
                const float4 x = *(const float4 *)(G.v + v_index(n, s0, j));
                out[0] = x.x;
                out[1] = x.y;
                out[2] = x.z;
                out[3] = x.w;
            } else {
#pragma unroll
                for (int q = 0; q < KS; ++q) out[q] = G.v[v_index(n, min(s0 + q, s_end - 1), j)];
            }
        };
        load_v(i, vi);
#pragma unroll
        for (int q = 0; q < KS; ++q) {
            m1[q] = m2[q] = FLT_MAX;
            j1[q] = -1;
        }
        // The node's neighbours from the sliced lists (t & 63 is the lane:
        // jobs start at multiples of 256 nodes), kGgdPad per round: their
        // indices load together (coalesced across the wavefront), then their
        // V values, so a round waits for two memory latencies. Slots past
        // the node's degree read other entries of the same lists or the
        // padding (valid node ids) and take no part in the minima; the slots
        // are scanned in CSR order, so the first minimum wins as in a plain
        // scan.
        const int deg = G.sell_deg[t];
        const int32_t *__restrict__ sc = G.sell_col + G.sell_off[t >> 6] + (t & 63);
        for (int k = 0; k < deg; k += kGgdPad) {
            int j[kGgdPad];
            float vj[kGgdPad][KS];
#pragma unroll
            for (int u = 0; u < kGgdPad; ++u) j[u] = sc[64 * (k + u)];
#pragma unroll
            for (int u = 0; u < kGgdPad; ++u) load_v(j[u], vj[u]);
#pragma unroll
            for (int u = 0; u < kGgdPad; ++u) {
                if (k + u < deg) {
#pragma unroll
                    for (int q = 0; q < KS; ++q) {
                        if (vj[u][q] < m1[q]) { m2[q] = m1[q]; m1[q] = vj[u][q]; j1[q] = j[u]; }
                        else if (vj[u][q] < m2[q]) m2[q] = vj[u][q];
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < KS; ++q) {
            const int s = s0 + q;
            if (s >= s_end) break;
            int parent = i;
            if (j1[q] >= 0) {
                const float tau = kTieTau;
                const float hi = fmaxf(m1[q], vi[q]), lo = fminf(m1[q], vi[q]);
                bool ambiguous = (hi - lo <= tau * hi);
                // which neighbour is lowest matters only when the node moves:
                // with the lowest clearly above the node, every neighbour's
                // FP64 V is above the node's too (tau exceeds twice the FP32
                // error), and the node is a root whatever the near ties
                if (m1[q] < vi[q] && m2[q] - m1[q] <= tau * m2[q]) ambiguous = true;
                if (!ambiguous) {
                    parent = (m1[q] < vi[q]) ? j1[q] : i;
                } else {
                    parent = fp64_decide(tie_mode, G, s, t, i, m1[q]);
                    rechecked[q] = true;
                }
            }
            G.parent[(int64_t)s * n + t] = parent;   // thread order: coalesced
        }
    }
    // one counter update per wavefront
    unsigned int total = 0;
#pragma unroll
    for (int q = 0; q < KS; ++q) total += (unsigned)__popcll(__ballot(rechecked[q]));
    if (total && __lane_id() == 0) atomicAdd(G.recheck, (unsigned long long)total);
}

hipError_t launch_ggd_parent(int tie_mode, const GraphDev *graphs, const NodeJob *jobs,
                             int n_jobs, int sigma_base, int n_sig, hipStream_t stream)
{
    if (n_jobs <= 0 || n_sig <= 0) return hipSuccess;
    const int end = sigma_base + n_sig;
    static_assert(kGgdSigmas == kVGroup || kGgdSigmas == 1, "the descent's sigma groups are V's");
    if (n_sig >= kGgdSigmas && sigma_base % kVGroup == 0) {
        hipLaunchKernelGGL(k_ggd_parent<kGgdSigmas>, dim3(n_jobs, (n_sig + kGgdSigmas - 1) / kGgdSigmas),
                           dim3(256), 0, stream, tie_mode, graphs, jobs, sigma_base, end);
    } else {
        hipLaunchKernelGGL(k_ggd_parent<1>, dim3(n_jobs, n_sig), dim3(256), 0, stream, tie_mode,
                           graphs, jobs, sigma_base, end);
    }
    return hipGetLastError();
}

// ===========================================================================
// Algorithm 3 for every node: pointer jumping lab[i] <- lab[lab[i]] until
// every node points at a root (a node that is its own parent). Parents only
// ever point to strictly lower (V, id) nodes, so the forest has no cycles and
// the loop ends after about log2(height) rounds. One workgroup per (graph,
// sigma); updates in place are safe because every value written is an
// ancestor on the same path.
// ===========================================================================

__global__ __launch_bounds__(1024) void k_jump(const GraphDev *__restrict__ graphs,
                                               const NodeJob *__restrict__ jobs, int sigma_base,
                                               int32_t *labels_base, int64_t labels_ld)
{
    const NodeJob job = jobs[blockIdx.x];
    const GraphDev &G = graphs[job.g];
    const int n = G.n;
    const int s = sigma_base + (int)blockIdx.y;
    if (s >= G.n_sigmas) return;
    // parents are stored in the descent's thread order: node order[t]'s at t
    const int32_t *__restrict__ par = G.parent + (int64_t)s * n;
    int32_t *lab = labels_base + (int64_t)blockIdx.y * labels_ld + job.out_off;
    for (int t = threadIdx.x; t < n; t += blockDim.x) lab[G.order[t]] = par[t];
    __syncthreads();
    for (int round = 0; round < 64; ++round) {
        int changed = 0;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const int p = __hip_atomic_load(&lab[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            const int q = __hip_atomic_load(&lab[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (q != p) {
                __hip_atomic_store(&lab[i], q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                changed = 1;
            }
        }
        if (!__syncthreads_or(changed)) break;
    }
}

// The same rounds on a copy of the parents in LDS (graphs of up to CAP
// nodes): one coalesced read of the parents, the jumps at LDS latency, one
// coalesced write of the labels.
template <int CAP>
__global__ __launch_bounds__(1024) void k_jump_lds(const GraphDev *__restrict__ graphs,
                                                   const NodeJob *__restrict__ jobs, int sigma_base,
                                                   int32_t *labels_base, int64_t labels_ld)
{
    __shared__ int32_t lab[CAP];
    const NodeJob job = jobs[blockIdx.x];
    const GraphDev &G = graphs[job.g];
    const int n = G.n;
    const int s = sigma_base + (int)blockIdx.y;
    if (s >= G.n_sigmas || n > CAP) return;
    // parents are stored in the descent's thread order: node order[t]'s at t
    const int32_t *__restrict__ par = G.parent + (int64_t)s * n;
    for (int t = threadIdx.x; t < n; t += blockDim.x) lab[G.order[t]] = par[t];
    __syncthreads();
    for (int round = 0; round < 64; ++round) {
        int changed = 0;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const int p = __hip_atomic_load(&lab[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            const int q = __hip_atomic_load(&lab[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (q != p) {
                __hip_atomic_store(&lab[i], q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                changed = 1;
            }
        }
        if (!__syncthreads_or(changed)) break;
    }
    int32_t *out = labels_base + (int64_t)blockIdx.y * labels_ld + job.out_off;
    for (int i = threadIdx.x; i < n; i += blockDim.x) out[i] = lab[i];
}

hipError_t launch_pointer_jump(const GraphDev *graphs, const NodeJob *jobs, int n_jobs,
                               int sigma_base, int n_sig, int32_t *labels_base,
                               int64_t labels_ld, int max_n, hipStream_t stream, int variant)
{
    if (n_jobs <= 0 || n_sig <= 0) return hipSuccess;
    const dim3 grid(n_jobs, n_sig), block(1024);
    if (variant == 1)     // in global memory whatever the size
        hipLaunchKernelGGL(k_jump, grid, block, 0, stream, graphs, jobs, sigma_base, labels_base,
                           labels_ld);
    else if (max_n <= 20480)   // 80 KB of LDS: two workgroups per CU
        hipLaunchKernelGGL(k_jump_lds<20480>, grid, block, 0, stream, graphs, jobs, sigma_base,
                           labels_base, labels_ld);
    else if (max_n <= 40704)
        hipLaunchKernelGGL(k_jump_lds<40704>, grid, block, 0, stream, graphs, jobs, sigma_base,
                           labels_base, labels_ld);
    else
        hipLaunchKernelGGL(k_jump, grid, block, 0, stream, graphs, jobs, sigma_base, labels_base,
                           labels_ld);
    return hipGetLastError();
}

// ===========================================================================

__global__ void k_fill_i32(int32_t *p, int64_t count, int32_t value)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

hipError_t launch_fill_i32(int32_t *p, int64_t count, int32_t value, hipStream_t stream)
{
    if (count <= 0) return hipSuccess;
    int blocks = (int)((count + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks), dim3(256), 0, stream, p, count, value);
    return hipGetLastError();
}

__global__ void k_fill_u64(unsigned long long *p, int64_t count)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

hipError_t launch_fill_u64(unsigned long long *p, int64_t count, hipStream_t stream)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, stream, p, count);
    return hipGetLastError();
}

__global__ void k_set_desc(GraphDev *dst, GraphDev src)
{
    if (threadIdx.x == 0) *dst = src;
}

hipError_t launch_set_desc(GraphDev *dst, const GraphDev &src, hipStream_t stream)
{
    hipLaunchKernelGGL(k_set_desc, dim3(1), dim3(64), 0, stream, dst, src);
    return hipGetLastError();
}

}  // namespace qc
