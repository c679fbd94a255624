// Multi-source BFS kernel template (instantiated per batch width by
// qc_bfs_<bw>.hip).
//
// One workgroup owns a batch of BW sources, entries s0..s0+BW-1 of the
// graph's source order, and runs the level-synchronous search of all of them
// at once. LDS holds three bit
// fields per node: `seen` (the batch sources that have reached the node),
// `front` (those that reached it at the previous level) and `nxt` (those
// reaching it at the current level). A level is:
//   A. edge-parallel pull: for every edge (r, c), the sources that reached c
//      at the previous level are offered to r:
//        nxt[r] |= front[c]        (LDS atomic OR, no return, no branch)
//      (level 1, whose frontier is the sources themselves, is pushed from
//      them along their CSR rows instead);
//   B. word-owner update: every thread owns whole 32-bit words of the fields;
//      the new pairs are nxt & ~seen; it moves them into front and seen and
//      records the level in the distance bit-planes (nxt keeps accumulating:
//      bits of earlier levels are in seen already).
//
// Distances live in registers for the whole search, as P bit-planes of the
// level (plane p holds bit p of every pair's distance; P = 7 covers every
// distance up to 126, fewer planes suffice once the graph's largest distance
// is known). Each batch therefore writes its BW output rows exactly once, at
// the end. Bit b at node v means that the batch's source b has reached v, so the
// pair's distance is entry (src[s0+b], v) of the row-major matrix (the edge
// list holds in-edges, so for a directed graph this is the distance from the
// source): those BW rows are this workgroup's.
//
// The edge list (packed (row << 16) | col, rows ascending, padded with no-op
// (0, 0) entries to a multiple of 4) is streamed every level with 16-byte
// buffer loads; every thread takes 8 consecutive edges (the next 8 in
// flight), issues their 8 front gathers together, then up to 8 atomics.
#pragma once

#include "qc_internal.h"

namespace qc {

template <int BW> struct BfsWord {
    using T = uint32_t;
    static constexpr int kBits = 32;
    static constexpr int kPer = 32 / BW;  // nodes per word
};
template <> struct BfsWord<64> {
    using T = unsigned long long;
    static constexpr int kBits = 64;
    static constexpr int kPer = 1;
};

// A copy of x the compiler cannot see through: indices derived from it are
// recomputed where they are used instead of being held in registers for the
// whole search (the registers go to the distance planes).
__device__ __forceinline__ int opaque(int x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// Sum of v over the 64 lanes of the wavefront, returned to every lane: an
// inclusive scan within each row of 16 lanes (DPP row shifts by 1, 2, 4, 8;
// lanes shifted in from outside the row add 0), then row 15's total is
// broadcast into rows 1 and 3 and lane 31's into rows 2 and 3, so lane 63
// holds the total.
__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// 4-bit mask -> 4 bytes of 0x01 / 0x00 (bit i selects byte i).
__device__ __forceinline__ uint32_t spread4(uint32_t m4)
{
    return (m4 * 0x00204081u) & 0x01010101u;
}

template <int BW>
__device__ __forceinline__ typename BfsWord<BW>::T field_of(const typename BfsWord<BW>::T *a, int v)
{
    using W = BfsWord<BW>;
    if constexpr (BW >= 32) {
        return a[v];
    } else {
        const uint32_t w = a[v / W::kPer];
        return (w >> ((v % W::kPer) * BW)) & ((1u << BW) - 1u);
    }
}

// Pull along 8 consecutive edges (rows ascending): the 8 gathers of the
// source field are issued together (one wait); the OR over each run of edges
// of one row is formed with selects (no branches), and only the last edge of
// a run with something to deliver issues a no-return LDS atomic into nxt[r].
// Bits r has already seen are harmless: the word's owner masks with seen.
// brk[k] (edge k ends a run) serves both as "edge k is a run's last" and as
// "edge k + 1 starts a new run". `dst` is nxt, or the start of the fields when
// the rows are packed with the bias that reaches nxt from there.
template <int BW>
__device__ __forceinline__ void pull_oct(const u32x4 &a, const u32x4 &b,
                                         const typename BfsWord<BW>::T *src,
                                         typename BfsWord<BW>::T *dst)
{
    using W = BfsWord<BW>;
    using T = typename W::T;
    const uint32_t e[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    T x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = field_of<BW>(src, (int)(e[k] & 0xFFFFu));
    bool brk[8];
#pragma unroll
    for (int k = 0; k < 7; ++k) brk[k] = (e[k] >> 16) != (e[k + 1] >> 16);
    brk[7] = true;
    T acc = x[0];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t r = e[k] >> 16;
        if (k > 0) acc = brk[k - 1] ? x[k] : (acc | x[k]);
        if (brk[k] && acc)
            __hip_atomic_fetch_or(&dst[r / W::kPer], (T)(acc << ((r % W::kPer) * BW)),
                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

// Transpose the 8 x 8 bit matrix in each byte lane of a[0..7]: afterwards
// bit 8j + p of a[k] is what bit 8j + k of a[p] was. Three rounds of swaps
// between words 4, 2 and 1 apart (bit-field inserts of the shifted partner).
__device__ __forceinline__ void transpose8x8_lanes(uint32_t (&a)[8])
{
    constexpr uint32_t kMask[3] = {0x0F0F0F0Fu, 0x33333333u, 0x55555555u};
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const int s = 4 >> r;
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            if (p & s) continue;
            const uint32_t x = a[p], y = a[p + s], m = kMask[r];
            a[p] = (x & m) | ((y << s) & ~m);
            a[p + s] = ((x >> s) & m) | (y & ~m);
        }
    }
}

// 16 bytes of the packed edge list at byte offset `off`; offsets at or past
// the end read as zeros (the buffer's range check), i.e. no-op edges (0, 0).
__device__ __forceinline__ u32x4 edge_quad(__amdgpu_buffer_rsrc_t rsrc, uint32_t off)
{
    return __builtin_amdgcn_raw_buffer_load_b128(rsrc, (int)off, 0, 0);
}

// Level 1 pushed from the sources: source b of the batch (node srcs[b]) is
// offered to each of its out-neighbours, nxt[u] |= bit b. kT / BW threads
// share a source and stride over its CSR row, four independent loads in
// flight each. (A second pushed level, over the neighbours' rows, serialises
// on the rows of high-degree neighbours and measured slower than a pull.)
template <int BW, int kT, bool WEIGHTED>
__device__ __forceinline__ void push_level1(const GraphDev &G, const int32_t *srcs, int nb,
                                            typename BfsWord<BW>::T *nxt)
{
    using W = BfsWord<BW>;
    using T = typename W::T;
    constexpr int kTps = kT / BW;           // threads per source (>= 8)
    const int b = (int)threadIdx.x / kTps;
    const int part = (int)threadIdx.x % kTps;
    if (b >= nb) return;
    const int s = srcs[b];
    const int32_t *__restrict__ rp = WEIGHTED ? G.bfs_row_ptr : G.row_ptr;
    const int32_t *__restrict__ col = WEIGHTED ? G.bfs_col : G.col;
    const int e1 = rp[s + 1];
    for (int e = rp[s] + part; e < e1; e += 4 * kTps) {
        int u[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) u[k] = (e + k * kTps < e1) ? col[e + k * kTps] : -1;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (u[k] >= 0)
                __hip_atomic_fetch_or(&nxt[u[k] / W::kPer], (T)((T)1 << ((u[k] % W::kPer) * BW + b)),
                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

// Workgroup shapes (kBfsNarrow, kBfsWide, kBfsWide1024, kBfsFront):
//   narrow   1024 threads, three fields (pull from `front`);
//   front    1024 threads, pull from `front` like narrow, but `seen` lives in
//            the registers of each word's owner (only the owner ever reads or
//            writes it: phase B and the decode), so only `front` and `nxt`
//            take LDS: the three-field search at the two-field LDS budget,
//            for one more register per word and plane set;
//   wide      512 threads, two fields (pull from `seen`, which is also
//             exact: a source that reached c before the previous level has
//             already reached r), so twice the words fit the LDS and each
//             thread has 256 registers for its planes: twice the sources per
//             batch on mid-size graphs;
//   wide1024 1024 threads, two fields: up to 16 words per thread fit 128
//             registers, so a batch that needs the two-field layout (and
//             fits 16 words) runs with four wavefronts per SIMD, not two.
// Pulling from `seen` delivers bits that `front` would not (sources that
// reached c long ago), so for one batch width the three-field shape issues
// fewer atomics; the planner prefers it whenever the batch fits.
template <int SHAPE> struct BfsShape {
    static constexpr int kThreads = (SHAPE == kBfsWide) ? kBfsThreadsWide : kBfsThreads;
    // two LDS fields [seen | nxt], pulling from seen
    static constexpr bool kPullSeen = SHAPE == kBfsWide || SHAPE == kBfsWide1024;
    // seen in the owners' registers, two LDS fields [front | nxt]
    static constexpr bool kSeenRegs = SHAPE == kBfsFront;
    static constexpr int kFields = (kPullSeen || kSeenRegs) ? 2 : 3;
};

// WEIGHTED: the graph's edges carry integer weights and the search walks the
// subdivided graph (G.n_bfs nodes, G.nnz_bfs edges, the first G.n being the
// graph's own nodes); otherwise the graph itself.
template <int BW, int NW, int P, int SHAPE, bool WEIGHTED>
__global__ __launch_bounds__(BfsShape<SHAPE>::kThreads) void k_bfs(const GraphDev *__restrict__ graphs,
                                                                   const BfsJob *__restrict__ jobs)
{
    constexpr bool WIDE = BfsShape<SHAPE>::kPullSeen;
    constexpr bool SREG = BfsShape<SHAPE>::kSeenRegs;
    using W = BfsWord<BW>;
    using T = typename W::T;
    constexpr int kT = BfsShape<SHAPE>::kThreads;
    constexpr int NWW = (BW == 64) ? NW / 2 : NW;   // words of type T per thread
    constexpr int kLdsWords = NWW * kT;
    constexpr int kLevels = (P >= 7) ? kMaxDist : ((1 << P) - 1);  // largest encodable level
    // Word ownership: with 32-bit words and a multiple of 4 per thread, a
    // thread owns runs of 4 consecutive words, (g kT + tid) * 4 + i for its
    // g-th run (V = 4): phase B reads and writes them with 16-byte LDS
    // accesses, and with one node per word the decode holds 4 consecutive
    // nodes and transposes their bytes in registers. Otherwise word
    // j kT + tid (V = 1).
    constexpr int V = (BW <= 32 && NWW % 4 == 0) ? 4 : 1;

    // The fields share one LDS array, the field the pull gathers from first
    // (LDS address 0, so a gather's address is the column's word offset):
    // two fields [seen | nxt], three fields [front | nxt | seen], or, with
    // seen in registers, [front | nxt].
    __shared__ __attribute__((aligned(16))) T fields[BfsShape<SHAPE>::kFields * kLdsWords];
    __shared__ uint32_t found_pairs;
    __shared__ int32_t srcs[BW];          // the batch's sources
    T *const front = fields;
    T *const nxt = fields + kLdsWords;
    T *const seen = WIDE ? fields : fields + 2 * kLdsWords;   // (not with SREG)
    // where the pull's row field points: with a row bias, rows count from the
    // start of the fields (nxt = fields + kLdsWords)
    constexpr int kRowBias = bfs_row_bias(BW, NW, SHAPE);
    static_assert(kRowBias == 0 || kRowBias == kLdsWords * W::kPer, "row bias reaches nxt");
    T *const pull_dst = kRowBias ? fields : nxt;
    T seen_r[SREG ? NWW : 1];             // SREG: seen of the owned words

    const BfsJob job = jobs[blockIdx.x];
    const GraphDev &G = graphs[job.g];
    const int n = G.n;
    const int s0 = job.s0;
    const int nb = min(BW, n - s0);
    // with weights the BFS walks n_bfs nodes (n plus the nodes that subdivide
    // edges, which count as reached pairs and levels like any node); only
    // the first n are sources and get distances written
    const int nwords = ((WEIGHTED ? G.n_bfs : n) + W::kPer - 1) / W::kPer;
    const int tid = threadIdx.x;
    const uint32_t quad_bytes = (uint32_t)(((WEIGHTED ? G.nnz_bfs : G.nnz) + 3) >> 2) * 16u;
    const __amdgpu_buffer_rsrc_t edges =
        __builtin_amdgcn_make_buffer_rsrc((void *)G.edges, 0, (int)quad_bytes, kBufferWord3);

    T plane[NWW][P];
#pragma unroll
    for (int j = 0; j < NWW; ++j)
#pragma unroll
        for (int p = 0; p < P; ++p) plane[j][p] = 0;

    // Level 0: each source has reached itself (distance 0: no plane bits).
    if constexpr (V == 4) {
        const uint4 z = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
        for (int g = 0; g < NWW / 4; ++g) {
            const int w0 = (g * kT + tid) * 4;
            if constexpr (!SREG) *(uint4 *)(seen + w0) = z;
            if constexpr (!WIDE) *(uint4 *)(front + w0) = z;
            *(uint4 *)(nxt + w0) = z;
        }
    } else {
#pragma unroll
        for (int j = 0; j < NWW; ++j) {
            const int w = j * kT + tid;
            if constexpr (!SREG) seen[w] = 0;
            if constexpr (!WIDE) front[w] = 0;
            nxt[w] = 0;
        }
    }
    if (tid < nb) srcs[tid] = G.src[s0 + tid];
    if (tid == 0) found_pairs = (uint32_t)nb;   // level 0: every source itself
    __syncthreads();
    if (tid < nb) {
        const int v = srcs[tid];
        const T bit = (T)1 << ((v % W::kPer) * BW + tid);
        if constexpr (!SREG)
            __hip_atomic_fetch_or(&seen[v / W::kPer], bit, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_WORKGROUP);
        if constexpr (!WIDE)
            __hip_atomic_fetch_or(&front[v / W::kPer], bit, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __syncthreads();
    if constexpr (SREG) {
        // the owners take the sources' bits (level 0 = the frontier) into
        // their registers
        if constexpr (V == 4) {
#pragma unroll
            for (int g = 0; g < NWW / 4; ++g) {
                const uint4 f = *(const uint4 *)(front + (g * kT + tid) * 4);
                seen_r[4 * g + 0] = f.x;
                seen_r[4 * g + 1] = f.y;
                seen_r[4 * g + 2] = f.z;
                seen_r[4 * g + 3] = f.w;
            }
        } else {
#pragma unroll
            for (int j = 0; j < NWW; ++j) seen_r[j] = front[j * kT + tid];
        }
    }
    uint32_t found_before = (uint32_t)nb;

    int last = 0;
    int overflow = 0;
    int pulled = 0;   // levels pulled over the whole edge list
    for (int level = 1;; ++level) {
        if (level == 1) {
            // A'. level 1 is pushed from the sources along their CSR rows
            //     (out-edges): a few hundred edges where a pull would scan
            //     the whole edge list.
            push_level1<BW, kT, WEIGHTED>(G, srcs, nb, nxt);
        } else {
            ++pulled;
            // A. pull over every edge, 8 consecutive edges (two quads) per
            //    thread, the next 8 in flight. Loads past the end read no-op
            //    edges, so they need no bounds check.
            //    Unrolled twice where the registers allow, so the two sets of
            //    quads alternate roles instead of being copied.
            constexpr uint32_t kStep = 2u * kT * 16u;   // bytes per round of the workgroup
            constexpr bool kAlternate = !(kT == 1024 && NWW * (P + (SREG ? 1 : 0)) > 80);
            uint32_t off = (uint32_t)opaque(tid) * 32u;
            u32x4 a0 = edge_quad(edges, off);
            u32x4 b0 = edge_quad(edges, off + 16u);
            if constexpr (kAlternate) {
                while (off < quad_bytes) {
                    const u32x4 a1 = edge_quad(edges, off + kStep);
                    const u32x4 b1 = edge_quad(edges, off + kStep + 16u);
                    pull_oct<BW>(a0, b0, front, pull_dst);
                    off += kStep;
                    if (off >= quad_bytes) break;
                    a0 = edge_quad(edges, off + kStep);
                    b0 = edge_quad(edges, off + kStep + 16u);
                    pull_oct<BW>(a1, b1, front, pull_dst);
                    off += kStep;
                }
            } else {
                for (; off < quad_bytes; off += kStep) {
                    const u32x4 a1 = edge_quad(edges, off + kStep);
                    const u32x4 b1 = edge_quad(edges, off + kStep + 16u);
                    pull_oct<BW>(a0, b0, front, pull_dst);
                    a0 = a1;
                    b0 = b1;
                }
            }
        }
        __syncthreads();
        // B. move the new bits of owned words into front / seen / planes.
        //    nxt is not cleared: it accumulates over the levels, and what an
        //    earlier level delivered is already in seen, so nxt & ~seen is
        //    still exactly this level's new pairs.
        uint32_t cnt = 0;
        const int tb = opaque(tid);
        if constexpr (V == 4) {
            // runs of 4 words; a run may reach past nwords into words no
            // edge delivers to (zero in nxt, so nothing changes there)
#pragma unroll
            for (int g = 0; g < NWW / 4; ++g) {
                const int w0 = (g * kT + tb) * 4;
                if (w0 < nwords) {
                    const uint4 raw4 = *(const uint4 *)(nxt + w0);
                    uint4 sw4;
                    if constexpr (SREG)
                        sw4 = make_uint4(seen_r[4 * g], seen_r[4 * g + 1], seen_r[4 * g + 2],
                                         seen_r[4 * g + 3]);
                    else
                        sw4 = *(const uint4 *)(seen + w0);
                    const uint4 y4 = make_uint4(raw4.x & ~sw4.x, raw4.y & ~sw4.y, raw4.z & ~sw4.z,
                                                raw4.w & ~sw4.w);
                    if constexpr (!WIDE) *(uint4 *)(front + w0) = y4;
                    const uint4 ns4 = make_uint4(sw4.x | y4.x, sw4.y | y4.y, sw4.z | y4.z, sw4.w | y4.w);
                    if constexpr (SREG) {
                        seen_r[4 * g + 0] = ns4.x;
                        seen_r[4 * g + 1] = ns4.y;
                        seen_r[4 * g + 2] = ns4.z;
                        seen_r[4 * g + 3] = ns4.w;
                    } else if (y4.x | y4.y | y4.z | y4.w) {
                        *(uint4 *)(seen + w0) = ns4;
                    }
                    const uint32_t y[4] = {y4.x, y4.y, y4.z, y4.w};
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        cnt += (uint32_t)__popc(y[i]);
#pragma unroll
                        for (int p = 0; p < P; ++p)
                            if ((level >> p) & 1) plane[4 * g + i][p] |= (T)y[i];   // uniform branch
                    }
                }
            }
        } else
#pragma unroll
        for (int j = 0; j < NWW; ++j) {
            const int w = j * kT + tb;
            if (w < nwords) {
                const T raw = nxt[w];
                const T sw = SREG ? seen_r[j] : seen[w];
                const T y = raw & ~sw;        // newly reached (node, source) pairs
                if constexpr (!WIDE) front[w] = y;
                if constexpr (SREG)
                    seen_r[j] = sw | y;
                else if (y)
                    seen[w] = sw | y;
                cnt += (uint32_t)__popcll((unsigned long long)y);
#pragma unroll
                for (int p = 0; p < P; ++p)
                    if ((level >> p) & 1) plane[j][p] |= y;   // uniform branch
            }
        }
        // one LDS atomic per wavefront with the wavefront's count of new pairs
        cnt = wave_sum(cnt);
        if ((tid & 63) == 0 && cnt) atomicAdd(&found_pairs, cnt);
        __syncthreads();
        const uint32_t found = found_pairs;
        if (found == found_before) break;   // nothing new: every search ended
        found_before = found;
        last = level;
        if (level > kLevels) {
            // this level does not fit the planes (P = 7: a distance above 126)
            overflow = (P >= 7) ? 1 : 2;
            break;
        }
        if (found >= job.target) break;     // every reachable pair found: skip the empty level
    }

    // Decode the planes of every owned word into distance bytes and write
    // rows srcs[0..nb-1], columns = owned nodes. Unreached pairs get -1 (0xFF).
    // Only the loop over words is unrolled (so the planes keep static register
    // indices); the loop over the word's dwords shifts by a variable amount.
    // The output row of every source, dist + srcs[b] * n, computed once into
    // the LDS of nxt (which the search no longer needs), so that a byte's
    // address is its row pointer plus its column: four pointers per group of
    // four bytes come with two 16-byte LDS reads.
    typedef __attribute__((address_space(1))) int8_t gbyte;
    typedef uint32_t __attribute__((aligned(1))) u32_any;   // rows need not be 4-byte aligned
    typedef __attribute__((address_space(1))) u32_any gu32;
    // With one node per 32-bit word (BW = 32) the decode takes sources 8j + k
    // (j = 0..3) together for each k, so their pointers sit side by side:
    // source b at 4 (b % 8) + b / 8.
    constexpr bool kLanes = BW == 32;
    gbyte **const rows = (gbyte **)nxt;
    if (tid < nb) rows[kLanes ? 4 * (tid & 7) + (tid >> 3) : tid] = (gbyte *)G.dist + (int64_t)srcs[tid] * G.ld;
    __syncthreads();
    // words of the graph's own nodes (the first n)
    const int own_words = WEIGHTED ? (n + W::kPer - 1) / W::kPer : nwords;
    const int td = opaque(tid);
    if constexpr (kLanes && V == 4) {
        // runs of 4 consecutive nodes v0..v0+3 (BW = 32). Per node, word p of
        // eight holds plane p (all ones past the planes) OR-ed with the
        // unreached pairs, so an unreached pair reads 0xFF; transposing the
        // bit matrix in each byte lane turns word k into the distance bytes
        // of sources k, 8 + k, 16 + k, 24 + k. For each k the four nodes'
        // words are then transposed as a 4 x 4 byte matrix into one dword per
        // source (byte i = node v0 + i), stored with one 4-byte store, so a
        // wavefront's store covers 256 consecutive bytes of a row.
#pragma unroll
        for (int g = 0; g < NWW / 4; ++g) {
            const int v0 = (g * kT + td) * 4;
            if (v0 < own_words) {
                uint32_t a[4][8];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const uint32_t u = ~(uint32_t)(SREG ? seen_r[4 * g + i] : seen[v0 + i]);
#pragma unroll
                    for (int p = 0; p < 8; ++p) a[i][p] = (p < P) ? ((uint32_t)plane[4 * g + i][p] | u) : u;
                    transpose8x8_lanes(a[i]);
                }
                // the quad's 4 x 4 byte transposes for sources 8j + k, j = 0..3
                auto quad = [&](int k, uint32_t (&o)[4]) {
                    const uint32_t d[4] = {a[0][k], a[1][k], a[2][k], a[3][k]};
                    const uint32_t t0 = __builtin_amdgcn_perm(d[1], d[0], 0x05010400u);
                    const uint32_t t1 = __builtin_amdgcn_perm(d[1], d[0], 0x07030602u);
                    const uint32_t t2 = __builtin_amdgcn_perm(d[3], d[2], 0x05010400u);
                    const uint32_t t3 = __builtin_amdgcn_perm(d[3], d[2], 0x07030602u);
                    o[0] = __builtin_amdgcn_perm(t2, t0, 0x05040100u);
                    o[1] = __builtin_amdgcn_perm(t2, t0, 0x07060302u);
                    o[2] = __builtin_amdgcn_perm(t3, t1, 0x05040100u);
                    o[3] = __builtin_amdgcn_perm(t3, t1, 0x07060302u);
                };
                if (v0 + 3 < n && nb == BW) {
                    // the common case, without branches: a whole quad, a full batch
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        uint32_t o[4];
                        quad(k, o);
                        const ulonglong2 r01 = *(const ulonglong2 *)(rows + 4 * k);
                        const ulonglong2 r23 = *(const ulonglong2 *)(rows + 4 * k + 2);
                        *(gu32 *)((gbyte *)r01.x + v0) = o[0];
                        *(gu32 *)((gbyte *)r01.y + v0) = o[1];
                        *(gu32 *)((gbyte *)r23.x + v0) = o[2];
                        *(gu32 *)((gbyte *)r23.y + v0) = o[3];
                    }
                } else {
                    // the graph's last quad or a partial batch
#pragma unroll 1
                    for (int k = 0; k < 8; ++k) {
                        uint32_t o[4];
#pragma unroll
                        for (int kk = 0; kk < 8; ++kk)
                            if (kk == k) quad(kk, o);
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            if (8 * j + k >= nb) continue;
                            gbyte *const r = rows[4 * k + j];
#pragma unroll
                            for (int i = 0; i < 4; ++i)
                                if (v0 + i < n) r[v0 + i] = (int8_t)((o[j] >> (8 * i)) & 0xFFu);
                        }
                    }
                }
            }
        }
    } else if constexpr (kLanes) {
        // one node per lane (BW = 32, word j kT + tid): the same per-node
        // transpose, then for each k the four lanes of a quad, which hold four
        // consecutive nodes, transpose their words' bytes across the quad
        // (swap 16-bit halves with lane ^ 2, then bytes with lane ^ 1), so
        // lane q stores source 8q + k's bytes for the quad's four nodes with
        // one 4-byte store. Taken when the whole quad is in the graph and the
        // batch is full (the same for the quad's four lanes).
        const int q = td & 3;
        const uint32_t sel2 = (q >> 1) ? 0x03020706u : 0x05040100u;
        const uint32_t sel1 = (q & 1) ? 0x03070105u : 0x06020400u;
#pragma unroll
        for (int j = 0; j < NWW; ++j) {
            const int w = j * kT + td;
            if (w < own_words) {
                uint32_t a[8];
                const uint32_t u = ~(uint32_t)(SREG ? seen_r[j] : seen[w]);
#pragma unroll
                for (int p = 0; p < 8; ++p) a[p] = (p < P) ? ((uint32_t)plane[j][p] | u) : u;
                transpose8x8_lanes(a);
                if (w - q + 3 < n && nb == BW) {
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const uint32_t d = a[k];
                        const uint32_t p2 = (uint32_t)__builtin_amdgcn_mov_dpp((int)d, 0x4E, 0xF, 0xF, false);
                        const uint32_t h = __builtin_amdgcn_perm(p2, d, sel2);
                        const uint32_t p1 = (uint32_t)__builtin_amdgcn_mov_dpp((int)h, 0xB1, 0xF, 0xF, false);
                        *(gu32 *)(rows[4 * k + q] + (w - q)) = __builtin_amdgcn_perm(p1, h, sel1);
                    }
                } else {
#pragma unroll 1
                    for (int k = 0; k < 8; ++k) {
                        uint32_t d = 0;
#pragma unroll
                        for (int kk = 0; kk < 8; ++kk)
                            if (kk == k) d = a[kk];
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            if (8 * i + k < nb && w < n) rows[4 * k + i][w] = (int8_t)((d >> (8 * i)) & 0xFFu);
                    }
                }
            }
        }
    } else
#pragma unroll
    for (int jv = 0; jv < NWW; ++jv) {
        // word j of the thread, at its position in the V-word runs
        const int j = jv;
        const int w = (V == 4) ? ((j / 4) * kT + td) * 4 + (j % 4) : j * kT + td;
        if (w < own_words) {
            const T sw = SREG ? seen_r[j] : seen[w];
            T lp[P];
#pragma unroll
            for (int p = 0; p < P; ++p) lp[p] = plane[j][p];
#pragma unroll 1
            for (int t = 0; t < W::kBits / 4; ++t) {
                // pairs 4t..4t+3: one node, sources b0..b0+3 (BW is a multiple
                // of 4)
                const int qn = (4 * t) / BW;       // node within the word
                const int b0 = (4 * t) % BW;       // first source of the four
                const int v = w * W::kPer + qn;
                // pairs 4t..4t+3 of the word -> one dword of 4 distance bytes
                uint32_t d = spread4((uint32_t)(~sw >> (4 * t)) & 0xFu) * 0xFFu;
#pragma unroll
                for (int p = 0; p < P; ++p) d |= spread4((uint32_t)(lp[p] >> (4 * t)) & 0xFu) << p;
                // One node per lane (W::kPer == 1): the four lanes of a quad
                // hold four consecutive nodes. A 4 x 4 byte transpose within
                // the quad (swap 16-bit halves with lane ^ 2, then bytes with
                // lane ^ 1) gives lane q the bytes of source b0 + q for the
                // quad's four nodes: one 4-byte store instead of four byte
                // stores. Taken when the whole quad is in the graph and all
                // four sources in the batch (the same for its four lanes).
                const int q = td & 3;
                if (W::kPer == 1 && b0 + 4 <= nb && v - q + 3 < n) {
                    const uint32_t hi = (uint32_t)(q >> 1), odd = (uint32_t)(q & 1);
                    const uint32_t p2 = (uint32_t)__builtin_amdgcn_mov_dpp((int)d, 0x4E, 0xF, 0xF, false);
                    const uint32_t a = __builtin_amdgcn_perm(p2, d, hi ? 0x03020706u : 0x05040100u);
                    const uint32_t p1 = (uint32_t)__builtin_amdgcn_mov_dpp((int)a, 0xB1, 0xF, 0xF, false);
                    const uint32_t e = __builtin_amdgcn_perm(p1, a, odd ? 0x03070105u : 0x06020400u);
                    *(gu32 *)(rows[b0 + q] + (v - q)) = e;
                } else {
                    const ulonglong2 r01 = *(const ulonglong2 *)(rows + b0);
                    const ulonglong2 r23 = *(const ulonglong2 *)(rows + b0 + 2);
                    gbyte *const r[4] = {(gbyte *)r01.x, (gbyte *)r01.y, (gbyte *)r23.x, (gbyte *)r23.y};
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if (v < n && b0 + k < nb) r[k][v] = (int8_t)((d >> (8 * k)) & 0xFFu);
                }
            }
        }
    }
    if (tid == 0) {
        atomicMax(&G.status[0], last);
        if (overflow) atomicOr(&G.status[1], overflow);
    }
    if (G.visits && tid < 64) {
        // the work of this batch: every edge entry per pulled level, and the
        // sources' row entries the first level pushed
        const int32_t *__restrict__ rp = WEIGHTED ? G.bfs_row_ptr : G.row_ptr;
        const uint32_t deg = (tid < nb) ? (uint32_t)(rp[srcs[tid] + 1] - rp[srcs[tid]]) : 0u;
        const uint32_t pushed = wave_sum(deg);
        if (tid == 0) {
            const unsigned long long v =
                (unsigned long long)pulled * (unsigned long long)(WEIGHTED ? G.nnz_bfs : G.nnz) +
                pushed;
            atomicAdd(&G.visits[0], v);
            atomicAdd(&G.visits[1], v * (unsigned long long)sizeof(T));
        }
    }
}

template <int BW, int NW, int P, int SHAPE>
hipError_t launch_bfs_t(bool weighted, const GraphDev *graphs, const BfsJob *jobs, int n_jobs,
                        hipStream_t stream)
{
    if (weighted)
        hipLaunchKernelGGL((k_bfs<BW, NW, P, SHAPE, true>), dim3(n_jobs),
                           dim3(BfsShape<SHAPE>::kThreads), 0, stream, graphs, jobs);
    else
        hipLaunchKernelGGL((k_bfs<BW, NW, P, SHAPE, false>), dim3(n_jobs),
                           dim3(BfsShape<SHAPE>::kThreads), 0, stream, graphs, jobs);
    return hipGetLastError();
}

template <int BW, int P>
hipError_t launch_bfs_p(int nw, bool weighted, const GraphDev *graphs, const BfsJob *jobs,
                        int n_jobs, hipStream_t stream)
{
    switch (nw) {
    case 1: if constexpr (BW != 64) return launch_bfs_t<BW, 1, P, kBfsNarrow>(weighted, graphs, jobs, n_jobs, stream);
            return hipErrorInvalidValue;
    case 2: return launch_bfs_t<BW, 2, P, kBfsNarrow>(weighted, graphs, jobs, n_jobs, stream);
    case 4: return launch_bfs_t<BW, 4, P, kBfsNarrow>(weighted, graphs, jobs, n_jobs, stream);
    case 6: return launch_bfs_t<BW, 6, P, kBfsNarrow>(weighted, graphs, jobs, n_jobs, stream);
    case 8: return launch_bfs_t<BW, 8, P, kBfsNarrow>(weighted, graphs, jobs, n_jobs, stream);
    case 10: return launch_bfs_t<BW, 10, P, kBfsNarrow>(weighted, graphs, jobs, n_jobs, stream);
    case 12: if constexpr (P < 7 || BW < 64) return launch_bfs_t<BW, 12, P, kBfsNarrow>(weighted, graphs, jobs, n_jobs, stream);
             return hipErrorInvalidValue;  // 7 planes x 12 64-bit halves exceed the registers
    default: return hipErrorInvalidValue;
    }
}

// Two-field, 512-thread shapes (planes 4 or 5 only).
template <int BW, int P>
hipError_t launch_bfs_wide_p(int nw, bool weighted, const GraphDev *graphs, const BfsJob *jobs,
                             int n_jobs, hipStream_t stream)
{
    if constexpr (P >= 7 || BW < 8) {
        return hipErrorInvalidValue;
    } else {
        switch (nw) {
        case 16: return launch_bfs_t<BW, 16, P, kBfsWide>(weighted, graphs, jobs, n_jobs, stream);
        case 24: return launch_bfs_t<BW, 24, P, kBfsWide>(weighted, graphs, jobs, n_jobs, stream);
        case 32: return launch_bfs_t<BW, 32, P, kBfsWide>(weighted, graphs, jobs, n_jobs, stream);
        case 38: if constexpr (P == 4) return launch_bfs_t<BW, 38, P, kBfsWide>(weighted, graphs, jobs, n_jobs, stream);
                 return hipErrorInvalidValue;  // 5 planes x 38 words exceed the registers
        case 39: if constexpr (P == 4 && BW != 64)
                     return launch_bfs_t<BW, 39, P, kBfsWide>(weighted, graphs, jobs, n_jobs, stream);
                 return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
        }
    }
}

// Two-field, 1024-thread shapes (planes 4 or 5): 19 words with 4 planes (18
// for 64-bit words) and 16 with 5 (18 for batches of 32) are the most that
// fit 128 registers without spills; 19 words of both fields also fill the
// 160 KB of LDS.
template <int BW, int P>
hipError_t launch_bfs_wide1024_p(int nw, bool weighted, const GraphDev *graphs,
                                 const BfsJob *jobs, int n_jobs, hipStream_t stream)
{
    if constexpr (P >= 7 || BW < 8) {
        return hipErrorInvalidValue;
    } else {
        switch (nw) {
        case 14: return launch_bfs_t<BW, 14, P, kBfsWide1024>(weighted, graphs, jobs, n_jobs, stream);
        case 16: return launch_bfs_t<BW, 16, P, kBfsWide1024>(weighted, graphs, jobs, n_jobs, stream);
        case 18: if constexpr (P == 4 || BW == 32)
                     return launch_bfs_t<BW, 18, P, kBfsWide1024>(weighted, graphs, jobs, n_jobs, stream);
                 return hipErrorInvalidValue;
        case 19: if constexpr (P == 4 && BW != 64)
                     return launch_bfs_t<BW, 19, P, kBfsWide1024>(weighted, graphs, jobs, n_jobs, stream);
                 return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
        }
    }
}

// Seen-in-registers 1024-thread shapes (planes 4 or 5): the registers hold
// (planes + 1) words per owned word, so up to 16 words per thread with 4
// planes and 14 with 5 fit 128 registers without spills.
template <int BW, int P>
hipError_t launch_bfs_front_p(int nw, bool weighted, const GraphDev *graphs, const BfsJob *jobs,
                              int n_jobs, hipStream_t stream)
{
    if constexpr (P >= 7 || BW < 8) {
        return hipErrorInvalidValue;
    } else {
        switch (nw) {
        case 4: return launch_bfs_t<BW, 4, P, kBfsFront>(weighted, graphs, jobs, n_jobs, stream);
        case 8: return launch_bfs_t<BW, 8, P, kBfsFront>(weighted, graphs, jobs, n_jobs, stream);
        case 12: return launch_bfs_t<BW, 12, P, kBfsFront>(weighted, graphs, jobs, n_jobs, stream);
        case 14: return launch_bfs_t<BW, 14, P, kBfsFront>(weighted, graphs, jobs, n_jobs, stream);
        case 16: if constexpr (P == 4)
                     return launch_bfs_t<BW, 16, P, kBfsFront>(weighted, graphs, jobs, n_jobs, stream);
                 return hipErrorInvalidValue;  // 6 x 16 words exceed the registers
        default: return hipErrorInvalidValue;
        }
    }
}

template <int BW>
hipError_t launch_bfs_bw(int nw, int planes, int shape, const GraphDev *graphs, const BfsJob *jobs,
                         int n_jobs, hipStream_t stream)
{
    const bool weighted = (shape & kBfsWeighted) != 0;
    shape &= ~kBfsWeighted;
    if (shape == kBfsWide) {
        switch (planes) {
        case 4: return launch_bfs_wide_p<BW, 4>(nw, weighted, graphs, jobs, n_jobs, stream);
        case 5: return launch_bfs_wide_p<BW, 5>(nw, weighted, graphs, jobs, n_jobs, stream);
        default: return hipErrorInvalidValue;
        }
    }
    if (shape == kBfsWide1024) {
        switch (planes) {
        case 4: return launch_bfs_wide1024_p<BW, 4>(nw, weighted, graphs, jobs, n_jobs, stream);
        case 5: return launch_bfs_wide1024_p<BW, 5>(nw, weighted, graphs, jobs, n_jobs, stream);
        default: return hipErrorInvalidValue;
        }
    }
    if (shape == kBfsFront) {
        switch (planes) {
        case 4: return launch_bfs_front_p<BW, 4>(nw, weighted, graphs, jobs, n_jobs, stream);
        case 5: return launch_bfs_front_p<BW, 5>(nw, weighted, graphs, jobs, n_jobs, stream);
        default: return hipErrorInvalidValue;
        }
    }
    if (shape != kBfsNarrow) return hipErrorInvalidValue;
    switch (planes) {
    case 4: return launch_bfs_p<BW, 4>(nw, weighted, graphs, jobs, n_jobs, stream);
    case 5: return launch_bfs_p<BW, 5>(nw, weighted, graphs, jobs, n_jobs, stream);
    case 7: return launch_bfs_p<BW, 7>(nw, weighted, graphs, jobs, n_jobs, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace qc
