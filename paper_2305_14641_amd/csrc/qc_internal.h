// Internal declarations shared by the host runtime and the HIP kernels.
// Not part of the public ABI (include/qc.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qc {

// Largest finite hop distance an int8 distance can hold; reaching level 127
// in a breadth-first search is reported as an overflow.
constexpr int kMaxDist = 126;
// Largest supported node count: edges are packed as (row << 16 | col).
constexpr int kMaxNodes = 65536;
// Edge entries must stay below this (also after subdividing weighted edges):
// the packed edge list the BFS streams then spans less than 2 GB, within the
// 32-bit byte offsets of its buffer loads.
constexpr int64_t kMaxEdges = (int64_t)1 << 29;
// Threads per workgroup of the multi-source BFS: the three-field shape (and
// the 1024-thread two-field one) and the 512-thread two-field ("wide") shape.
constexpr int kBfsThreads = 1024;
constexpr int kBfsThreadsWide = 512;
// BFS workgroup shapes: three fields x 1024 threads, two fields x 512
// threads, two fields x 1024 threads, and two LDS fields x 1024 threads with
// the third (`seen`) in registers.
enum { kBfsNarrow = 0, kBfsWide = 1, kBfsWide1024 = 2, kBfsFront = 3 };
// Widest batch of sources the planner picks: 64-source batches halve the
// batches but double each workgroup's LDS and registers, while the search is
// bound by the latency of its LDS gathers, which more wavefronts per CU hide.
constexpr int kBfsFullWidth = 32;
// Added to a shape at launch: the graph carries integer edge weights.
constexpr int kBfsWeighted = 16;
// Row bias of the packed edge list for a BFS launch shape. The pull's atomic
// goes to nxt[row], and nxt starts one field (F words) after the field the
// pull gathers from; when that offset in bytes exceeds the 16-bit offset of
// an LDS instruction, every address would need an add. The host then packs
// each edge's row as row + F * (nodes per word), so that the row field alone
// addresses nxt from the start of the fields. Zero (rows as they are) when
// the offset fits, or when the biased rows would not fit 16 bits.
constexpr int bfs_row_bias(int bw, int nw, int shape)
{
    const int threads = ((shape & ~kBfsWeighted) == kBfsWide) ? kBfsThreadsWide : kBfsThreads;
    const int words = (bw == 64 ? nw / 2 : nw) * threads;   // one field
    const int word_bytes = bw == 64 ? 8 : 4;
    const int per = bw >= 32 ? 1 : 32 / bw;                 // nodes per word
    if ((long long)words * word_bytes <= 65535) return 0;
    if (2LL * words * per > 65536) return 0;
    return words * per;
}

// Row stride of a distance matrix the library owns: rows start on 128-byte
// lines, so that the search's 256-byte stores of a row cover whole lines.
constexpr int64_t owned_ld(int32_t n) { return ((int64_t)n + 127) & ~(int64_t)127; }

// 32-bit words of each LDS bit field one BFS thread owns at most (the three
// fields of 13 x 1024 words fill 156 KB of the 160 KB LDS).
constexpr int kBfsMaxWordsPerThread = 13;

// Global-memory vector type for 16-byte loads through an explicit global
// address-space pointer (keeps loads off the flat path).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) u32x4 *global_u4;
// Word 3 of a buffer resource for raw (untyped, unswizzled) loads on gfx9-family
// GPUs: 32-bit data format, range checked against the byte count in word 2.
constexpr int kBufferWord3 = 0x00020000;

// Device-visible description of one graph and its resident buffers.
// Kernels receive an array of these plus a job table, so one launch can
// serve one graph or many.
struct GraphDev {
    int32_t n;
    int32_t K;            // histogram row length (multiple of 32)
    int32_t dmax;         // largest finite distance (valid after the BFS)
    int32_t n_sigmas;
    int64_t nnz;
    const int32_t *row_ptr;   // [n+1]
    const int32_t *col;       // [nnz]
    // The graph the BFS walks: the same CSR, or (integer edge weights) the
    // graph with every edge of weight w subdivided into w unit edges; its
    // first n nodes are the graph's nodes.
    int32_t n_bfs;
    int32_t pad_bfs;
    int64_t nnz_bfs;              // its edges (= nnz without weights)
    const int32_t *bfs_row_ptr;   // [n_bfs+1]
    const int32_t *bfs_col;
    const int32_t *order;     // [n] nodes by decreasing degree within windows of kOrderWindow
    // The descent's neighbour lists in sliced ELL layout: slice w holds the
    // nodes order[64w .. 64w+63], slot-major (entry k of the slice's lane l
    // at sell_col[sell_off[w] + 64k + l]), so the lanes of a wavefront read
    // the k-th neighbours of their nodes from one contiguous 256-byte row.
    const int32_t *sell_col;  // [sell_off[n_slices] + 64 * kGgdPad]
    const int32_t *sell_off;  // [n_slices + 1]
    const int32_t *sell_deg;  // [n] degree of node order[t]
    const int32_t *src;       // [n] BFS sources in batch order (a permutation of 0..n-1)
    const uint32_t *edges;    // packed in-edges (row << 16) | col of the BFS graph, rows ascending
    int8_t *dist;             // [n rows of ld] row-major
    int64_t ld;               // its row stride: n for a caller's matrix, owned_ld(n) for the library's
    int32_t *hist;            // [n*K]
    float *psi;               // [n_sigmas*n] resident
    float *v;                 // resident, sigma groups of kVGroup interleaved by node (v_index)
    double *v64;              // [n_sigmas*n] canonical FP64 V, or null (FP32C potentials)
    const double *w64;        // [n_sigmas*K] exp(-k^2/a), host C library exp
    const double *u64;        // [n_sigmas*K] k^2 * w / a
    const double *inv_a;      // [n_sigmas] 1/a, a = (2 sigma) sigma
    const float *w32c;        // [n_sigmas*K*4] FP32 (w_hi, w_lo, u_hi, u_lo)
    const uint16_t *wbf16;    // [n_sigmas*K*2] BF16 (w, u) pairs for the matrix-core variant
    int32_t *parent;          // [n_sigmas][n] descent parents, node order[t]'s at t
    int32_t *status;          // [2]: 0 largest finite distance, 1 overflow flag
    unsigned long long *recheck;  // count of FP64 re-decided nodes
    // Search work counted by the BFS, or null: [0] edge visits (every edge
    // entry of every pulled level, plus the row entries the first level
    // pushes from the sources), [1] bytes of the bit fields those visits
    // gathered from LDS.
    unsigned long long *visits;
};

// graph index, first source, and the number of (source, node) pairs the
// batch's sources can reach (sum of their component sizes): the search stops
// as soon as that many pairs have been found.
struct BfsJob { int32_t g; int32_t s0; uint32_t target; uint32_t pad; };
struct NodeJob { int32_t g; int32_t i0; int64_t out_off; };  // graph, first node, output offset

// Rows of the distance matrix one histogram job covers, by bin count
// (wavefronts per workgroup x rows per wavefront; see launch_hist).
inline int hist_rows_per_job(int K) { return 32; }
// Nodes per job of the potential and descent kernels.
constexpr int kNodesPerJob = 256;
// Window (in nodes, a multiple of kNodesPerJob) within which the descent's
// thread order sorts nodes by degree.
#ifndef QC_ORDER_WINDOW
#define QC_ORDER_WINDOW 4096
#endif
constexpr int kOrderWindow = QC_ORDER_WINDOW;
// Neighbours one descent thread loads per round (the sliced neighbour lists
// carry this many padding rows after the last slice).
constexpr int kGgdPad = 4;
// The resident FP32 V keeps the sigmas in groups of kVGroup, interleaved by
// node: entry (s, i) at v_index(n, s, i), so the descent, which decides a
// node for a group of sigmas, gathers a neighbour's values with one 16-byte
// load. Allocations round the sigma count up to a whole group.
constexpr int kVGroup = 4;
__host__ __device__ inline int64_t v_index(int n, int s, int i)
{
    return ((int64_t)(s / kVGroup) * n + i) * kVGroup + (s % kVGroup);
}
inline int64_t v_floats(int n, int n_sigmas)
{
    return (int64_t)((n_sigmas + kVGroup - 1) / kVGroup) * kVGroup * n;
}

// Sigmas one descent thread decides (when the launch covers that many).
#ifndef QC_GGD_SIGMAS
#define QC_GGD_SIGMAS 4
#endif
constexpr int kGgdSigmas = QC_GGD_SIGMAS;
// BFS sweeps per component behind the eccentricity bounds of the source order
constexpr int kSourceSweeps = 4;

// Relative FP32 gap under which a descent comparison is re-decided in FP64.
// It exceeds twice the worst FP32 error of V for both FP64ACC (about 2^-24)
// and FP32C (about 7 * 2^-24) potentials.
constexpr float kTieTau = 1.9073486328125e-06f;  // 2^-19

// ---- launchers (qc_kernels.hip); each returns hipSuccess or the launch error.

// Write one descriptor into device memory in stream order.
hipError_t launch_set_desc(GraphDev *dst, const GraphDev &src, hipStream_t stream);

// Multi-source BFS over `n_jobs` (graph, source-batch) jobs; every graph of the
// launch must share the batch width `bw`, words-per-thread `nw` and the
// number of distance bit-planes `planes` (4, 5 or 7; levels < 2^planes).
// `shape` is kBfsNarrow, kBfsWide or kBfsWide1024, plus kBfsWeighted for a
// graph with integer edge weights.
hipError_t launch_bfs(int bw, int nw, int planes, int shape, const GraphDev *graphs,
                      const BfsJob *jobs, int n_jobs, hipStream_t stream);
// One batch width (qc_bfs_<bw>.hip).
template <int BW>
hipError_t launch_bfs_bw(int nw, int planes, int shape, const GraphDev *graphs, const BfsJob *jobs,
                         int n_jobs, hipStream_t stream);

// Histograms of the resident distance rows (one job = hist_rows_per_job(K)
// rows of one graph). `K` is the shared bin count (32, 64 or 128).
// `variant` picks the workgroup shape (hist_waves): 0 default, 1 half, 2
// double the wavefronts per workgroup.
hipError_t launch_hist(int K, const GraphDev *graphs, const NodeJob *jobs, int n_jobs,
                       hipStream_t stream, int variant = 0);
// Wavefronts per workgroup of histogram variant `variant` for row length K.
int hist_waves(int K, int variant);

// psi/V of every (node, sigma); one job = kNodesPerJob nodes of one graph.
// Optional caller outputs: out[out_off + s*out_ld + (i - i0_of_graph)].
hipError_t launch_potential(int precision, int K, const GraphDev *graphs, const NodeJob *jobs,
                            int n_jobs, float *psi_out, float *v_out, int64_t out_ld,
                            hipStream_t stream);

// Descent parents for sigmas sigma_base .. sigma_base+n_sig-1 of every job.
hipError_t launch_ggd_parent(int tie_mode, const GraphDev *graphs, const NodeJob *jobs,
                             int n_jobs, int sigma_base, int n_sig, hipStream_t stream);

// Pointer jumping, one workgroup per (graph job, sigma); labels of sigma
// sigma_base + y go to labels_base + y*labels_ld + job.out_off. max_n: the
// largest node count among the jobs' graphs (up to 40,704 the rounds run in
// LDS unless `variant` is 1: always in global memory).
hipError_t launch_pointer_jump(const GraphDev *graphs, const NodeJob *jobs, int n_jobs,
                               int sigma_base, int n_sig, int32_t *labels_base,
                               int64_t labels_ld, int max_n, hipStream_t stream, int variant = 0);

// Stage timing (qc_timing.cpp): Timer brackets one launch when enabled.
class StageTimer {
  public:
    StageTimer(int stage, hipStream_t stream);
    ~StageTimer();
  private:
    int stage_;
    hipStream_t stream_;
    void *start_ = nullptr;
    void *stop_ = nullptr;
};
// While alive, the calling thread's stage timers record nothing (and create
// no HIP events).
class StageTimingOff {
  public:
    StageTimingOff();
    ~StageTimingOff();
  private:
    bool prev_;
};

// Algorithm 1 over a dense float distance matrix (qc_dense.hip): rows
// [0, n_rows) of `dist` (row stride `ld` floats), every width of `sigmas`
// (host); writes psi and V as FP64 [n_sigmas][n_rows].
hipError_t launch_dense(const float *dist, int64_t n_rows, int64_t n_cols, int64_t ld,
                        const double *sigmas, int n_sigmas, double *psi, double *v,
                        hipStream_t stream);

// Shortest paths under real edge weights (qc_sssp.hip): one workgroup per
// source s0 .. s0+count-1 over an n-node CSR (device row_ptr; col_w holds
// each entry's column and the bits of its float weight, normal and > 0, as
// consecutive 32-bit words, 8-byte aligned); row s of `dist` (stride
// ld >= n) receives the least binary32 path sums from s (+inf unreached).
// n <= kSsspMaxNodes (the row lives in LDS).
constexpr int kSsspMaxNodes = 32768;
hipError_t launch_sssp(int n, const int32_t *row_ptr, const uint32_t *col_w, float *dist, int64_t ld,
                       int src0, int count, hipStream_t stream);
// FP32 resident copy of an FP64 potential [n_sigmas][n] (v_index layout).
hipError_t launch_v_resident(const double *v64, int n, int n_sigmas, float *v32, hipStream_t stream);

// Fill kernel (used instead of hipMemsetAsync so work can be graph-captured).
hipError_t launch_fill_i32(int32_t *p, int64_t count, int32_t value, hipStream_t stream);
hipError_t launch_fill_u64(unsigned long long *p, int64_t count, hipStream_t stream);

}  // namespace qc
