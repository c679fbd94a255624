// Host-side helpers of the library that need no GPU: CSR validation and
// canonicalisation, connected components, BFS launch planning, weight tables.
#pragma once

#include <stdint.h>

#include <vector>

#include "qc.h"

namespace qc {

// Validate a CSR for qc_graph_create. Returns QC_OK, QC_E_INVAL (pointers,
// sizes, ranges) or QC_E_NOT_SYMMETRIC (ordering, duplicates, self-loops,
// and, unless `directed`, asymmetry). With `canonicalize`, only the range
// checks apply and the canonical form is written to rp_out / col_out (rows
// sorted, duplicates and self-loops dropped, symmetrised unless `directed`).
qc_status validate_csr(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col,
                       bool canonicalize, std::vector<int32_t> &rp_out,
                       std::vector<int32_t> &col_out, bool directed = false);

// Packed in-edge list of a canonical CSR for the BFS pull: one entry
// (head << 16) | tail per edge tail -> head, heads ascending, padded with
// no-op (0, 0) entries to a multiple of 4 plus one all-zero quad. For an
// undirected (symmetric) CSR this is the CSR itself.
std::vector<uint32_t> pack_in_edges(int32_t n, const std::vector<int32_t> &rp,
                                    const std::vector<int32_t> &col, bool directed);

// Reorders the packed edges inside each group of 8 (one thread's share of a
// pull round) so that the gathers of one LDS pass (the same slot of `banks`
// consecutive groups, one group per lane) fall into distinct banks where
// possible: a greedy choice per slot and lane of the edge whose field word
// shares its bank with the fewest words already chosen (a word already chosen
// costs nothing: lanes reading one word are served together), repeated for
// kSpreadTries lane orders (the first the natural one, the others shuffled by
// a fixed-seed generator), keeping the order whose slots' busiest banks add
// up to the least. The edges of
// one row stay contiguous within a group, so the pull's run merging (one
// atomic per run) is unchanged; any order of the edges gives the same search.
// `nodes_per_word` nodes share a field word (32 / batch width, at least 1);
// 64-bit words (batches of 64) span two 4-byte banks, so pass banks = 16.
constexpr int kSpreadTries = 8;
void spread_gather_banks(std::vector<uint32_t> &edges, int64_t nnz, int nodes_per_word,
                         int banks);

// Number of connected components (union-find over the canonical CSR); if
// comp_size is given it receives, for every node, the size of its component.
int32_t count_components(int32_t n, const std::vector<int32_t> &rp, const std::vector<int32_t> &col,
                         std::vector<int32_t> *comp_size = nullptr);

// The order in which the BFS takes its sources (batch k holds entries
// k*bw .. k*bw+bw-1). A batch searches until its farthest-reaching source is
// done, so sources with similar eccentricities go together: nodes sorted by
// a lower bound on their eccentricity, then by an upper bound. Both bounds
// come from `sweeps` BFS sweeps over every component of the undirected graph
// (rp, col) of n nodes: from its highest-degree node, then each time from the
// node the previous sweep reached last; for a sweep from c with eccentricity
// e(c), every node v of the component has max(d(v,c), e(c) - d(v,c)) <= e(v)
// <= e(c) + d(v,c). The order lists the first n_src nodes (the sources).
// If dist_bound is given it receives the largest upper bound, a bound on
// every finite distance of the graph.
std::vector<int32_t> source_order(int32_t n, const std::vector<int32_t> &rp,
                                  const std::vector<int32_t> &col, int32_t n_src, int sweeps,
                                  int32_t *dist_bound = nullptr);

// Integer edge weights (Section 3.1: a path's length is the sum of its edges'
// weights): an edge of weight w >= 2 becomes a path of w unit edges through
// w - 1 new nodes numbered from n on, so unit-edge hop distances between the
// original nodes are the weighted shortest-path lengths. `w` holds one weight
// (1..126) per CSR entry of the canonical CSR (rp, col). Returns QC_E_INVAL
// for a weight outside 1..126 or more than kMaxNodes nodes in all, and
// QC_E_NOT_SYMMETRIC when the two entries of an undirected edge differ.
qc_status subdivide_weighted(int32_t n, const std::vector<int32_t> &rp,
                             const std::vector<int32_t> &col, const uint8_t *w, bool directed,
                             int32_t &n_out, std::vector<int32_t> &rp_out,
                             std::vector<int32_t> &col_out);

// BFS launch shape for a graph of n nodes whose largest finite distance is
// dmax (or -1 while unknown): `planes` distance bit-planes (enough for dmax,
// 7 when unknown), and the widest batch of sources whose LDS bit fields and
// register planes fit one workgroup, with nw 32-bit words per thread per
// field. `shape` (kBfsNarrow, kBfsWide, kBfsWide1024, kBfsFront): batches of
// at most kBfsFullWidth sources; the seen-in-registers shape when it fits
// that width, else the widest batch of any shape (three fields before the
// two-field 1024-thread shape before the 512-thread one; the two-field and
// seen-in-registers shapes only with 4-5 planes).
struct BfsPlan { int bw; int nw; int planes; int n_batches; int shape; };
BfsPlan plan_bfs(int32_t n, int32_t dmax);
// The planner's rule with another widest batch (max_bw) and with or without
// the seen-in-registers shape first (the batch autotuner's candidates).
BfsPlan plan_bfs_policy(int32_t n, int32_t dmax, int max_bw, bool front_first);
// The plan of one shape alone (bw = 0 when n does not fit).
BfsPlan plan_bfs_shape(int32_t n, int32_t dmax, int shape, int max_bw = 64);
int planes_for(int32_t dmax);

// Histogram row length for a largest finite distance dmax.
inline int bins_for(int dmax) { return dmax < 32 ? 32 : (dmax < 64 ? 64 : 128); }

// Weight tables of one sigma list (host C library exp, FP64):
//   w64[s*K + k] = exp(-(k*k) / a_s),  a_s = (2 sigma_s) sigma_s
//   u64[s*K + k] = (k*k) * w64 / a_s
//   inv_a[s]     = 1 / a_s
//   w32c[(s*K + k)*4 + {0,1,2,3}] = FP32 hi/lo splits of w64 and u64
//   wbf16[(s*K + k)*2 + {0,1}] = BF16 roundings of w64 and u64
void weight_tables(const double *sigmas, int n_sigmas, int K, std::vector<double> &w64,
                   std::vector<double> &u64, std::vector<double> &inv_a,
                   std::vector<float> &w32c, std::vector<uint16_t> &wbf16);

// Check a sigma list (count 1..1024, every value finite and > 0).
qc_status validate_sigmas(const double *sigmas, int32_t n_sigmas);

}  // namespace qc
