// Host-side helpers that need no GPU (see qc_host.h).
#include "qc_host.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <numeric>

#include "qc_internal.h"

namespace qc {

qc_status validate_csr(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col,
                       bool canonicalize, std::vector<int32_t> &rp_out,
                       std::vector<int32_t> &col_out, bool directed)
{
    if (n < 1 || n > kMaxNodes) return QC_E_INVAL;
    if (nnz < 0 || nnz >= kMaxEdges) return QC_E_INVAL;
    if (!row_ptr) return QC_E_INVAL;
    if (nnz > 0 && !col) return QC_E_INVAL;
    if (row_ptr[0] != 0 || (int64_t)row_ptr[n] != nnz) return QC_E_INVAL;
    for (int32_t i = 0; i < n; ++i)
        if (row_ptr[i + 1] < row_ptr[i]) return QC_E_INVAL;
    for (int64_t e = 0; e < nnz; ++e)
        if (col[e] < 0 || col[e] >= n) return QC_E_INVAL;

    if (canonicalize) {
        std::vector<std::vector<int32_t>> adj(n);
        for (int32_t i = 0; i < n; ++i)
            for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
                const int32_t j = col[e];
                if (j == i) continue;
                adj[i].push_back(j);
                if (!directed) adj[j].push_back(i);
            }
        rp_out.assign(n + 1, 0);
        col_out.clear();
        for (int32_t i = 0; i < n; ++i) {
            auto &a = adj[i];
            std::sort(a.begin(), a.end());
            a.erase(std::unique(a.begin(), a.end()), a.end());
            col_out.insert(col_out.end(), a.begin(), a.end());
            rp_out[i + 1] = (int32_t)col_out.size();
        }
        if ((int64_t)col_out.size() >= ((int64_t)1 << 31)) return QC_E_INVAL;
        return QC_OK;
    }

    for (int32_t i = 0; i < n; ++i) {
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            if (col[e] == i) return QC_E_NOT_SYMMETRIC;
            if (e > row_ptr[i] && col[e] <= col[e - 1]) return QC_E_NOT_SYMMETRIC;
        }
    }
    for (int32_t i = 0; i < n && !directed; ++i) {
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const int32_t j = col[e];
            if (!std::binary_search(col + row_ptr[j], col + row_ptr[j + 1], i))
                return QC_E_NOT_SYMMETRIC;
        }
    }
    rp_out.assign(row_ptr, row_ptr + n + 1);
    col_out.assign(col, col + nnz);
    return QC_OK;
}

std::vector<uint32_t> pack_in_edges(int32_t n, const std::vector<int32_t> &rp,
                                    const std::vector<int32_t> &col, bool directed)
{
    const int64_t nnz = (int64_t)col.size();
    std::vector<uint32_t> edges(((nnz + 3) / 4) * 4 + 4, 0u);
    if (!directed) {
        for (int32_t i = 0; i < n; ++i)
            for (int32_t e = rp[i]; e < rp[i + 1]; ++e)
                edges[e] = ((uint32_t)i << 16) | (uint32_t)col[e];
        return edges;
    }
    // transpose: bucket the edges tail -> head by head (counting sort), so a
    // head's entries are contiguous and its tails ascending
    std::vector<int64_t> start(n + 1, 0);
    for (int64_t e = 0; e < nnz; ++e) ++start[col[e] + 1];
    for (int32_t v = 0; v < n; ++v) start[v + 1] += start[v];
    for (int32_t i = 0; i < n; ++i)
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e)
            edges[start[col[e]]++] = ((uint32_t)col[e] << 16) | (uint32_t)i;
    return edges;
}

namespace {

// One greedy pass over a window of `nl` groups, lanes visited in `order`;
// returns the pass's cost (sum over the 8 slots of the busiest bank's count).
int spread_window(const uint32_t (*in)[8], int nl, const int *order, int nodes_per_word, int banks,
                  uint32_t (*out)[8])
{
    bool used[64][8] = {};
    int32_t cur[64];
    for (int l = 0; l < nl; ++l) cur[l] = -1;
    int cost_total = 0;
    for (int k = 0; k < 8; ++k) {
        int occ[64] = {};
        uint32_t bank_words[64][8];
        int busiest = 0;
        for (int li = 0; li < nl; ++li) {
            const int l = order[li];
            // an open run (its row has edges left) must be continued
            bool open = false;
            for (int j = 0; j < 8; ++j)
                if (!used[l][j] && (int32_t)(in[l][j] >> 16) == cur[l]) open = true;
            int best = -1, best_cost = 1 << 30;
            uint32_t best_word = 0;
            for (int j = 0; j < 8; ++j) {
                if (used[l][j]) continue;
                if (open && (int32_t)(in[l][j] >> 16) != cur[l]) continue;
                const uint32_t word = (in[l][j] & 0xFFFFu) / (uint32_t)nodes_per_word;
                const int b = (int)(word % (uint32_t)banks);
                int cost = occ[b] + 1;
                for (int q = 0; q < occ[b] && q < 8; ++q)
                    if (bank_words[b][q] == word) cost = 0;   // same word: broadcast
                if (cost < best_cost) {
                    best_cost = cost;
                    best = j;
                    best_word = word;
                }
            }
            used[l][best] = true;
            out[l][k] = in[l][best];
            cur[l] = (int32_t)(in[l][best] >> 16);
            if (best_cost > 0) {
                const int b = (int)(best_word % (uint32_t)banks);
                if (occ[b] < 8) bank_words[b][occ[b]] = best_word;
                ++occ[b];
                busiest = std::max(busiest, occ[b]);
            }
        }
        cost_total += busiest;
    }
    return cost_total;
}

}  // namespace

void spread_gather_banks(std::vector<uint32_t> &edges, int64_t nnz, int nodes_per_word,
                         int banks)
{
    if (banks <= 0 || banks > 64) return;
    const int lanes = banks;
    const int64_t groups = nnz / 8;   // groups made of real edges only
    uint32_t in[64][8], out[64][8], best_out[64][8];
    int order[64];
    uint64_t rng = 0x9E3779B97F4A7C15ull;   // fixed seed: the order is deterministic
    for (int64_t g0 = 0; g0 < groups; g0 += lanes) {
        const int nl = (int)std::min<int64_t>(lanes, groups - g0);
        for (int l = 0; l < nl; ++l)
            for (int j = 0; j < 8; ++j) in[l][j] = edges[(g0 + l) * 8 + j];
        // the greedy in lane order, then in kSpreadTries - 1 shuffled lane
        // orders; the cheapest result is kept
        int best_cost = 1 << 30;
        for (int t = 0; t < kSpreadTries; ++t) {
            for (int l = 0; l < nl; ++l) order[l] = l;
            if (t > 0)
                for (int l = nl - 1; l > 0; --l) {   // Fisher-Yates with a 64-bit LCG
                    rng = rng * 6364136223846793005ull + 1442695040888963407ull;
                    std::swap(order[l], order[(int)((rng >> 33) % (uint64_t)(l + 1))]);
                }
            const int c = spread_window(in, nl, order, nodes_per_word, banks, out);
            if (c < best_cost) {
                best_cost = c;
                for (int l = 0; l < nl; ++l)
                    for (int j = 0; j < 8; ++j) best_out[l][j] = out[l][j];
            }
        }
        for (int l = 0; l < nl; ++l)
            for (int j = 0; j < 8; ++j) edges[(g0 + l) * 8 + j] = best_out[l][j];
    }
}

qc_status subdivide_weighted(int32_t n, const std::vector<int32_t> &rp,
                             const std::vector<int32_t> &col, const uint8_t *w, bool directed,
                             int32_t &n_out, std::vector<int32_t> &rp_out,
                             std::vector<int32_t> &col_out)
{
    if (!w && !col.empty()) return QC_E_INVAL;
    int64_t total = n;
    for (int32_t u = 0; u < n; ++u) {
        for (int32_t e = rp[u]; e < rp[u + 1]; ++e) {
            const int32_t v = col[e];
            if (w[e] < 1 || w[e] > kMaxDist) return QC_E_INVAL;
            if (!directed) {
                // the reverse entry exists (canonical CSR); it must agree
                const int32_t *b = col.data() + rp[v], *f = col.data() + rp[v + 1];
                const int32_t *it = std::lower_bound(b, f, u);
                if (it == f || *it != u || w[it - col.data()] != w[e]) return QC_E_NOT_SYMMETRIC;
                if (v < u) continue;
            }
            total += w[e] - 1;
        }
    }
    if (total > kMaxNodes) return QC_E_INVAL;
    n_out = (int32_t)total;
    std::vector<std::vector<int32_t>> adj(n_out);
    int32_t next = n;
    auto link = [&](int32_t a, int32_t b) {
        adj[a].push_back(b);
        if (!directed) adj[b].push_back(a);
    };
    for (int32_t u = 0; u < n; ++u) {
        for (int32_t e = rp[u]; e < rp[u + 1]; ++e) {
            const int32_t v = col[e];
            if (!directed && v < u) continue;
            int32_t prev = u;
            for (int k = 1; k < w[e]; ++k) {   // w - 1 new nodes along the edge
                link(prev, next);
                prev = next++;
            }
            link(prev, v);
        }
    }
    rp_out.assign(n_out + 1, 0);
    col_out.clear();
    for (int32_t v = 0; v < n_out; ++v) {
        std::sort(adj[v].begin(), adj[v].end());
        col_out.insert(col_out.end(), adj[v].begin(), adj[v].end());
        rp_out[v + 1] = (int32_t)col_out.size();
    }
    return QC_OK;
}

static int32_t uf_find(std::vector<int32_t> &p, int32_t x)
{
    while (p[x] != x) {
        p[x] = p[p[x]];
        x = p[x];
    }
    return x;
}

int32_t count_components(int32_t n, const std::vector<int32_t> &rp, const std::vector<int32_t> &col,
                         std::vector<int32_t> *comp_size)
{
    std::vector<int32_t> p(n);
    std::iota(p.begin(), p.end(), 0);
    int32_t comps = n;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            int32_t a = uf_find(p, i), b = uf_find(p, col[e]);
            if (a != b) {
                p[std::max(a, b)] = std::min(a, b);
                --comps;
            }
        }
    if (comp_size) {
        std::vector<int32_t> size(n, 0);
        for (int32_t i = 0; i < n; ++i) ++size[uf_find(p, i)];
        comp_size->assign(n, 0);
        for (int32_t i = 0; i < n; ++i) (*comp_size)[i] = size[uf_find(p, i)];
    }
    return comps;
}

std::vector<int32_t> source_order(int32_t n, const std::vector<int32_t> &rp,
                                  const std::vector<int32_t> &col, int32_t n_src, int sweeps,
                                  int32_t *dist_bound)
{
    auto deg = [&](int32_t v) { return rp[v + 1] - rp[v]; };
    // component labels (BFS) and each component's first seed
    std::vector<int32_t> comp(n, -1), queue(n), dist(n), seed;
    for (int32_t v = 0; v < n; ++v) {
        if (comp[v] >= 0) continue;
        const int32_t c = (int32_t)seed.size();
        int32_t head = 0, tail = 0, best = v;
        queue[tail++] = v;
        comp[v] = c;
        while (head < tail) {
            const int32_t u = queue[head++];
            if (deg(u) > deg(best) || (deg(u) == deg(best) && u < best)) best = u;
            for (int32_t e = rp[u]; e < rp[u + 1]; ++e)
                if (comp[col[e]] < 0) {
                    comp[col[e]] = c;
                    queue[tail++] = col[e];
                }
        }
        seed.push_back(best);
    }
    const size_t n_comp = seed.size();
    std::vector<int32_t> lo(n, 0), hi(n, INT32_MAX), ecc(n_comp), far(n_comp);
    for (int s = 0; s < sweeps; ++s) {
        // one multi-source BFS: each node is reached from its own component's seed
        std::fill(dist.begin(), dist.end(), -1);
        int32_t head = 0, tail = 0;
        for (int32_t x : seed) {
            dist[x] = 0;
            queue[tail++] = x;
        }
        while (head < tail) {
            const int32_t u = queue[head++];
            for (int32_t e = rp[u]; e < rp[u + 1]; ++e)
                if (dist[col[e]] < 0) {
                    dist[col[e]] = dist[u] + 1;
                    queue[tail++] = col[e];
                }
        }
        for (size_t c = 0; c < n_comp; ++c) {
            ecc[c] = 0;
            far[c] = seed[c];
        }
        for (int32_t i = 0; i < tail; ++i) {   // BFS order: the first node at the largest distance
            const int32_t u = queue[i], c = comp[u];
            if (dist[u] > ecc[c]) {
                ecc[c] = dist[u];
                far[c] = u;
            }
        }
        for (int32_t v = 0; v < n; ++v) {
            const int32_t d = dist[v], e = ecc[comp[v]];
            lo[v] = std::max(lo[v], std::max(d, e - d));
            hi[v] = std::min(hi[v], e + d);
        }
        seed = far;
    }
    if (dist_bound) {
        int32_t b = 0;
        for (int32_t v = 0; v < n; ++v) b = std::max(b, hi[v]);
        *dist_bound = b;
    }
    std::vector<int32_t> order(n_src);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return lo[a] != lo[b] ? lo[a] < lo[b] : hi[a] < hi[b];
    });
    return order;
}

int planes_for(int32_t dmax)
{
    if (dmax >= 0 && dmax <= 15) return 4;
    if (dmax >= 0 && dmax <= 31) return 5;
    return 7;
}

BfsPlan plan_bfs_shape(int32_t n, int32_t dmax, int shape, int max_bw)
{
    static const int kNarrow[] = {1, 2, 4, 6, 8, 10, 12};
    static const int kWide[] = {16, 24, 32, 38, 39};
    static const int kWide1024[] = {14, 16, 18, 19};
    static const int kFront[] = {4, 8, 12, 14, 16};
    const int planes = planes_for(dmax);
    const bool two = shape != kBfsNarrow;
    BfsPlan none = {0, 0, planes, 0, shape};
    if (two && planes >= 7) return none;
    const int threads = (shape == kBfsWide) ? kBfsThreadsWide : kBfsThreads;
    // words per thread that fit the registers without spills: three-field
    // shape 12 (10 with 7 planes and 64-source batches); two-field 512-thread
    // 39 with 4 planes, 32 with 5; two-field 1024-thread 19 with 4, 16 with 5
    // (18 for batches of 32); seen in registers 16 with 4, 14 with 5
    int max_nw;
    const int *opts;
    int nopts;
    if (shape == kBfsNarrow) {
        max_nw = 12;
        opts = kNarrow;
        nopts = 7;
    } else if (shape == kBfsWide) {
        max_nw = planes <= 4 ? 39 : 32;
        opts = kWide;
        nopts = 5;
    } else if (shape == kBfsFront) {
        // seen in registers: (planes + 1) registers per owned word
        max_nw = planes <= 4 ? 16 : 14;
        opts = kFront;
        nopts = 5;
    } else {
        max_nw = planes <= 4 ? 19 : 18;
        opts = kWide1024;
        nopts = 4;
    }
    for (int bw : {64, 32, 16, 8, 4}) {
        if (bw > max_bw || (two && bw < 8)) continue;
        const int64_t words = ((int64_t)n * bw + 31) / 32;  // 32-bit words of one bit field
        const int64_t need = (words + threads - 1) / threads;
        for (int k = 0; k < nopts; ++k) {
            const int nw = opts[k];
            if (nw > max_nw) break;
            if (bw == 64 && (nw % 2)) continue;
            if (bw == 64 && shape == kBfsNarrow && planes >= 7 && nw > 10) continue;
            if (shape == kBfsWide1024 && planes == 5 && nw > 16 && bw != 32) continue;
            // seen in registers with 4 planes: 16 words rather than 14, so a
            // thread owns its words four at a time (16-byte LDS accesses,
            // the decode's register transpose); measured faster on the sweep
            if (shape == kBfsFront && planes <= 4 && nw == 14) continue;
            if (nw >= need) {
                BfsPlan p;
                p.bw = bw;
                p.nw = nw;
                p.planes = planes;
                p.n_batches = (int)((n + bw - 1) / bw);
                p.shape = shape;
                return p;
            }
        }
    }
    return none;
}

BfsPlan plan_bfs_policy(int32_t n, int32_t dmax, int max_bw, bool front_first)
{
    // With front_first, the shape with seen in registers (pull from the
    // frontier at the two-field LDS budget) when the graph fits it at the
    // widest width; otherwise the widest batch wins, at equal width more
    // threads per workgroup, and pulling from the frontier (fewer atomics)
    // before pulling from seen.
    const BfsPlan front = plan_bfs_shape(n, dmax, kBfsFront, max_bw);
    if (front_first && front.bw == max_bw) return front;
    BfsPlan best = front;
    if (!front_first) best.bw = 0;
    for (int shape : {kBfsNarrow, kBfsWide1024, kBfsWide}) {
        const BfsPlan p = plan_bfs_shape(n, dmax, shape, max_bw);
        if (p.bw > best.bw) best = p;
    }
    return best.bw > 0 ? best : front;
}

BfsPlan plan_bfs(int32_t n, int32_t dmax)
{
    // QC_BFS_SHAPE=<shape> (a switch for measurements and tests): that
    // workgroup shape whenever the graph fits it
    if (const char *f = getenv("QC_BFS_SHAPE")) {
        const int shape = atoi(f);
        if (shape >= kBfsNarrow && shape <= kBfsFront) {
            const BfsPlan p = plan_bfs_shape(n, dmax, shape);
            if (p.bw > 0) return p;
        }
    }
    // At most kBfsFullWidth sources per batch (timed on the sweep graphs,
    // 32-source batches beat 64-source ones), the seen-in-registers shape
    // first.
    return plan_bfs_policy(n, dmax, kBfsFullWidth, true);
}

static void split_f32(double x, float &hi, float &lo)
{
    hi = (float)x;
    lo = (float)(x - (double)hi);
}

static uint16_t to_bf16(double x)
{
    // FP32 first, then round to nearest even at 8 significant bits
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

void weight_tables(const double *sigmas, int n_sigmas, int K, std::vector<double> &w64,
                   std::vector<double> &u64, std::vector<double> &inv_a, std::vector<float> &w32c,
                   std::vector<uint16_t> &wbf16)
{
    w64.assign((size_t)n_sigmas * K, 0.0);
    u64.assign((size_t)n_sigmas * K, 0.0);
    inv_a.assign(n_sigmas, 0.0);
    w32c.assign((size_t)n_sigmas * K * 4, 0.0f);
    wbf16.assign((size_t)n_sigmas * K * 2, 0);
    for (int s = 0; s < n_sigmas; ++s) {
        const double a = (2.0 * sigmas[s]) * sigmas[s];
        inv_a[s] = 1.0 / a;
        for (int k = 0; k < K; ++k) {
            const double w = exp(-(double)(k * k) / a);
            const double u = ((double)(k * k) * w) / a;
            w64[(size_t)s * K + k] = w;
            u64[(size_t)s * K + k] = u;
            float *c = &w32c[((size_t)s * K + k) * 4];
            split_f32(w, c[0], c[1]);
            split_f32(u, c[2], c[3]);
            wbf16[((size_t)s * K + k) * 2 + 0] = to_bf16(w);
            wbf16[((size_t)s * K + k) * 2 + 1] = to_bf16(u);
        }
    }
}

qc_status validate_sigmas(const double *sigmas, int32_t n_sigmas)
{
    if (!sigmas || n_sigmas < 1 || n_sigmas > 1024) return QC_E_INVAL;
    for (int32_t s = 0; s < n_sigmas; ++s)
        if (!(sigmas[s] > 0.0) || !isfinite(sigmas[s])) return QC_E_INVAL;
    return QC_OK;
}

}  // namespace qc
