/*
 * CPU oracle for graph Quantum Clustering (Wang, He, Liu, "Graph Analysis
 * Using a GPU-based Parallel Algorithm: Quantum Clustering").
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library may call, link or
 * include this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg load it. It shares no code with the HIP path.
 *
 * Plain, slow, obviously correct. All floating point is IEEE binary64 with
 * round-to-nearest; build with -ffp-contract=off so no multiply-add is fused.
 * Loops over sources run in parallel (OpenMP) because sources are independent;
 * nothing is blocked, fused or reordered inside one source's computation.
 *
 * Readings of the paper used here (each is argued in the design notes):
 *  - distance between nodes = unweighted hop count of a shortest path
 *    (Section 3.1 defines the distance from edges; the hot path uses hops);
 *    unreachable pairs contribute nothing to the sums (d -> infinity);
 *  - the self term j = i is included in both sums of Algorithm 1
 *    (it adds 1 to psi and 0 to the second-moment sum);
 *  - V is Algorithm 1's result, (1/(2 sigma^2)) * sum1 / sum2, i.e. the
 *    approximate form of Eq. 7 without the constant E - 1/2;
 *  - Algorithm 2 starts from the node itself and moves only to a strictly
 *    lower neighbour; among equal neighbours the smallest id wins (STRICT).
 *    The MERGE variant takes the (V, id)-lexicographic minimum over the node
 *    and its neighbours;
 *  - Algorithm 3 is find-root with path compression: a node's label is the id
 *    of the local minimum its descent ends at;
 *  - canonical FP64 potential (used for every GGD decision): a = (2 sigma) sigma,
 *    w_k = exp(-(k*k)/a) from the C library, S2 = sum_k h_k*w_k and
 *    S1 = sum_k (k*k*h_k)*w_k accumulated in ascending k from +0.0 with a
 *    separate multiply and add, V = (1/a) * (S1/S2), psi = S2.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define QCO_OK 0
#define QCO_E_OVERFLOW 2 /* a finite hop distance above 126 */
#define QCO_E_ARG 1

#define QCO_MAX_DIST 126

/* ------------------------------------------------------------------------
 * Hop distances by breadth-first search (textbook queue BFS), one source.
 * Writes row[v] = hop count from s to v, or -1 if v is unreachable.
 * Returns the eccentricity (largest finite distance), or -1 on overflow.
 */
static int bfs_one(int n, const int32_t *row_ptr, const int32_t *col, int s,
                   int8_t *row, int32_t *queue)
{
    for (int v = 0; v < n; ++v) row[v] = -1;
    int head = 0, tail = 0, ecc = 0;
    row[s] = 0;
    queue[tail++] = s;
    while (head < tail) {
        int u = queue[head++];
        int du = row[u];
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int v = col[e];
            if (row[v] < 0) {
                if (du + 1 > QCO_MAX_DIST) return -1;
                row[v] = (int8_t)(du + 1);
                if (du + 1 > ecc) ecc = du + 1;
                queue[tail++] = v;
            }
        }
    }
    return ecc;
}

/* All-pairs distances for the listed sources: dist[r*n + v] for source srcs[r].
 * dmax_out (may be NULL) gets the largest finite distance seen. */
int qco_bfs_rows(int n, const int32_t *row_ptr, const int32_t *col,
                 int nsrc, const int32_t *srcs, int8_t *dist, int32_t *dmax_out)
{
    if (n <= 0 || nsrc < 0) return QCO_E_ARG;
    int status = QCO_OK;
    int dmax = 0;
#pragma omp parallel
    {
        int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        int local_max = 0, local_bad = 0;
#pragma omp for schedule(dynamic, 8)
        for (int r = 0; r < nsrc; ++r) {
            int ecc = bfs_one(n, row_ptr, col, srcs[r], dist + (size_t)r * n, queue);
            if (ecc < 0) local_bad = 1;
            else if (ecc > local_max) local_max = ecc;
        }
#pragma omp critical
        {
            if (local_bad) status = QCO_E_OVERFLOW;
            if (local_max > dmax) dmax = local_max;
        }
        free(queue);
    }
    if (dmax_out) *dmax_out = dmax;
    return status;
}

/* Shortest-path lengths from s along CSR rows with positive integer edge
 * weights w[e] (Section 3.1: a path's length is the sum of its edges'
 * weights), by Dijkstra's algorithm with a bucket queue (Dial's variant):
 * bucket d lists the nodes whose tentative distance was lowered to d; the
 * buckets are drained in increasing d, and a node becomes final the first
 * time it is drained at its current distance. Every push takes a fresh list
 * entry from `pool` (node, next), at most one per edge plus the source.
 * Returns the largest finite distance, or -1 if one exceeds 126. */
static int dijkstra_one(int n, const int32_t *row_ptr, const int32_t *col, const uint8_t *w,
                        int s, int8_t *row, int32_t *dist, int32_t *pool_node,
                        int32_t *pool_next, int32_t *bucket_head)
{
    for (int v = 0; v < n; ++v) {
        dist[v] = INT32_MAX;
        row[v] = -1;
    }
    const int nb = QCO_MAX_DIST + 257;     /* tentative distances stay below 126 + 256 */
    for (int d = 0; d < nb; ++d) bucket_head[d] = -1;
    int used = 0;
    dist[s] = 0;
    pool_node[used] = s;
    pool_next[used] = -1;
    bucket_head[0] = used++;
    int ecc = 0;
    for (int d = 0; d < nb; ++d) {
        for (int it = bucket_head[d]; it >= 0; it = pool_next[it]) {
            int u = pool_node[it];
            if (dist[u] != d || row[u] >= 0) continue;   /* stale or already final */
            if (d > QCO_MAX_DIST) return -1;
            row[u] = (int8_t)d;
            if (d > ecc) ecc = d;
            for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                int v = col[e];
                int nd = d + (int)w[e];
                if (row[v] < 0 && nd < dist[v]) {
                    dist[v] = nd;
                    pool_node[used] = v;
                    pool_next[used] = bucket_head[nd];
                    bucket_head[nd] = used++;
                }
            }
        }
    }
    return ecc;
}

/* Weighted all-pairs distances for the listed sources (weights 1..255). */
int qco_dijkstra_rows(int n, const int32_t *row_ptr, const int32_t *col, const uint8_t *w,
                      int nsrc, const int32_t *srcs, int8_t *dist, int32_t *dmax_out)
{
    if (n <= 0 || nsrc < 0) return QCO_E_ARG;
    const int32_t m = row_ptr[n];
    for (int32_t e = 0; e < m; ++e)
        if (w[e] == 0) return QCO_E_ARG;
    int status = QCO_OK;
    int dmax = 0;
#pragma omp parallel
    {
        int32_t *d = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        int32_t *pn = (int32_t *)malloc(sizeof(int32_t) * ((size_t)m + 1));
        int32_t *px = (int32_t *)malloc(sizeof(int32_t) * ((size_t)m + 1));
        int32_t *head = (int32_t *)malloc(sizeof(int32_t) * (size_t)(QCO_MAX_DIST + 257));
        int local_max = 0, local_bad = 0;
#pragma omp for schedule(dynamic, 8)
        for (int r = 0; r < nsrc; ++r) {
            int ecc = dijkstra_one(n, row_ptr, col, w, srcs[r], dist + (size_t)r * n, d, pn, px, head);
            if (ecc < 0) local_bad = 1;
            else if (ecc > local_max) local_max = ecc;
        }
#pragma omp critical
        {
            if (local_bad) status = QCO_E_OVERFLOW;
            if (local_max > dmax) dmax = local_max;
        }
        free(d);
        free(pn);
        free(px);
        free(head);
    }
    if (dmax_out) *dmax_out = dmax;
    return status;
}

/* Shortest-path lengths from s along CSR rows with positive real edge
 * weights w[e] (Section 3.1: a path's length is the sum of its edges'
 * weights). A path's length is summed in binary32 from the source outward,
 * every partial sum rounded to nearest; d(s, v) is the least such sum over
 * all paths (+infinity when v is unreachable). Dijkstra's algorithm with a
 * binary min-heap of (tentative length, node) entries; an entry popped after
 * its node's length has dropped below it is skipped. The order Dijkstra
 * relies on holds in binary32: a partial sum never decreases along a path,
 * since the weights are positive and rounding is monotone. */
static void sssp_f32_one(int n, const int32_t *row_ptr, const int32_t *col, const float *w, int s,
                         float *row, unsigned char *done, float *hkey, int32_t *hnode)
{
    for (int v = 0; v < n; ++v) {
        row[v] = INFINITY;
        done[v] = 0;
    }
    int size = 0;
    /* push (key, node): sift the new entry up */
#define QCO_HEAP_PUSH(KEY, NODE)                                   \
    do {                                                           \
        int i_ = size++;                                           \
        while (i_ > 0) {                                           \
            int p_ = (i_ - 1) / 2;                                 \
            if (!(hkey[p_] > (KEY))) break;                        \
            hkey[i_] = hkey[p_];                                   \
            hnode[i_] = hnode[p_];                                 \
            i_ = p_;                                               \
        }                                                          \
        hkey[i_] = (KEY);                                          \
        hnode[i_] = (NODE);                                        \
    } while (0)
    row[s] = 0.0f;
    QCO_HEAP_PUSH(0.0f, s);
    while (size > 0) {
        const float key = hkey[0];
        const int u = hnode[0];
        /* pop: move the last entry to the root and sift it down */
        --size;
        if (size > 0) {
            const float lk = hkey[size];
            const int32_t ln = hnode[size];
            int i = 0;
            for (;;) {
                int c = 2 * i + 1;
                if (c >= size) break;
                if (c + 1 < size && hkey[c + 1] < hkey[c]) ++c;
                if (!(hkey[c] < lk)) break;
                hkey[i] = hkey[c];
                hnode[i] = hnode[c];
                i = c;
            }
            hkey[i] = lk;
            hnode[i] = ln;
        }
        if (done[u] || key > row[u]) continue;
        done[u] = 1;
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            const int v = col[e];
            const float nd = key + w[e];   /* binary32 sum, rounded to nearest */
            if (!done[v] && nd < row[v]) {
                row[v] = nd;
                QCO_HEAP_PUSH(nd, v);
            }
        }
    }
#undef QCO_HEAP_PUSH
}

/* Real-weighted shortest-path lengths (binary32) for the listed sources;
 * every weight must be finite and > 0. */
int qco_sssp_f32_rows(int n, const int32_t *row_ptr, const int32_t *col, const float *w,
                      int nsrc, const int32_t *srcs, float *dist)
{
    if (n <= 0 || nsrc < 0) return QCO_E_ARG;
    const int32_t m = row_ptr[n];
    for (int32_t e = 0; e < m; ++e)
        if (!(w[e] > 0.0f) || !isfinite(w[e])) return QCO_E_ARG;
#pragma omp parallel
    {
        unsigned char *done = (unsigned char *)malloc((size_t)n);
        float *hk = (float *)malloc(sizeof(float) * ((size_t)m + 1));
        int32_t *hn = (int32_t *)malloc(sizeof(int32_t) * ((size_t)m + 1));
#pragma omp for schedule(dynamic, 8)
        for (int r = 0; r < nsrc; ++r)
            sssp_f32_one(n, row_ptr, col, w, srcs[r], dist + (size_t)r * n, done, hk, hn);
        free(done);
        free(hk);
        free(hn);
    }
    return QCO_OK;
}

/* Histogram of each listed distance row: hist[r*K + k] = #{v : row_r[v] == k}.
 * Unreachable entries (-1) are not counted. Distances >= K are an error. */
int qco_hist_rows(int n, int nrows, const int8_t *dist, int K, int32_t *hist)
{
    if (K <= 0) return QCO_E_ARG;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int r = 0; r < nrows; ++r) {
        int32_t *h = hist + (size_t)r * K;
        for (int k = 0; k < K; ++k) h[k] = 0;
        const int8_t *row = dist + (size_t)r * n;
        for (int v = 0; v < n; ++v) {
            int d = row[v];
            if (d < 0) continue;
            if (d >= K) { bad = 1; continue; }
            h[d] += 1;
        }
    }
    return bad ? QCO_E_ARG : QCO_OK;
}

/* Histograms of every source without keeping the distance matrix (for graphs
 * whose N*N matrix is too large to hold twice): BFS per source, then count. */
int qco_hist_all(int n, const int32_t *row_ptr, const int32_t *col, int K,
                 int32_t *hist, int32_t *dmax_out)
{
    if (n <= 0 || K <= 0) return QCO_E_ARG;
    int status = QCO_OK, dmax = 0;
#pragma omp parallel
    {
        int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        int8_t *row = (int8_t *)malloc((size_t)n);
        int local_max = 0, local_bad = 0;
#pragma omp for schedule(dynamic, 8)
        for (int s = 0; s < n; ++s) {
            int ecc = bfs_one(n, row_ptr, col, s, row, queue);
            int32_t *h = hist + (size_t)s * K;
            for (int k = 0; k < K; ++k) h[k] = 0;
            if (ecc < 0 || ecc >= K) { local_bad = 1; continue; }
            if (ecc > local_max) local_max = ecc;
            for (int v = 0; v < n; ++v)
                if (row[v] >= 0) h[row[v]] += 1;
        }
#pragma omp critical
        {
            if (local_bad) status = QCO_E_OVERFLOW;
            if (local_max > dmax) dmax = local_max;
        }
        free(row);
        free(queue);
    }
    if (dmax_out) *dmax_out = dmax;
    return status;
}

/* ------------------------------------------------------------------------
 * Algorithm 1 written out literally over one distance row per node:
 *   sum1 += d^2 * exp(-d^2 / (2 sigma^2)),  sum2 += exp(-d^2 / (2 sigma^2))
 *   v = (1 / (2 sigma^2)) * sum1 / sum2,    psi = sum2 (Eq. 2)
 * j runs over all nodes in ascending order; unreachable j are skipped.
 */
void qco_potential_pairsum(int n, int nrows, const int8_t *dist, double sigma,
                           double *psi, double *v)
{
    const double two_s2 = 2.0 * sigma * sigma;
#pragma omp parallel for schedule(static)
    for (int r = 0; r < nrows; ++r) {
        const int8_t *row = dist + (size_t)r * n;
        double sum1 = 0.0, sum2 = 0.0;
        for (int j = 0; j < n; ++j) {
            if (row[j] < 0) continue;
            double d = (double)row[j];
            double e = exp(-(d * d) / two_s2);
            sum1 = sum1 + (d * d) * e;
            sum2 = sum2 + e;
        }
        psi[r] = sum2;
        v[r] = (1.0 / two_s2) * (sum1 / sum2);
    }
}

/* The canonical FP64 evaluation of the same quantities from the histogram
 * h_k = #{j : d(i,j) = k} (an exact regrouping of Algorithm 1's sums by
 * distance value). Every GGD decision of the oracle uses these values. */
void qco_potential_canonical(int nrows, int K, const int32_t *hist, double sigma,
                             double *psi, double *v)
{
    const double a = (2.0 * sigma) * sigma;
    double *w = (double *)malloc(sizeof(double) * (size_t)K);
    for (int k = 0; k < K; ++k) w[k] = exp(-(double)(k * k) / a);
#pragma omp parallel for schedule(static)
    for (int r = 0; r < nrows; ++r) {
        const int32_t *h = hist + (size_t)r * K;
        double s2 = 0.0, s1 = 0.0;
        for (int k = 0; k < K; ++k) {
            double hk = (double)h[k];
            s2 = s2 + hk * w[k];
            s1 = s1 + ((double)(k * k) * hk) * w[k];
        }
        psi[r] = s2;
        v[r] = (1.0 / a) * (s1 / s2);
    }
    free(w);
}

/* The weights the canonical form uses, exposed so tests can inspect them. */
void qco_weights(int K, double sigma, double *w_out, double *a_out)
{
    const double a = (2.0 * sigma) * sigma;
    for (int k = 0; k < K; ++k) w_out[k] = exp(-(double)(k * k) / a);
    if (a_out) *a_out = a;
}

/* ------------------------------------------------------------------------
 * Algorithm 2 (Graph Gradient Descent), first half: every node picks the
 * neighbour it descends to. tie_mode 0 = STRICT, 1 = MERGE (see header).
 */
void qco_ggd_parent(int n, const int32_t *row_ptr, const int32_t *col,
                    const double *v, int tie_mode, int32_t *parent)
{
    for (int i = 0; i < n; ++i) {
        int best = i;
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            int j = col[e];
            if (v[j] < v[best]) best = j;
            else if (tie_mode == 1 && v[j] == v[best] && j < best) best = j;
        }
        parent[i] = best;
    }
}

/* Algorithm 3 for every node: follow parents to the root (a node that is its
 * own parent) and compress the path, so each node points at its centre. */
void qco_find_centers(int n, const int32_t *parent, int32_t *labels)
{
    for (int i = 0; i < n; ++i) labels[i] = parent[i];
    for (int i = 0; i < n; ++i) {
        int r = i;
        int steps = 0;
        while (labels[r] != r) {
            r = labels[r];
            if (++steps > n) { r = -1; break; } /* a cycle: cannot happen */
        }
        int x = i;
        while (r >= 0 && labels[x] != r) {
            int nx = labels[x];
            labels[x] = r;
            x = nx;
        }
        if (r < 0) labels[i] = -1;
    }
}

/* ------------------------------------------------------------------------
 * Literal distance reading (Section 3.1): an edge gives distance = its weight,
 * a missing edge gives one value cap larger than every weight, and a node's
 * distance to itself is 0. Algorithm 1 over that dense matrix, for weighted
 * graphs given as CSR with a weight per entry. */
void qco_potential_literal(int n, const int32_t *row_ptr, const int32_t *col,
                           const double *weight, double cap, double sigma,
                           double *psi, double *v)
{
    const double two_s2 = 2.0 * sigma * sigma;
#pragma omp parallel
    {
        double *drow = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
        for (int i = 0; i < n; ++i) {
            for (int j = 0; j < n; ++j) drow[j] = cap;
            drow[i] = 0.0;
            for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
                drow[col[e]] = weight ? weight[e] : 1.0;
            double sum1 = 0.0, sum2 = 0.0;
            for (int j = 0; j < n; ++j) {
                double d = drow[j];
                double e = exp(-(d * d) / two_s2);
                sum1 = sum1 + (d * d) * e;
                sum2 = sum2 + e;
            }
            psi[i] = sum2;
            v[i] = (1.0 / two_s2) * (sum1 / sum2);
        }
        free(drow);
    }
}

/* Algorithm 1 on a dense real-valued distance matrix (one row per node, as
 * the paper's GPU experiment runs it on fully connected graphs, Section 3.2).
 * Only finite entries >= 0 are distances; any other entry (negative, NaN,
 * infinite) means "no path" and is skipped. */
void qco_potential_dense(int n, int nrows, const float *dist, double sigma, double *psi, double *v)
{
    const double two_s2 = 2.0 * sigma * sigma;
#pragma omp parallel for schedule(static)
    for (int r = 0; r < nrows; ++r) {
        const float *row = dist + (size_t)r * n;
        double sum1 = 0.0, sum2 = 0.0;
        for (int j = 0; j < n; ++j) {
            if (!(row[j] >= 0.0f) || isinf(row[j])) continue;
            double d = (double)row[j];
            double e = exp(-(d * d) / two_s2);
            sum1 = sum1 + (d * d) * e;
            sum2 = sum2 + e;
        }
        psi[r] = sum2;
        v[r] = (1.0 / two_s2) * (sum1 / sum2);
    }
}

int qco_num_threads(void)
{
    int t = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            t = omp_get_num_threads();
#endif
        }
    }
    return t;
}

/* Threads of the parallel regions that follow (timing at one thread and at
 * every core); k < 1 is taken as 1. */
void qco_set_num_threads(int k)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(k < 1 ? 1 : k);
#else
    (void)k;
#endif
}
