"""Pins for the oracle's hop distances and histograms (CPU only).

The distance of Section 3.1, read as the hop count of a shortest path, has a
textbook definition, so the oracle's BFS is checked against two library
routines (scipy's csgraph shortest paths and networkx's BFS lengths), against
the pure-Python oracle, and against structural invariants.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import oracle
from oracle import tiny
from paper_2305_14641_amd import graphgen as gg


def scipy_dist(g):
    A = sp.csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(g.n, g.n))
    D = csg.shortest_path(A, unweighted=True, directed=False)
    out = np.where(np.isfinite(D), D, -1).astype(np.int64)
    return out


SMALL = [
    gg.path_graph(1), gg.path_graph(2), gg.path_graph(9), gg.star_graph(6),
    gg.complete_graph(5), gg.barbell_graph(4), gg.empty_graph(5),
    gg.disjoint_union(gg.path_graph(4), gg.empty_graph(2), gg.complete_graph(3)),
    gg.twin_leaves(3, 4), gg.random_graph(40, 0.08, 1), gg.random_graph(33, 0.2, 2),
]


@pytest.mark.parametrize("g", SMALL + [gg.config1()], ids=lambda g: g.name)
def test_bfs_matches_scipy(g):
    dist, dmax = oracle.distances(g.n, g.row_ptr, g.col)
    ref = scipy_dist(g)
    np.testing.assert_array_equal(dist.astype(np.int64), ref)
    assert dmax == (ref.max() if g.n else 0)


def test_bfs_config2_matches_scipy():
    g = gg.config2()
    dist, dmax = oracle.distances(g.n, g.row_ptr, g.col)
    np.testing.assert_array_equal(dist.astype(np.int64), scipy_dist(g))


def test_bfs_rows_config3_sample_matches_scipy():
    g = gg.config3()
    rng = np.random.default_rng(5)
    src = rng.choice(g.n, 24, replace=False).astype(np.int32)
    rows, _ = oracle.bfs_rows(g.n, g.row_ptr, g.col, src)
    A = sp.csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(g.n, g.n))
    D = csg.shortest_path(A, unweighted=True, directed=False, indices=src)
    ref = np.where(np.isfinite(D), D, -1).astype(np.int64)
    np.testing.assert_array_equal(rows.astype(np.int64), ref)


@pytest.mark.parametrize("g", SMALL[:8], ids=lambda g: g.name)
def test_bfs_matches_networkx(g):
    import networkx as nx
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    for i in range(g.n):
        for j in g.col[g.row_ptr[i]:g.row_ptr[i + 1]]:
            G.add_edge(i, int(j))
    dist, _ = oracle.distances(g.n, g.row_ptr, g.col)
    for s in range(g.n):
        lengths = nx.single_source_shortest_path_length(G, s)
        for v in range(g.n):
            assert dist[s, v] == lengths.get(v, -1)


@pytest.mark.parametrize("g", SMALL, ids=lambda g: g.name)
def test_bfs_matches_tiny_oracle(g):
    adj = tiny.adjacency(g.n, g.row_ptr, g.col)
    ref = tiny.hop_distances(adj)
    dist, _ = oracle.distances(g.n, g.row_ptr, g.col)
    for s in range(g.n):
        assert [(-1 if x is None else x) for x in ref[s]] == dist[s].tolist()


def test_distance_invariants_config2():
    g = gg.config2()
    dist, dmax = oracle.distances(g.n, g.row_ptr, g.col)
    assert (np.diag(dist) == 0).all()
    np.testing.assert_array_equal(dist, dist.T)
    # every edge (u, v): |d(s,u) - d(s,v)| <= 1 for reachable s, and reachability agrees
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    du = dist[:, rows].astype(np.int32)
    dv = dist[:, g.col].astype(np.int32)
    assert ((du < 0) == (dv < 0)).all()
    fin = du >= 0
    assert (np.abs(du - dv)[fin] <= 1).all()


def test_distance_limit_126_ok_127_overflow():
    ok = gg.path_graph(127)          # diameter 126 fits int8 distances
    dist, dmax = oracle.distances(ok.n, ok.row_ptr, ok.col)
    assert dmax == 126 and dist[0, 126] == 126
    bad = gg.path_graph(128)         # diameter 127 does not
    with pytest.raises(oracle.OracleError):
        oracle.distances(bad.n, bad.row_ptr, bad.col)


def test_histogram_invariants_config2():
    g = gg.config2()
    dist, dmax = oracle.distances(g.n, g.row_ptr, g.col)
    K = dmax + 1
    h = oracle.hist_rows(dist, K)
    deg = g.degrees()
    assert (h[:, 0] == 1).all()                     # the node itself
    np.testing.assert_array_equal(h[:, 1], deg)      # its neighbours
    A = sp.csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(g.n, g.n))
    _, comp = csg.connected_components(A, directed=False)
    sizes = np.bincount(comp)
    np.testing.assert_array_equal(h.sum(axis=1), sizes[comp])  # component size
    # ordered pairs at distance k >= 1 come in symmetric couples
    assert (h[:, 1:].sum(axis=0) % 2 == 0).all()


def test_hist_all_equals_hist_of_matrix():
    g = gg.config2()
    dist, dmax = oracle.distances(g.n, g.row_ptr, g.col)
    h1 = oracle.hist_rows(dist, 32)
    h2, dmax2 = oracle.hist_all(g.n, g.row_ptr, g.col, 32)
    assert dmax2 == dmax
    np.testing.assert_array_equal(h1, h2)


def test_generator_is_canonical_and_seeded():
    for g in [gg.config1(), gg.config2()]:
        rp, col = g.row_ptr, g.col
        for i in range(g.n):
            r = col[rp[i]:rp[i + 1]]
            assert (np.diff(r) > 0).all() and (r != i).all()
        A = sp.csr_matrix((np.ones(g.nnz), col, rp), shape=(g.n, g.n))
        assert (A != A.T).nnz == 0
    a, b = gg.config2(), gg.config2()
    np.testing.assert_array_equal(a.col, b.col)
    c3 = gg.config3()
    assert c3.n == 19717 and c3.nnz == 2 * int(round(19717 * 4.5 / 2))
    assert gg.config2().nnz == 2 * 5416


# --- directed graphs: distances follow edge direction (row i = from i) -------

DIGRAPHS = [gg.random_digraph(30, 0.06, seed=s) for s in range(4)] + [
    gg.dcsbm_directed(400, [0.5, 0.3, 0.2], 2.0, seed=5)]


@pytest.mark.parametrize("g", DIGRAPHS, ids=lambda g: g.name)
def test_directed_bfs_matches_scipy_and_networkx(g):
    import networkx as nx
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path
    d, dmax = oracle.distances(g.n, g.row_ptr, g.col)
    a = csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(g.n, g.n))
    ref = shortest_path(a, directed=True, unweighted=True)
    ref = np.where(np.isinf(ref), -1, ref).astype(np.int8)
    np.testing.assert_array_equal(d, ref)
    assert dmax == ref.max()
    G = nx.DiGraph()
    G.add_nodes_from(range(g.n))
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    G.add_edges_from(zip(rows.tolist(), g.col.tolist()))
    for s in range(0, g.n, max(1, g.n // 7)):
        lengths = nx.single_source_shortest_path_length(G, s)
        want = np.full(g.n, -1, dtype=np.int8)
        for v, l in lengths.items():
            want[v] = l
        np.testing.assert_array_equal(d[s], want)
    if g.n <= 40:
        t = tiny.hop_distances(tiny.adjacency(g.n, g.row_ptr, g.col))
        np.testing.assert_array_equal(d, np.array([[-1 if x is None else x for x in r] for r in t]))


def test_directed_generator_is_canonical_and_seeded():
    g = gg.dcsbm_directed(500, [0.6, 0.4], 2.5, seed=9)
    h = gg.dcsbm_directed(500, [0.6, 0.4], 2.5, seed=9)
    np.testing.assert_array_equal(g.col, h.col)
    assert g.nnz == 1250
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    assert (rows != g.col).all()
    for i in range(g.n):
        r = g.col[g.row_ptr[i]:g.row_ptr[i + 1]]
        assert (np.diff(r) > 0).all()
    # genuinely directed: most arcs have no reverse arc
    fwd = set(zip(rows.tolist(), g.col.tolist()))
    assert sum((b, a) in fwd for a, b in fwd) < 0.2 * len(fwd)


# --- integer edge weights: shortest-path lengths (Dijkstra with buckets) -----

WEIGHTED = [(gg.random_graph(30, 0.12, seed=s), 1 + s % 5) for s in range(4)] + [
    (gg.config2(), 3), (gg.dcsbm_directed(300, [0.5, 0.5], 2.0, seed=8), 4)]


@pytest.mark.parametrize("case", range(len(WEIGHTED)))
def test_weighted_rows_match_scipy_and_networkx(case):
    import networkx as nx
    g, wmax = WEIGHTED[case]
    directed = g.name.startswith("dcsbm_directed")
    w = gg.edge_weights(g, wmax, seed=case, directed=directed)
    d, dmax = oracle.weighted_distances(g.n, g.row_ptr, g.col, w)
    a = sp.csr_matrix((w.astype(np.float64), g.col, g.row_ptr), shape=(g.n, g.n))
    ref = csg.shortest_path(a, directed=directed)
    ref = np.where(np.isinf(ref), -1, ref).astype(np.int8)
    np.testing.assert_array_equal(d, ref)
    assert dmax == ref.max()
    G = nx.DiGraph() if directed else nx.Graph()
    G.add_nodes_from(range(g.n))
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    G.add_weighted_edges_from(zip(rows.tolist(), g.col.tolist(), w.tolist()))
    for s in range(0, g.n, max(1, g.n // 5)):
        want = np.full(g.n, -1, dtype=np.int8)
        for v, l in nx.single_source_dijkstra_path_length(G, s).items():
            want[v] = l
        np.testing.assert_array_equal(d[s], want)


def test_unit_weights_equal_hop_distances():
    g = gg.config1()
    d_hop, _ = oracle.distances(g.n, g.row_ptr, g.col)
    d_w, _ = oracle.weighted_distances(g.n, g.row_ptr, g.col, np.ones(g.nnz, dtype=np.uint8))
    np.testing.assert_array_equal(d_hop, d_w)


def test_weighted_overflow_and_zero_weight():
    g = gg.path_graph(4)
    with pytest.raises(oracle.OracleError):
        oracle.weighted_distances(g.n, g.row_ptr, g.col, np.full(g.nnz, 50, dtype=np.uint8))
    with pytest.raises(oracle.OracleError):
        oracle.weighted_distances(g.n, g.row_ptr, g.col, np.zeros(g.nnz, dtype=np.uint8))


# --- real edge weights: binary32 path sums (Dijkstra with a binary heap) -----

REAL = [gg.random_graph(40, 0.1, seed=s) for s in range(3)] + [
    gg.config2(), gg.dcsbm_directed(300, [0.5, 0.5], 2.0, seed=8),
    gg.disjoint_union(gg.path_graph(5), gg.star_graph(6), gg.empty_graph(3))]


def _is_directed(g):
    return g.name.startswith("dcsbm_directed")


@pytest.mark.parametrize("case", range(len(REAL)))
def test_real_rows_equal_scipy_when_sums_are_exact(case):
    """Weights that are multiples of 1/8: every path sum is exact in float32,
    so the binary32 Dijkstra must equal scipy's float64 shortest paths bit
    for bit (unreachable = +inf in both)."""
    g = REAL[case]
    directed = _is_directed(g)
    w = gg.real_edge_weights(g, seed=case, directed=directed, dyadic=True)
    d = oracle.real_distances(g.n, g.row_ptr, g.col, w)
    a = sp.csr_matrix((w.astype(np.float64), g.col, g.row_ptr), shape=(g.n, g.n))
    ref = csg.shortest_path(a, method="D", directed=directed)
    np.testing.assert_array_equal(d, ref.astype(np.float32))


@pytest.mark.parametrize("case", range(len(REAL)))
def test_real_rows_close_to_float64_shortest_paths(case):
    """Uniform real weights: within binary32 rounding of each path's length
    (relative 2^-24 per edge) of scipy's float64 shortest paths, and the same
    reachability."""
    g = REAL[case]
    directed = _is_directed(g)
    w = gg.real_edge_weights(g, seed=10 + case, directed=directed)
    d = oracle.real_distances(g.n, g.row_ptr, g.col, w)
    a = sp.csr_matrix((w.astype(np.float64), g.col, g.row_ptr), shape=(g.n, g.n))
    ref = csg.shortest_path(a, method="D", directed=directed)
    assert (np.isinf(d) == np.isinf(ref)).all()
    fin = np.isfinite(ref)
    np.testing.assert_allclose(d[fin], ref[fin], rtol=64 * 2.0 ** -24, atol=0)
    assert (np.diag(d) == 0).all()


def _brute_force_f32(n, row_ptr, col, w):
    """Least binary32 left-to-right path sum over all simple paths (tiny n)."""
    out = np.full((n, n), np.inf, dtype=np.float32)
    def walk(s, u, acc, seen):
        if acc < out[s, u]:
            out[s, u] = acc
        for e in range(row_ptr[u], row_ptr[u + 1]):
            v = int(col[e])
            if v not in seen:
                seen.add(v)
                walk(s, v, np.float32(acc + w[e]), seen)
                seen.remove(v)
    for s in range(n):
        walk(s, s, np.float32(0.0), {s})
    return out


def test_real_rows_brute_force_binary32():
    """Every simple path enumerated, its length summed in binary32 from the
    source outward: the oracle's least sums equal these bit for bit, on tiny
    random graphs whose weights mix magnitudes so that rounding decides."""
    rng = np.random.default_rng(5)
    scales = np.array([1.0, 2.0 ** -24, 3 * 2.0 ** -25, 0.1, 1e-3, 7.0], dtype=np.float32)
    for trial in range(40):
        g = gg.random_graph(7, 0.45, seed=100 + trial)
        directed = trial % 3 == 2
        if directed:
            g = gg.random_digraph(7, 0.35, seed=200 + trial)
        rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
        key = np.minimum(rows, g.col) * g.n + np.maximum(rows, g.col) if not directed else \
            np.arange(g.nnz)
        uniq, inv = np.unique(key, return_inverse=True)
        w = (rng.choice(scales, uniq.shape[0]) *
             rng.uniform(1.0, 1.5, uniq.shape[0]).astype(np.float32)).astype(np.float32)[inv]
        d = oracle.real_distances(g.n, g.row_ptr, g.col, w)
        np.testing.assert_array_equal(d, _brute_force_f32(g.n, g.row_ptr, g.col, w),
                                      err_msg=f"trial {trial}")


def test_real_rows_rounding_decides():
    """A path 1 + 2^-24 + 2^-24 sums to 1.0 in binary32 (each partial sum
    rounds to even), below a direct edge of 1 + 2^-23, although its exact
    length equals that edge: the least binary32 sum is 1.0, not the rounded
    exact minimum. Path s=0 - 1 - 2 - 3 and the edge 0 - 3."""
    rp, col = gg.csr_from_edges(4, np.array([0, 1, 2, 0]), np.array([1, 2, 3, 3]))
    g = gg.Graph(4, rp, col, np.zeros(4, dtype=np.int32), "rounding")
    eps = np.float32(2.0 ** -24)
    wt = {(0, 1): np.float32(1.0), (1, 2): eps, (2, 3): eps, (0, 3): np.float32(1.0 + 2.0 ** -23)}
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    w = np.array([wt[(min(a, b), max(a, b))] for a, b in zip(rows, g.col)], dtype=np.float32)
    d = oracle.real_distances(g.n, g.row_ptr, g.col, w)
    # from 3 the same path sums 2^-24 + 2^-24 first, exactly, then 1 + 2^-23
    assert d[0, 3] == np.float32(1.0) and d[3, 0] == np.float32(1.0 + 2.0 ** -23)
    np.testing.assert_array_equal(d, _brute_force_f32(g.n, g.row_ptr, g.col, w))


def test_real_rows_reject_bad_weights():
    g = gg.path_graph(4)
    for bad in (0.0, -1.0, np.nan, np.inf):
        w = np.ones(g.nnz, dtype=np.float32)
        w[1] = bad
        with pytest.raises(oracle.OracleError):
            oracle.real_distances(g.n, g.row_ptr, g.col, w)
