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
