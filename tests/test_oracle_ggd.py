"""Pins for the oracle's Graph Gradient Descent (Algorithms 2-4, CPU only).

Three independent checks:
  * hand-derived labels on named graphs (tests/golden/ggd_named_graphs.txt);
  * a characterisation checked on every graph of at most 7 nodes
    (networkx's graph atlas, 1,253 graphs): each parent is the rule's choice
    computed with Python's own ``min``, roots are exactly the nodes without a
    strictly lower neighbour (STRICT), and labels are the ends of the descent;
  * structural invariants on the seeded workloads (V strictly decreases along
    parent links, labels are fixed points).
"""
import os

import numpy as np
import pytest

import oracle
from oracle import tiny
from paper_2305_14641_amd import graphgen as gg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "ggd_named_graphs.txt")

NAMED = {
    "path5": lambda: gg.path_graph(5),
    "star4": lambda: gg.star_graph(4),
    "K4": lambda: gg.complete_graph(4),
    "barbell4": lambda: gg.barbell_graph(4),
}


def golden_cases():
    out = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            out.append((parts[0], float(parts[1]), parts[2], [int(x) for x in parts[3:]]))
    return out


def oracle_labels(g, sigma, mode):
    dist, dmax = oracle.distances(g.n, g.row_ptr, g.col)
    hist = oracle.hist_rows(dist, dmax + 1)
    _, v = oracle.potential_canonical(hist, sigma)
    tie = oracle.TIE_MERGE if mode == "merge" else oracle.TIE_STRICT
    parent = oracle.ggd_parent(g.n, g.row_ptr, g.col, v, tie)
    return v, parent, oracle.find_centers(parent)


@pytest.mark.parametrize("case", golden_cases(), ids=lambda c: f"{c[0]}-{c[1]}-{c[2]}")
def test_named_graph_labels(case):
    name, sigma, mode, expected = case
    g = NAMED[name]()
    _, _, labels = oracle_labels(g, sigma, mode)
    assert labels.tolist() == expected


def check_characterisation(adj, v, parent, labels, merge):
    n = len(adj)
    for i in range(n):
        if merge:
            want = min([i] + adj[i], key=lambda j: (v[j], j))
        else:
            lower = [j for j in adj[i] if v[j] < v[i]]
            want = min(lower, key=lambda j: (v[j], j)) if lower else i
        assert parent[i] == want
    for i in range(n):
        r = labels[i]
        assert parent[r] == r                     # a label is a root
        if not merge:
            assert all(v[j] >= v[r] for j in adj[r])  # no strictly lower neighbour
        assert labels[parent[i]] == r             # descent keeps the label
        if parent[i] != i:
            if merge:
                assert (v[parent[i]], parent[i]) < (v[i], i)
            else:
                assert v[parent[i]] < v[i]


def test_atlas_all_graphs_up_to_7_nodes():
    import networkx as nx
    atlas = nx.graph_atlas_g()
    assert len(atlas) == 1253
    count = 0
    for G in atlas:
        n = G.number_of_nodes()
        if n == 0:
            continue
        edges = np.array(list(G.edges()), dtype=np.int64).reshape(-1, 2)
        rp, col = gg.csr_from_edges(n, edges[:, 0], edges[:, 1])
        g = gg.Graph(n, rp, col, np.zeros(n, np.int32))
        adj = tiny.adjacency(n, rp, col)
        dist, dmax = oracle.distances(n, rp, col)
        hist = oracle.hist_rows(dist, dmax + 1)
        for sigma in (0.5, 1.0, 2.0):
            _, v = oracle.potential_canonical(hist, sigma)
            for merge in (False, True):
                parent = oracle.ggd_parent(n, rp, col, v, oracle.TIE_MERGE if merge else oracle.TIE_STRICT)
                labels = oracle.find_centers(parent)
                check_characterisation(adj, v.tolist(), parent.tolist(), labels.tolist(), merge)
                # same answer from the pure-Python descent
                tp, tl = tiny.descend(adj, v.tolist(), merge)
                assert tp == parent.tolist() and tl == labels.tolist()
                count += 1
    assert count == 1252 * 6


@pytest.mark.parametrize("cfg", ["c1", "c2"])
def test_invariants_on_workloads(cfg):
    g = gg.config1() if cfg == "c1" else gg.config2()
    sigmas = gg.SIGMAS_C1 if cfg == "c1" else gg.SIGMAS_C2
    adj = tiny.adjacency(g.n, g.row_ptr, g.col)
    dist, dmax = oracle.distances(g.n, g.row_ptr, g.col)
    hist = oracle.hist_rows(dist, dmax + 1)
    for s in sigmas:
        _, v = oracle.potential_canonical(hist, s)
        for merge in (False, True):
            parent = oracle.ggd_parent(g.n, g.row_ptr, g.col, v,
                                       oracle.TIE_MERGE if merge else oracle.TIE_STRICT)
            labels = oracle.find_centers(parent)
            check_characterisation(adj, v.tolist(), parent.tolist(), labels.tolist(), merge)
            # isolated nodes are their own cluster
            iso = np.flatnonzero(g.degrees() == 0)
            assert (labels[iso] == iso).all()


def test_twin_leaves_tie_to_smallest_id():
    """Leaves hanging off one hub have identical histograms, hence exactly
    equal V: a hub that descends picks the smallest-id leaf."""
    g = gg.star_graph(6)
    v, parent, labels = oracle_labels(g, 0.5, "strict")
    assert len(set(v[1:].tolist())) == 1
    assert parent[0] == 1


def test_cluster_end_to_end_small():
    g = gg.config1()
    res = oracle.cluster(g.n, g.row_ptr, g.col, [1.0])
    r = res["per_sigma"][0]
    assert res["dist"].shape == (200, 200)
    assert r["labels"].shape == (200,)
    roots = np.unique(r["labels"])
    assert 1 <= roots.size < 200


@pytest.mark.parametrize("seed", range(40))
def test_directed_descent_matches_tiny(seed):
    """On directed graphs a node descends only to an out-neighbour; the C
    oracle's parents and labels equal the pure-Python ones."""
    g = gg.random_digraph(12 + seed % 9, 0.15 + 0.01 * (seed % 5), seed=100 + seed)
    adj = tiny.adjacency(g.n, g.row_ptr, g.col)
    dist = tiny.hop_distances(adj)
    for sigma in (0.5, 1.0, 2.5):
        _, v = tiny.potential(dist, sigma)
        for mode, merge in ((oracle.TIE_STRICT, False), (oracle.TIE_MERGE, True)):
            par = oracle.ggd_parent(g.n, g.row_ptr, g.col, np.array(v), mode)
            tpar, tlab = tiny.descend(adj, v, merge=merge)
            np.testing.assert_array_equal(par, tpar)
            np.testing.assert_array_equal(oracle.find_centers(par), tlab)
