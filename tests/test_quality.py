"""The Section 4.2 measures against independent implementations
(scikit-learn's ARI, NMI (geometric normalisation), FMI; networkx's
modularity) and textbook special cases."""
import numpy as np
import pytest

from paper_2305_14641_amd import graphgen as gg
from paper_2305_14641_amd import quality


@pytest.mark.parametrize("seed", range(6))
def test_against_sklearn(seed):
    from sklearn import metrics
    rng = np.random.default_rng(seed)
    a = rng.integers(0, 5, 300)
    b = np.where(rng.random(300) < 0.6, a, rng.integers(0, 7, 300))
    assert abs(quality.ari(a, b) - metrics.adjusted_rand_score(a, b)) < 1e-12
    assert abs(quality.fmi(a, b) - metrics.fowlkes_mallows_score(a, b)) < 1e-12
    ref = metrics.normalized_mutual_info_score(a, b, average_method="geometric")
    assert abs(quality.nmi(a, b) - ref) < 1e-12


def test_special_cases():
    a = np.array([0, 0, 1, 1, 2, 2])
    assert quality.ari(a, a) == 1.0 and quality.fmi(a, a) == 1.0 and quality.nmi(a, a) == 1.0
    relabel = np.array([5, 5, 3, 3, 9, 9])
    assert quality.ari(a, relabel) == 1.0           # labels are names only
    one = np.zeros(6, dtype=int)
    assert quality.nmi(a, one) == 0.0


@pytest.mark.parametrize("g", [gg.config1(), gg.barbell_graph(5), gg.config2()], ids=lambda g: g.name)
def test_modularity_against_networkx(g):
    import networkx as nx
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    G.add_edges_from(zip(rows.tolist(), g.col.tolist()))
    labels = g.blocks if len(set(g.blocks.tolist())) > 1 else (np.arange(g.n) % 3)
    comms = [set(np.flatnonzero(labels == c).tolist()) for c in np.unique(labels)]
    ref = nx.algorithms.community.modularity(G, comms)
    assert abs(quality.modularity(g.row_ptr, g.col, labels) - ref) < 1e-12
