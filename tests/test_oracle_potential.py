"""Pins for the oracle's wave function psi and potential V (CPU only).

psi and V (Eq. 2, Eq. 7, Algorithm 1) depend on a node only through the
histogram of its hop distances, so on graph families whose histograms are
known by construction they have closed forms. These are evaluated here at 50
significant digits with mpmath and compared with both oracle forms (the
literal pair sum and the canonical histogram form). A dropped self term, a
wrong power of d, a wrong sign or a swapped numerator and denominator each
move the result far outside the tolerance.
"""
import math

import mpmath
import numpy as np
import pytest

import oracle
from oracle import tiny
from paper_2305_14641_amd import graphgen as gg

mpmath.mp.dps = 50


def closed_form(hist, sigma):
    """Eq. 2 and Eq. 7 (approximate form) for one node with distance
    histogram ``hist`` (hist[k] nodes at distance k, self included)."""
    a = 2 * mpmath.mpf(sigma) ** 2
    psi = mpmath.fsum(h * mpmath.e ** (-(k * k) / a) for k, h in enumerate(hist))
    s1 = mpmath.fsum(h * k * k * mpmath.e ** (-(k * k) / a) for k, h in enumerate(hist))
    return psi, s1 / (a * psi)


def family_histograms():
    """(graph, {node: histogram}) with histograms read off the construction."""
    out = []
    for n in (2, 4, 7):
        out.append((gg.complete_graph(n), {i: [1, n - 1] for i in range(n)}))
    for leaves in (1, 4, 9):
        g = gg.star_graph(leaves)
        hs = {0: [1, leaves]}
        for i in range(1, leaves + 1):
            hs[i] = [1, 1, leaves - 1] if leaves > 1 else [1, 1]
        out.append((g, hs))
    for n in (5, 8):
        g = gg.path_graph(n)
        hs = {}
        for i in range(n):
            h = [0] * n
            for k in range(n):
                h[k] = int(k <= i) + int(k <= n - 1 - i)
            h[0] = 1
            while h and h[-1] == 0:
                h.pop()
            hs[i] = h
        out.append((g, hs))
    for m in (3, 4):
        g = gg.barbell_graph(m)
        hs = {}
        for i in range(2 * m):
            bridge = i in (m - 1, m)
            hs[i] = [1, m, m - 1] if bridge else [1, m - 1, 1, m - 1]
        out.append((g, hs))
    g = gg.disjoint_union(gg.empty_graph(1), gg.path_graph(2))
    out.append((g, {0: [1], 1: [1, 1], 2: [1, 1]}))
    return out


FAMILIES = family_histograms()


@pytest.mark.parametrize("sigma", [0.25, 0.5, 1.0, 2.0, 3.0, 8.0])
@pytest.mark.parametrize("case", FAMILIES, ids=lambda c: c[0].name)
def test_closed_forms(case, sigma):
    g, hs = case
    dist, dmax = oracle.distances(g.n, g.row_ptr, g.col)
    hist = oracle.hist_rows(dist, dmax + 1)
    psi_p, v_p = oracle.potential_pairsum(dist, sigma)
    psi_c, v_c = oracle.potential_canonical(hist, sigma)
    # a-priori bound for a recursive fp64 sum of m positive terms whose
    # weights carry at most one ulp of exp error: (m + 2) u, u = 2^-53
    u = 2.0 ** -53
    tol_psi = (g.n + 4) * 2 * u
    tol_v = 2 * tol_psi + 4 * u
    for i, h in hs.items():
        psi_x, v_x = closed_form(h, sigma)
        for psi, v in ((psi_p[i], v_p[i]), (psi_c[i], v_c[i])):
            assert abs(psi - float(psi_x)) <= tol_psi * float(psi_x)
            if v_x == 0:
                assert v == 0.0
            else:
                assert abs(v - float(v_x)) <= tol_v * float(v_x), (i, v, float(v_x))


def test_worked_values_sigma1():
    """A few values of the closed forms, written out to 15 digits."""
    psi, v = closed_form([1, 3], 1.0)            # K4
    assert abs(float(psi) - 2.81959197913790) < 1e-13
    assert abs(float(v) - 0.322669377803778) < 1e-14
    psi, v = closed_form([1, 4], 1.0)            # centre of a 4-leaf star
    assert abs(float(v) - 0.354062433629711) < 1e-14
    psi, v = closed_form([1, 1, 3], 1.0)         # its leaves
    assert abs(float(v) - 0.554164868092773) < 1e-14
    g = gg.star_graph(4)
    dist, dmax = oracle.distances(g.n, g.row_ptr, g.col)
    _, vc = oracle.potential_canonical(oracle.hist_rows(dist, dmax + 1), 1.0)
    assert abs(vc[0] - 0.354062433629711) < 1e-14
    assert abs(vc[3] - 0.554164868092773) < 1e-14


def test_isolated_node_exact():
    g = gg.empty_graph(3)
    dist, _ = oracle.distances(g.n, g.row_ptr, g.col)
    psi, v = oracle.potential_canonical(oracle.hist_rows(dist, 1), 0.7)
    assert (psi == 1.0).all() and (v == 0.0).all()
    psi, v = oracle.potential_pairsum(dist, 0.7)
    assert (psi == 1.0).all() and (v == 0.0).all()


@pytest.mark.parametrize("seed", [3, 4])
def test_pairsum_vs_mpmath_random_graph(seed):
    """The fp64 pair sum is within a few ulp of a 50-digit evaluation of
    Algorithm 1 over scipy's distances (not the oracle's)."""
    import scipy.sparse as sp
    import scipy.sparse.csgraph as csg
    g = gg.random_graph(30, 0.12, seed)
    A = sp.csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(g.n, g.n))
    D = csg.shortest_path(A, unweighted=True, directed=False)
    dist, dmax = oracle.distances(g.n, g.row_ptr, g.col)
    for sigma in (0.5, 1.3):
        psi_p, v_p = oracle.potential_pairsum(dist, sigma)
        psi_c, v_c = oracle.potential_canonical(oracle.hist_rows(dist, dmax + 1), sigma)
        a = 2 * mpmath.mpf(sigma) ** 2
        for i in range(g.n):
            ds = [int(x) for x in D[i] if np.isfinite(x)]
            psi_x = mpmath.fsum(mpmath.e ** (-(d * d) / a) for d in ds)
            v_x = mpmath.fsum(d * d * mpmath.e ** (-(d * d) / a) for d in ds) / (a * psi_x)
            tol = (len(ds) + 4) * 2.0 ** -52
            for psi, v in ((psi_p[i], v_p[i]), (psi_c[i], v_c[i])):
                assert abs(psi - float(psi_x)) <= tol * float(psi_x)
                if v_x != 0:
                    assert abs(v - float(v_x)) <= 2 * tol * float(v_x)


@pytest.mark.parametrize("cfg", ["c1", "c2"])
def test_pairsum_and_canonical_agree(cfg):
    g = gg.config1() if cfg == "c1" else gg.config2()
    sigmas = gg.SIGMAS_C1 if cfg == "c1" else gg.SIGMAS_C2
    dist, dmax = oracle.distances(g.n, g.row_ptr, g.col)
    hist = oracle.hist_rows(dist, dmax + 1)
    for s in sigmas + [0.25, 8.0]:
        psi_p, v_p = oracle.potential_pairsum(dist, s)
        psi_c, v_c = oracle.potential_canonical(hist, s)
        np.testing.assert_allclose(psi_c, psi_p, rtol=1e-12, atol=0)
        np.testing.assert_allclose(v_c, v_p, rtol=1e-12, atol=0)


def test_large_sigma_limit_mean_square_distance():
    """As sigma grows, V * 2 sigma^2 tends to the mean of d^2 over the node's
    component (every weight tends to 1)."""
    g = gg.config1()
    dist, dmax = oracle.distances(g.n, g.row_ptr, g.col)
    hist = oracle.hist_rows(dist, dmax + 1)
    sigma = 1e4
    _, v = oracle.potential_canonical(hist, sigma)
    d = dist.astype(np.float64)
    fin = dist >= 0
    mean_sq = np.where(fin, d * d, 0).sum(axis=1) / fin.sum(axis=1)
    np.testing.assert_allclose(v * 2 * sigma * sigma, mean_sq, rtol=1e-6)


def test_weights_match_high_precision_exp():
    """The canonical weights w_k = exp(-k^2 / a), a = 2 sigma^2 (Eq. 2's
    Gaussian at hop distance k), are the exponential of the rounded FP64
    quotient to within one rounding of a 50-digit evaluation; for a dyadic
    sigma, a itself is exact."""
    for sigma in (0.3, 1.5, 6.0):
        w, a = oracle.weights(12, sigma)
        if sigma != 0.3:
            assert a == float(2 * mpmath.mpf(sigma) ** 2)
        for k in range(12):
            q = -(k * k) / a                      # one IEEE division, as in the definition
            x = mpmath.e ** mpmath.mpf(q)
            assert abs(w[k] - float(x)) <= 2.3e-16 * float(x), (sigma, k)


@pytest.mark.parametrize("g", [gg.random_graph(25, 0.15, 7), gg.barbell_graph(5), gg.config1()],
                         ids=lambda g: g.name)
def test_matches_tiny_oracle(g):
    adj = tiny.adjacency(g.n, g.row_ptr, g.col)
    ref_dist = tiny.hop_distances(adj)
    dist, dmax = oracle.distances(g.n, g.row_ptr, g.col)
    for sigma in (0.5, 1.0, 2.5):
        psi_t, v_t = tiny.potential(ref_dist, sigma)
        psi_o, v_o = oracle.potential_pairsum(dist, sigma)
        np.testing.assert_allclose(psi_o, psi_t, rtol=1e-13)
        np.testing.assert_allclose(v_o, v_t, rtol=1e-13)


def test_literal_reading_cap2_equals_hop_distance_capped():
    """With unit edge weights and every non-edge at distance 2, Algorithm 1
    on the literal distance equals the histogram form with h = [1, deg, rest]."""
    g = gg.config1()
    psi, v = oracle.potential_literal(g.n, g.row_ptr, g.col, 1.3, cap=2.0)
    deg = g.degrees()
    for i in (0, 7, 99):
        h = [1, int(deg[i]), g.n - 1 - int(deg[i])]
        psi_x, v_x = closed_form(h, 1.3)
        assert abs(psi[i] - float(psi_x)) <= 1e-13 * float(psi_x)
        assert abs(v[i] - float(v_x)) <= 1e-13 * float(v_x)


def test_dense_form_vs_mpmath_and_literal():
    """Algorithm 1 on a dense float matrix: a 50-digit evaluation of the same
    float entries, and equality with the literal-reading function when the
    matrix is the literal distance of a graph."""
    d = gg.dense_points(40, dim=3, clusters=3, seed=4)
    d[3, 7] = d[7, 3] = -1.0                     # missing pairs are skipped
    d[3, 9] = np.nan
    d[3, 11] = np.inf
    for sigma in (0.7, 2.5):
        psi, v = oracle.potential_dense(d, sigma)
        a = 2 * mpmath.mpf(sigma) ** 2
        for i in (0, 3, 39):
            ds = [mpmath.mpf(float(x)) for x in d[i] if np.isfinite(x) and x >= 0]
            psi_x = mpmath.fsum(mpmath.e ** (-(x * x) / a) for x in ds)
            v_x = mpmath.fsum(x * x * mpmath.e ** (-(x * x) / a) for x in ds) / (a * psi_x)
            assert abs(psi[i] - float(psi_x)) <= 1e-14 * float(psi_x)
            assert abs(v[i] - float(v_x)) <= 1e-14 * float(v_x)
    g = gg.config1()
    lit = np.full((g.n, g.n), 2.0, dtype=np.float32)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    lit[rows, g.col] = 1.0
    np.fill_diagonal(lit, 0.0)
    psi_d, v_d = oracle.potential_dense(lit, 1.3)
    psi_l, v_l = oracle.potential_literal(g.n, g.row_ptr, g.col, 1.3, cap=2.0)
    np.testing.assert_allclose(psi_d, psi_l, rtol=1e-14)
    np.testing.assert_allclose(v_d, v_l, rtol=1e-14)


def test_literal_reading_weighted_star_closed_form():
    """Section 3.1 read literally with real edge weights: on a star whose
    edges all differ, the centre sees every leaf at its own edge's weight and
    a leaf sees the centre at its edge's weight and every other leaf at the
    cap. Both follow from the construction alone (50 digits, mpmath), so an
    entry's weight taken from the wrong index (the neighbour's id instead of
    the entry, or the row's first entry) moves the result far off."""
    leaves = 6
    g = gg.star_graph(leaves)
    # weights per CSR entry; the two entries of an edge carry the same value
    w_edge = {leaf: 0.25 + 0.375 * leaf for leaf in range(1, leaves + 1)}
    weight = np.empty(g.nnz, dtype=np.float64)
    for i in range(g.n):
        for e in range(g.row_ptr[i], g.row_ptr[i + 1]):
            j = int(g.col[e])
            weight[e] = w_edge[max(i, j)]
    cap = 3.5
    for sigma in (0.6, 1.0, 2.2):
        psi, v = oracle.potential_literal(g.n, g.row_ptr, g.col, sigma, weight=weight, cap=cap)
        a = 2 * mpmath.mpf(sigma) ** 2

        def pv(ds):
            ds = [mpmath.mpf(x) for x in ds]
            p = mpmath.fsum(mpmath.e ** (-(x * x) / a) for x in ds)
            return p, mpmath.fsum(x * x * mpmath.e ** (-(x * x) / a) for x in ds) / (a * p)

        for i in range(g.n):
            if i == 0:
                ds = [0.0] + [w_edge[l] for l in range(1, leaves + 1)]
            else:
                ds = [0.0, w_edge[i]] + [cap] * (leaves - 1)
            psi_x, v_x = pv(ds)
            assert abs(psi[i] - float(psi_x)) <= 1e-14 * float(psi_x), (sigma, i)
            assert abs(v[i] - float(v_x)) <= 1e-14 * float(v_x), (sigma, i)


def test_literal_reading_weighted_equals_dense_on_written_matrix():
    """The weighted literal reading equals the dense form (itself pinned to a
    50-digit evaluation above) on the literal matrix written out on the host:
    the entry's weight for an edge, the cap for a missing edge, 0 on the
    diagonal. Random symmetric weights, exactly representable in float32."""
    g = gg.random_graph(60, 0.12, 11)
    rng = np.random.default_rng(5)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    w_sym = np.zeros((g.n, g.n))
    up = rows < g.col
    w_sym[rows[up], g.col[up]] = rng.integers(1, 40, up.sum()) / 8.0
    w_sym = w_sym + w_sym.T
    weight = w_sym[rows, g.col].astype(np.float64)
    cap = 6.0
    lit = np.full((g.n, g.n), cap, dtype=np.float32)
    lit[rows, g.col] = weight.astype(np.float32)
    np.fill_diagonal(lit, 0.0)
    for sigma in (0.8, 1.7, 4.0):
        psi_l, v_l = oracle.potential_literal(g.n, g.row_ptr, g.col, sigma, weight=weight, cap=cap)
        psi_d, v_d = oracle.potential_dense(lit, sigma)
        np.testing.assert_allclose(psi_l, psi_d, rtol=1e-14, atol=0)
        np.testing.assert_allclose(v_l, v_d, rtol=1e-14, atol=0)
