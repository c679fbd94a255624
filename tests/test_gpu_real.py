"""Real edge weights (qc_distances_real, qc_cluster_real) against the oracle.

Distances must equal the oracle's binary32 Dijkstra bit for bit: in full on
small graphs (uniform and dyadic weights, directed, disconnected, one node, a
case where rounding decides, a dense graph) and on the first benchmark-like
graph of each workgroup size (up to 4,096, 8,192, 16,384 and 32,768 nodes,
the last one at the maximum) on sampled rows, once with a padded row stride.
The one-call form must give psi and V within 1e-6 of the oracle's dense
Algorithm 1 on the oracle's distances, and labels equal to the oracle's
descent run on the GPU's own FP64 V (the values it decided on), in both tie
modes; integer-valued weights must give the integer-weight path's distances.
"""
import numpy as np
import pytest

import oracle
from paper_2305_14641_amd import graphgen as gg

pytestmark = pytest.mark.gpu

TOL = 1e-6


def _qc():
    import torch
    from paper_2305_14641_amd import qc
    assert torch.cuda.is_available()
    return torch, qc


def _rounding_case():
    rp, col = gg.csr_from_edges(4, np.array([0, 1, 2, 0]), np.array([1, 2, 3, 3]))
    g = gg.Graph(4, rp, col, np.zeros(4, dtype=np.int32), "rounding")
    wt = {(0, 1): 1.0, (1, 2): 2.0 ** -24, (2, 3): 2.0 ** -24, (0, 3): 1.0 + 2.0 ** -23}
    rows = np.repeat(np.arange(4), np.diff(rp))
    w = np.array([wt[(min(a, b), max(a, b))] for a, b in zip(rows, col)], dtype=np.float32)
    return g, w


def _cases():
    out = []
    for s in range(2):
        g = gg.random_graph(60, 0.08, seed=s)
        out.append((f"random{s}-uniform", g, gg.real_edge_weights(g, seed=s), False))
    g = gg.random_graph(80, 0.06, seed=7)
    out.append(("random-dyadic", g, gg.real_edge_weights(g, seed=7, dyadic=True), False))
    g = gg.dcsbm_directed(300, [0.5, 0.5], 2.0, seed=8)
    out.append(("directed", g, gg.real_edge_weights(g, seed=8, directed=True), True))
    g = gg.disjoint_union(gg.path_graph(5), gg.star_graph(6), gg.empty_graph(3))
    out.append(("disconnected", g, gg.real_edge_weights(g, seed=9), False))
    g = gg.path_graph(1)
    out.append(("one-node", g, np.zeros(0, dtype=np.float32), False))
    g, w = _rounding_case()
    out.append(("rounding", g, w, False))
    g = gg.complete_graph(50)
    out.append(("complete", g, gg.real_edge_weights(g, seed=11, lo=0.01, hi=100.0), False))
    g = gg.config2()
    out.append(("config2", g, gg.real_edge_weights(g, seed=12), False))
    return out


CASES = _cases()


@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
def test_real_distances_bit_exact(case):
    torch, qc = _qc()
    name, g, w, directed = CASES[case]
    print(f"[gpu] real distances {name} n={g.n}", flush=True)
    d = qc.distances_real(g.n, g.row_ptr, g.col, w, directed=directed)
    torch.cuda.synchronize()
    want = oracle.real_distances(g.n, g.row_ptr, g.col, w)
    np.testing.assert_array_equal(d.cpu().numpy(), want)


@pytest.mark.parametrize("n", [3000, 6000, 12000, 20000, 32768])
def test_real_distances_each_shape_sampled(n):
    """One graph per workgroup size, sampled rows (first, last, spread);
    the 12,000-node case writes into a padded row stride."""
    torch, qc = _qc()
    g = gg.dcsbm(n, [0.25, 0.25, 0.25, 0.25], 4.0, seed=n)
    w = gg.real_edge_weights(g, seed=n)
    print(f"[gpu] real distances dcsbm n={n} nnz={g.nnz}", flush=True)
    ld = n + 13 if n == 12000 else n
    buf = torch.full((n, ld), -5.0, dtype=torch.float32, device="cuda")
    qc.distances_real(g.n, g.row_ptr, g.col, w, out=buf[:, :n] if ld != n else buf)
    torch.cuda.synchronize()
    rows = np.unique(np.concatenate([[0, n - 1], np.linspace(0, n - 1, 30).astype(np.int64)]))
    want = oracle.real_rows(g.n, g.row_ptr, g.col, w, rows.astype(np.int32))
    got = buf[torch.as_tensor(rows, device="cuda")].cpu().numpy()
    np.testing.assert_array_equal(got[:, :n], want)
    if ld != n:   # the padding past each row is untouched
        assert (got[:, n:] == -5.0).all()


def _check_cluster(g, w, directed, sigmas, tie, with_dist):
    torch, qc = _qc()
    S = len(sigmas)
    dist = torch.empty((g.n, g.n), dtype=torch.float32, device="cuda") if with_dist else None
    psi = torch.empty((S, g.n), dtype=torch.float64, device="cuda")
    v = torch.empty((S, g.n), dtype=torch.float64, device="cuda")
    lab = qc.cluster_real(g.n, g.row_ptr, g.col, w, sigmas, tie_mode=tie, directed=directed,
                          dist=dist, psi=psi, v=v)
    torch.cuda.synchronize()
    want_d = oracle.real_distances(g.n, g.row_ptr, g.col, w)
    if with_dist:
        np.testing.assert_array_equal(dist.cpu().numpy(), want_d)
    psi, v, lab = psi.cpu().numpy(), v.cpu().numpy(), lab.cpu().numpy()
    for s, sigma in enumerate(sigmas):
        psi_o, v_o = oracle.potential_dense(want_d, sigma)
        np.testing.assert_allclose(psi[s], psi_o, rtol=TOL, atol=0)
        np.testing.assert_allclose(v[s], v_o, rtol=TOL, atol=1e-300)
        # the descent decided on these FP64 values: the oracle's descent on
        # them must give the same labels exactly
        ref = oracle.find_centers(oracle.ggd_parent(g.n, g.row_ptr, g.col, v[s], tie))
        np.testing.assert_array_equal(lab[s], ref, err_msg=f"sigma={sigma}")


@pytest.mark.parametrize("tie", [0, 1])
def test_cluster_real_matches_oracle(tie):
    g = gg.dcsbm(1500, [0.3, 0.3, 0.4], 5.0, seed=21)
    w = gg.real_edge_weights(g, seed=21)
    print(f"[gpu] cluster_real n={g.n} tie={tie}", flush=True)
    _check_cluster(g, w, False, [0.5, 1.0, 2.0, 4.0, 7.5], tie, with_dist=(tie == 0))


def test_cluster_real_directed_and_small_cases():
    g = gg.dcsbm_directed(400, [0.5, 0.5], 3.0, seed=31)
    _check_cluster(g, gg.real_edge_weights(g, seed=31, directed=True), True, [1.0, 3.0], 0, True)
    g, w = _rounding_case()
    _check_cluster(g, w, False, [0.7], 0, True)
    g = gg.disjoint_union(gg.star_graph(8), gg.path_graph(4), gg.empty_graph(2))
    _check_cluster(g, gg.real_edge_weights(g, seed=3, dyadic=True), False, [0.5, 2.0], 1, False)


def test_integer_valued_weights_match_the_integer_path():
    """Weights that are small integers: the real path's lengths equal the
    integer-weight (subdivided) path's hop counts."""
    torch, qc = _qc()
    g = gg.dcsbm(900, [0.5, 0.5], 4.0, seed=41)
    wi = gg.edge_weights(g, 4, seed=41)
    G = qc.Graph.from_graph(g, weights=wi)
    d_int = torch.empty((g.n, g.n), dtype=torch.int8, device="cuda")
    G.distances(d_int)
    d_real = qc.distances_real(g.n, g.row_ptr, g.col, wi.astype(np.float32))
    torch.cuda.synchronize()
    di = d_int.cpu().numpy().astype(np.float32)
    di[di < 0] = np.inf
    np.testing.assert_array_equal(d_real.cpu().numpy(), di)
    G.close()
