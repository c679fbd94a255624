"""Integer edge weights (qc_graph_create_weighted): distances are weighted
shortest-path lengths, against the oracle's Dijkstra; then histograms, psi/V
and labels through the same path as hop distances.

Cases: small random graphs, the 2,708-node citation-shaped graph, a
directed graph, a weighted path (closed form), unit weights (equal to the
unweighted handle), a larger graph on sampled rows, a batch mixing weighted
and unweighted handles, and the distance limit.
"""
import numpy as np
import pytest

import oracle
from paper_2305_14641_amd import graphgen as gg

pytestmark = pytest.mark.gpu

RTOL = 1e-6


def rel_err(got, want):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    zero = want == 0
    assert (got[zero] == 0).all()
    return float((np.abs(got - want)[~zero] / np.abs(want[~zero])).max()) if (~zero).any() else 0.0


def check(g, w, sigmas, directed=False, rows=None):
    import torch
    from paper_2305_14641_amd import qc
    G = qc.Graph(g.n, g.row_ptr, g.col, directed=directed, weights=w)
    dist = torch.empty((g.n, g.n), dtype=torch.int8, device="cuda")
    dmax = G.distances(dist)
    psi, v = G.potential(sigmas)
    labels = {(s, t): G.labels(s, t).cpu().numpy() for s in range(len(sigmas)) for t in (0, 1)}
    G.sync()
    hist = G.histograms().cpu().numpy()
    if rows is None:
        ref, ref_dmax = oracle.weighted_distances(g.n, g.row_ptr, g.col, w)
        np.testing.assert_array_equal(dist.cpu().numpy(), ref)
        ref_hist = oracle.hist_rows(ref, hist.shape[1])
    else:
        rows = np.asarray(rows, dtype=np.int32)
        ref_rows, _ = oracle.weighted_rows(g.n, g.row_ptr, g.col, w, rows)
        got = dist[torch.as_tensor(rows.astype(np.int64), device="cuda")].cpu().numpy()
        np.testing.assert_array_equal(got, ref_rows)
        ref_full, ref_dmax = oracle.weighted_distances(g.n, g.row_ptr, g.col, w)
        ref_hist = oracle.hist_rows(ref_full, hist.shape[1])
        del ref_full
    assert dmax == ref_dmax
    np.testing.assert_array_equal(hist, ref_hist)
    psi, v = psi.cpu().numpy(), v.cpu().numpy()
    for s, sigma in enumerate(sigmas):
        psi_c, v_c = oracle.potential_canonical(ref_hist, sigma)
        assert rel_err(psi[s], psi_c) <= RTOL
        assert rel_err(v[s], v_c) <= RTOL
        for t in (0, 1):
            lab = oracle.find_centers(oracle.ggd_parent(g.n, g.row_ptr, g.col, v_c, t))
            np.testing.assert_array_equal(labels[(s, t)], lab, err_msg=f"{g.name} sigma={sigma} tie={t}")
    G.close()


@pytest.mark.parametrize("seed", range(5))
def test_small_random_weighted(seed):
    g = gg.random_graph(40 + 10 * seed, 0.08, seed=seed)
    check(g, gg.edge_weights(g, 1 + seed, seed=seed), [0.7, 2.0, 5.0])


def test_citation_shaped_weighted():
    g = gg.config2()
    check(g, gg.edge_weights(g, 3, seed=11), gg.SIGMAS_C2)


def test_directed_weighted():
    g = gg.dcsbm_directed(1500, [0.5, 0.3, 0.2], 2.0, seed=12)
    check(g, gg.edge_weights(g, 4, seed=12, directed=True), [1.0, 3.0], directed=True)


def test_weighted_path_closed_form():
    import torch
    from paper_2305_14641_amd import qc
    n = 30
    g = gg.path_graph(n)
    rng = np.random.default_rng(3)
    wl = rng.integers(1, 5, n - 1)                    # weight of edge (i, i+1)
    rows = np.repeat(np.arange(n), np.diff(g.row_ptr))
    w = wl[np.minimum(rows, g.col)].astype(np.uint8)
    pos = np.concatenate([[0], np.cumsum(wl)])        # distance from node 0 along the path
    want = np.abs(pos[:, None] - pos[None, :]).astype(np.int8)
    G = qc.Graph(n, g.row_ptr, g.col, weights=w)
    dist = torch.empty((n, n), dtype=torch.int8, device="cuda")
    assert G.distances(dist) == int(pos[-1])
    np.testing.assert_array_equal(dist.cpu().numpy(), want)
    G.close()


def test_unit_weights_equal_unweighted():
    import torch
    from paper_2305_14641_amd import qc
    g = gg.config2()
    a = qc.Graph.from_graph(g)
    b = qc.Graph(g.n, g.row_ptr, g.col, weights=np.ones(g.nnz, dtype=np.uint8))
    da = torch.empty((g.n, g.n), dtype=torch.int8, device="cuda")
    db = torch.empty_like(da)
    assert a.distances(da) == b.distances(db)
    assert torch.equal(da, db)
    a.close()
    b.close()


def test_larger_weighted_sampled_rows():
    g = gg.dcsbm(9000, [0.5, 0.5], 3.0, seed=13)
    w = gg.edge_weights(g, 2, seed=13)
    rows = np.random.default_rng(13).choice(g.n, 40, replace=False)
    check(g, w, [1.5, 4.0], rows=rows)


def test_batch_mixes_weighted_and_unweighted():
    import torch
    from paper_2305_14641_amd import qc
    gs = [gg.config2(), gg.dcsbm(3000, [0.6, 0.4], 3.0, seed=14), gg.config1()]
    ws = [gg.edge_weights(gs[0], 3, seed=1), None, gg.edge_weights(gs[2], 2, seed=2)]
    handles = [qc.Graph(g.n, g.row_ptr, g.col, weights=w) for g, w in zip(gs, ws)]
    sigmas = [0.8, 2.0]
    b = qc.Batch(handles, sigmas, hipgraph=True)
    psi, v, lab = b.outputs()
    b.run(psi, v, lab)
    b.run(psi, v, lab)
    torch.cuda.synchronize()
    lab = lab.cpu().numpy()
    for i, (g, w) in enumerate(zip(gs, ws)):
        if w is None:
            ref, _ = oracle.distances(g.n, g.row_ptr, g.col)
        else:
            ref, _ = oracle.weighted_distances(g.n, g.row_ptr, g.col, w)
        ref_hist = oracle.hist_rows(ref, 128)
        o0, o1 = b.offsets[i], b.offsets[i + 1]
        for s, sigma in enumerate(sigmas):
            _, v_c = oracle.potential_canonical(ref_hist, sigma)
            want = oracle.find_centers(oracle.ggd_parent(g.n, g.row_ptr, g.col, v_c, 0))
            np.testing.assert_array_equal(lab[s, o0:o1], want, err_msg=f"graph {i} sigma {sigma}")
    b.close()


def test_weighted_distance_limit():
    import torch
    from paper_2305_14641_amd import qc
    g = gg.path_graph(4)
    ok = qc.Graph(g.n, g.row_ptr, g.col, weights=np.full(g.nnz, 42, dtype=np.uint8))
    dist = torch.empty((4, 4), dtype=torch.int8, device="cuda")
    assert ok.distances(dist) == 126
    ok.close()
    bad = qc.Graph(g.n, g.row_ptr, g.col, weights=np.full(g.nnz, 43, dtype=np.uint8))
    with pytest.raises(qc.QCError) as e:
        bad.distances()
        bad.sync()
    assert e.value.status == qc.QC_E_OVERFLOW
    bad.close()
