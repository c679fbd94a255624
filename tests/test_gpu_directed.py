"""Directed graphs (QC_GRAPH_DIRECTED): distances along edge direction, row i
holding the distances from i, and a descent over out-neighbours, against the
oracle (which walks CSR rows as out-edges).

Cases: small random digraphs, citation-shaped directed DC-SBM graphs of
2,708 and 19,717 nodes (full matrices), BFS width classes on sampled rows,
a directed cycle (every source reaches every node, so the search's early
stop fires), a directed path (a closed form: d(i, j) = j - i for j >= i;
no early stop) at the largest distance, 126, and one past it (overflow),
and a batch mixing directed and undirected handles.
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


def directed(g):
    from paper_2305_14641_amd import qc
    return qc.Graph.from_graph(g, directed=True)


def check_full(g, sigmas, dist_rows=None):
    import torch
    G = directed(g)
    dist = torch.empty((g.n, g.n), dtype=torch.int8, device="cuda")
    dmax = G.distances(dist)
    psi, v = G.potential(sigmas)
    labels = {(s, t): G.labels(s, t).cpu().numpy() for s in range(len(sigmas)) for t in (0, 1)}
    G.sync()
    hist = G.histograms().cpu().numpy()
    if dist_rows is None:
        ref, ref_dmax = oracle.distances(g.n, g.row_ptr, g.col)
        np.testing.assert_array_equal(dist.cpu().numpy(), ref)
        ref_hist = oracle.hist_rows(ref, hist.shape[1])
    else:
        ref_hist, ref_dmax = oracle.hist_all(g.n, g.row_ptr, g.col, hist.shape[1])
        rows = np.asarray(dist_rows, dtype=np.int32)
        ref_rows, _ = oracle.bfs_rows(g.n, g.row_ptr, g.col, rows)
        got = dist[torch.as_tensor(rows.astype(np.int64), device="cuda")].cpu().numpy()
        np.testing.assert_array_equal(got, ref_rows)
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


@pytest.mark.parametrize("seed", range(6))
def test_small_random_digraphs(seed):
    g = gg.random_digraph(20 + 7 * seed, 0.04 + 0.02 * seed, seed=seed)
    check_full(g, [0.5, 1.0, 2.0])


@pytest.mark.parametrize("n,deg,seed", [(2708, 2.0, 31), (19717, 2.25, 32)])
def test_citation_shaped_digraphs(n, deg, seed):
    g = gg.dcsbm_directed(n, [0.4, 0.3, 0.2, 0.1], deg, seed=seed)
    print(f"[gpu] directed {g.name}: nnz {g.nnz}", flush=True)
    check_full(g, [0.5, 1.0, 2.0, 3.0])


@pytest.mark.parametrize("n", [3000, 9000, 15000, 40000])
def test_width_classes_sampled_rows(n):
    g = gg.dcsbm_directed(n, [0.5, 0.5], 3.0, seed=n)
    rows = np.random.default_rng(n).choice(n, 48, replace=False)
    check_full(g, [1.0, 2.5], dist_rows=rows)


@pytest.mark.parametrize("n", [120, 127])
def test_directed_cycle_early_stop(n):
    """Distances up to n - 1 (at most 126): every source reaches every node."""
    t = np.arange(n)
    rp, col = gg.csr_from_arcs(n, t, (t + 1) % n)
    g = gg.Graph(n, rp, col, np.zeros(n, dtype=np.int32), name=f"cycle{n}")
    check_full(g, [1.0, 4.0])


@pytest.mark.parametrize("n", [100, 127])
def test_directed_path_closed_form(n):
    import torch
    t = np.arange(n - 1)
    rp, col = gg.csr_from_arcs(n, t, t + 1)
    g = gg.Graph(n, rp, col, np.zeros(n, dtype=np.int32), name=f"dipath{n}")
    G = directed(g)
    dist = torch.empty((n, n), dtype=torch.int8, device="cuda")
    assert G.distances(dist) == n - 1
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    want = np.where(j >= i, j - i, -1).astype(np.int8)
    np.testing.assert_array_equal(dist.cpu().numpy(), want)
    G.close()
    check_full(g, [2.0, 8.0])


def test_directed_path_overflow():
    from paper_2305_14641_amd import qc
    n = 128
    t = np.arange(n - 1)
    rp, col = gg.csr_from_arcs(n, t, t + 1)
    G = qc.Graph(n, rp, col, directed=True)
    with pytest.raises(qc.QCError) as e:
        G.distances()
        G.sync()
    assert e.value.status == qc.QC_E_OVERFLOW
    G.close()


def test_batch_mixes_directed_and_undirected():
    import torch
    from paper_2305_14641_amd import qc
    gs = [gg.dcsbm_directed(1500, [0.5, 0.5], 2.0, seed=41), gg.config2(),
          gg.dcsbm_directed(5000, [0.3, 0.7], 2.5, seed=42)]
    flags = [True, False, True]
    handles = [qc.Graph.from_graph(g, directed=d) for g, d in zip(gs, flags)]
    sigmas = [0.7, 1.5, 3.0]
    b = qc.Batch(handles, sigmas, hipgraph=True)
    psi, v, lab = b.outputs()
    b.run(psi, v, lab)
    b.run(psi, v, lab)
    torch.cuda.synchronize()
    lab = lab.cpu().numpy()
    for i, g in enumerate(gs):
        o0, o1 = b.offsets[i], b.offsets[i + 1]
        ref_hist, _ = oracle.hist_all(g.n, g.row_ptr, g.col, 128)
        for s, sigma in enumerate(sigmas):
            _, v_c = oracle.potential_canonical(ref_hist, sigma)
            ref = oracle.find_centers(oracle.ggd_parent(g.n, g.row_ptr, g.col, v_c, 0))
            np.testing.assert_array_equal(lab[s, o0:o1], ref, err_msg=f"graph {i} sigma {sigma}")
    b.close()
