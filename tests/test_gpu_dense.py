"""Algorithm 1 on dense real-valued distances (qc_potential_dense) against the
oracle's dense pair sum and its literal-reading function.

Cases: several tiles of rows with a ragged row tail, chunked sigma lists
(1, 3, 8 and 11 widths: padded chunks and a second pass), unaligned rows
(scalar path), padded rows (16-byte path with a column tail), entries that
mean "no path" (negative, NaN, infinite), empty rows and columns, the
weighted literal distance of Section 3.1, the hop-distance matrix (which must
agree with the histogram path) and, at the full size of the fully connected
workload, sampled rows.
"""
import numpy as np
import pytest

import oracle
from paper_2305_14641_amd import graphgen as gg

pytestmark = pytest.mark.gpu

TOL = 1e-6


def rel_err(got, want):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    assert np.array_equal(np.isnan(got), np.isnan(want))
    ok = ~np.isnan(want)
    got, want = got[ok], want[ok]
    zero = want == 0
    assert (got[zero] == 0).all()
    return float((np.abs(got - want)[~zero] / np.abs(want[~zero])).max()) if (~zero).any() else 0.0


def run(d_host, sigmas, n_cols=None, ld=None):
    import torch
    from paper_2305_14641_amd import qc
    n_rows, n = d_host.shape
    if ld is None:
        dev = torch.as_tensor(d_host).cuda()
    else:
        buf = torch.full((n_rows, ld), 7.0, dtype=torch.float32, device="cuda")
        buf[:, :n] = torch.as_tensor(d_host).cuda()
        dev = buf[:, :n] if n_cols is None else buf
    psi, v = qc.potential_dense(dev, sigmas, n_cols=n if ld is not None else n_cols)
    torch.cuda.synchronize()
    return psi.cpu().numpy(), v.cpu().numpy()


def check(d_host, sigmas, **kw):
    psi, v = run(d_host, sigmas, **kw)
    worst = 0.0
    for s, sigma in enumerate(sigmas):
        psi_o, v_o = oracle.potential_dense(d_host, sigma)
        worst = max(worst, rel_err(psi[s], psi_o), rel_err(v[s], v_o))
    assert worst <= TOL, worst
    return worst


@pytest.mark.parametrize("n_sig", [1, 3, 8, 11])
def test_points_chunked_sigmas(n_sig):
    d = gg.dense_points(1029, dim=8, clusters=6, seed=n_sig)
    sigmas = list(np.geomspace(0.3, 12.0, n_sig))
    w = check(d, sigmas)
    print(f"[gpu] dense n=1029 S={n_sig}: worst rel err {w:.2e}", flush=True)


@pytest.mark.parametrize("ld", [None, 1003, 1008])
def test_row_layouts(ld):
    """Unit-stride rows of 1003 floats: packed (unaligned rows, scalar path)
    and padded to 1008 (16-byte rows, column tail of 3)."""
    d = gg.dense_points(1003, dim=5, clusters=3, seed=7)[:517]
    check(d, [0.8, 2.0], ld=ld)


def test_no_path_entries_and_degenerate_rows():
    d = gg.dense_points(300, dim=4, clusters=3, seed=9)
    rng = np.random.default_rng(9)
    mask = rng.random(d.shape)
    d[mask < 0.05] = -1.0
    d[(mask >= 0.05) & (mask < 0.07)] = np.nan
    d[(mask >= 0.07) & (mask < 0.09)] = np.inf
    d[(mask >= 0.09) & (mask < 0.10)] = -np.inf
    d[(mask >= 0.10) & (mask < 0.11)] = 3.0e38      # finite, weight underflows to 0
    d[5, :] = -1.0                                   # a row with no counted entry
    psi, v = run(d, [1.5])
    assert psi[0, 5] == 0.0 and np.isnan(v[0, 5])
    check(d, [0.5, 1.5, 40.0])


def test_empty_inputs():
    import torch
    from paper_2305_14641_amd import qc
    none = torch.empty((0, 16), dtype=torch.float32, device="cuda")
    psi, v = qc.potential_dense(none, [1.0])
    assert psi.shape == (1, 0)
    cols0 = torch.empty((6, 0), dtype=torch.float32, device="cuda")
    psi, v = qc.potential_dense(cols0, [1.0, 2.0])
    torch.cuda.synchronize()
    assert (psi.cpu().numpy() == 0).all() and np.isnan(v.cpu().numpy()).all()


def test_weighted_literal_distance():
    """Section 3.1 read literally on a weighted graph: an edge's weight, a cap
    above every weight for a non-edge, zero on the diagonal. The dense matrix
    is written out on the host; the oracle reads the CSR directly."""
    g = gg.config2()
    rng = np.random.default_rng(21)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    lo, hi = np.minimum(rows, g.col), np.maximum(rows, g.col)
    w_pair = 0.5 + 1.5 * rng.random(g.n * g.n // 2 + g.n)   # symmetric via the pair key
    key = lo.astype(np.int64) * g.n + hi - lo * (lo + 1) // 2
    weight = w_pair[key % w_pair.shape[0]].astype(np.float32).astype(np.float64)
    cap = 3.0
    d = np.full((g.n, g.n), cap, dtype=np.float32)
    d[rows, g.col] = weight
    np.fill_diagonal(d, 0.0)
    sigmas = [0.5, 1.0, 2.0, 3.0]
    psi, v = run(d, sigmas)
    for s, sigma in enumerate(sigmas):
        psi_o, v_o = oracle.potential_literal(g.n, g.row_ptr, g.col, sigma, weight=weight, cap=cap)
        assert rel_err(psi[s], psi_o) <= TOL
        assert rel_err(v[s], v_o) <= TOL


def test_hop_matrix_agrees_with_histogram_path():
    """The hop-distance matrix as floats (unreachable = -1, skipped) gives the
    psi and V of the histogram path and of the oracle's canonical sums."""
    import torch
    from paper_2305_14641_amd import qc
    g = gg.config2()
    G = qc.Graph.from_graph(g)
    dist = torch.empty((g.n, g.n), dtype=torch.int8, device="cuda")
    G.distances(dist)
    sigmas = gg.SIGMAS_C2
    psi_h, v_h = G.potential(sigmas)
    psi_d, v_d = qc.potential_dense(dist.float(), sigmas)
    torch.cuda.synchronize()
    ref_hist, _ = oracle.hist_all(g.n, g.row_ptr, g.col, G.histograms().shape[1])
    for s, sigma in enumerate(sigmas):
        psi_c, v_c = oracle.potential_canonical(ref_hist, sigma)
        assert rel_err(psi_d[s].cpu().numpy(), psi_c) <= TOL
        assert rel_err(v_d[s].cpu().numpy(), v_c) <= TOL
        assert rel_err(psi_d[s].cpu().numpy(), psi_h[s].cpu().numpy()) <= 2 * TOL
    G.close()


def test_full_size_fully_connected_sampled_rows():
    """The fully connected workload at n = 20,000 (a 1.6 GB float matrix):
    64 sampled rows against the oracle, every row finite and positive."""
    import torch
    from paper_2305_14641_amd import qc
    n = 20000
    d = gg.dense_points(n, dim=16, clusters=8, seed=3)
    dev = torch.as_tensor(d).cuda()
    sigmas = [2.0, 4.0, 8.0]
    psi, v = qc.potential_dense(dev, sigmas)
    torch.cuda.synchronize()
    psi, v = psi.cpu().numpy(), v.cpu().numpy()
    assert np.isfinite(psi).all() and (psi >= 1.0).all() and np.isfinite(v).all()
    rows = np.random.default_rng(5).choice(n, 64, replace=False)
    for s, sigma in enumerate(sigmas):
        psi_o, v_o = oracle.potential_dense(d[rows], sigma)
        assert rel_err(psi[s, rows], psi_o) <= TOL
        assert rel_err(v[s, rows], v_o) <= TOL
