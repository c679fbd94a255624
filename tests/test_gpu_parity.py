"""Parity of the HIP path (through the C ABI) against the CPU oracle.

Bars: distances, histograms and labels bit-exact; psi and V within 1e-6
relative of the oracle's FP64 values (both the literal pair sum of
Algorithm 1 and the canonical histogram form).
"""
import numpy as np
import pytest

import oracle
from paper_2305_14641_amd import graphgen as gg

pytestmark = pytest.mark.gpu

RTOL = 1e-6


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible gfx950 device"
    from paper_2305_14641_amd import qc
    assert qc.device_count() >= 1, "no gfx950 device visible to the HIP library"
    return torch


def rel_err(got, want):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    denom = np.where(want == 0, 1.0, np.abs(want))
    err = np.abs(got - want) / denom
    zero = want == 0
    assert (got[zero] == 0).all(), "exact zeros must stay exact"
    return float(err.max()) if err.size else 0.0


def run_gpu(torch, g, sigmas, ties=(0, 1), precision=0, want_dist=True, repeat=1):
    from paper_2305_14641_amd import qc
    G = qc.Graph.from_graph(g)
    dist = torch.empty((g.n, g.n), dtype=torch.int8, device="cuda") if want_dist else None
    for _ in range(repeat):   # later runs: the final batch width and edge order
        dmax = G.distances(dist)
    hist = G.histograms()
    psi, v = G.potential(sigmas, precision=precision)
    labels = {}
    for s in range(len(sigmas)):
        for t in ties:
            labels[(s, t)] = G.labels(s, t).cpu().numpy()
    G.sync()
    out = dict(G=G, dmax=dmax, hist=hist.cpu().numpy(), psi=psi.cpu().numpy(),
               v=v.cpu().numpy(), labels=labels)
    if want_dist:
        out["dist"] = dist.cpu().numpy()
    return out


def check_against_oracle(g, sigmas, res, ties=(0, 1), pairsum=True):
    ref_dist, ref_dmax = oracle.distances(g.n, g.row_ptr, g.col)
    assert res["dmax"] == ref_dmax
    if "dist" in res:
        np.testing.assert_array_equal(res["dist"], ref_dist)
    K = res["hist"].shape[1]
    assert K >= ref_dmax + 1 and K % 32 == 0
    ref_hist = oracle.hist_rows(ref_dist, K)
    np.testing.assert_array_equal(res["hist"], ref_hist)
    for s, sigma in enumerate(sigmas):
        psi_c, v_c = oracle.potential_canonical(ref_hist, sigma)
        assert rel_err(res["psi"][s], psi_c) <= RTOL
        assert rel_err(res["v"][s], v_c) <= RTOL
        if pairsum:
            psi_p, v_p = oracle.potential_pairsum(ref_dist, sigma)
            assert rel_err(res["psi"][s], psi_p) <= RTOL
            assert rel_err(res["v"][s], v_p) <= RTOL
        for t in ties:
            par = oracle.ggd_parent(g.n, g.row_ptr, g.col, v_c, t)
            lab = oracle.find_centers(par)
            np.testing.assert_array_equal(res["labels"][(s, t)], lab,
                                          err_msg=f"labels sigma={sigma} tie={t}")


SMALL = [
    gg.path_graph(1), gg.path_graph(2), gg.path_graph(5), gg.path_graph(70), gg.star_graph(4),
    gg.star_graph(200), gg.complete_graph(4), gg.complete_graph(65), gg.barbell_graph(4),
    gg.empty_graph(7), gg.disjoint_union(gg.path_graph(4), gg.empty_graph(2), gg.complete_graph(3)),
    gg.twin_leaves(5, 40), gg.random_graph(300, 0.01, 3), gg.random_graph(129, 0.05, 4),
]


@pytest.mark.parametrize("g", SMALL, ids=lambda g: g.name)
def test_small_graphs(torch_cuda, g):
    print(f"[gpu] small graph {g.name} n={g.n} nnz={g.nnz}", flush=True)
    sigmas = [0.5, 1.0, 2.0]
    res = run_gpu(torch_cuda, g, sigmas)
    check_against_oracle(g, sigmas, res)


def test_config1(torch_cuda):
    g = gg.config1()
    print(f"[gpu] config1 n={g.n}", flush=True)
    res = run_gpu(torch_cuda, g, gg.SIGMAS_C1 + [0.25, 8.0])
    check_against_oracle(g, gg.SIGMAS_C1 + [0.25, 8.0], res)


def test_config2(torch_cuda):
    g = gg.config2()
    print(f"[gpu] config2 n={g.n}", flush=True)
    res = run_gpu(torch_cuda, g, gg.SIGMAS_C2)
    check_against_oracle(g, gg.SIGMAS_C2, res)


def test_config2_fp32c(torch_cuda):
    from paper_2305_14641_amd import qc
    g = gg.config2()
    print(f"[gpu] config2 fp32c n={g.n}", flush=True)
    res = run_gpu(torch_cuda, g, gg.SIGMAS_C2, precision=qc.PREC_FP32C, want_dist=False)
    check_against_oracle(g, gg.SIGMAS_C2, res, pairsum=False)


def test_config3_full(torch_cuda):
    """Full N=19,717 graph: the whole 389 MB distance matrix bit-exact."""
    g = gg.config3()
    print(f"[gpu] config3 n={g.n} nnz={g.nnz}", flush=True)
    res = run_gpu(torch_cuda, g, gg.SIGMAS_C3 + [0.5])
    check_against_oracle(g, gg.SIGMAS_C3 + [0.5], res, pairsum=False)
    # the literal pair sum on sampled rows
    rng = np.random.default_rng(11)
    rows = np.sort(rng.choice(g.n, 64, replace=False)).astype(np.int32)
    drows, _ = oracle.bfs_rows(g.n, g.row_ptr, g.col, rows)
    for s, sigma in enumerate(gg.SIGMAS_C3 + [0.5]):
        psi_p, v_p = oracle.potential_pairsum(drows, sigma)
        assert rel_err(res["psi"][s][rows], psi_p) <= RTOL
        assert rel_err(res["v"][s][rows], v_p) <= RTOL


def test_config3_fp32c(torch_cuda):
    """Config 3 (N=19,717) with compensated FP32 potentials and the FP64
    re-decision of near ties: psi/V within 1e-6 of the oracle's canonical FP64
    values and labels bit-exact in both tie modes."""
    from paper_2305_14641_amd import qc
    g = gg.config3()
    sig = [2.0, 0.5]
    print(f"[gpu] config3 fp32c n={g.n}", flush=True)
    res = run_gpu(torch_cuda, g, sig, precision=qc.PREC_FP32C, want_dist=False)
    assert res["G"].recheck_count() >= 0
    check_against_oracle(g, sig, res, pairsum=False)


@pytest.mark.parametrize("n,deg,seed", [
    (3000, 5.0, 21),     # batch width 64
    (9000, 4.0, 22),     # 32, then 64 (two fields, 1024 threads, 18 words) once dmax is known
    (12000, 4.0, 31),    # 32 (three fields, 12 words, 7 planes), then 32 with 4 planes
    (15000, 4.0, 26),    # 16, then 32 (two fields, 1024 threads, 16 words, 4 planes)
    (18000, 4.0, 27),    # 16, then 32 (two fields, 1024 threads, 18 words)
    (19000, 4.0, 28),    # 16, then 32 (two fields, 1024 threads, 19 words: all of the LDS)
    (19800, 4.5, 29),    # 16, then 32 (two fields, 512 threads, 39 words)
    (20001, 3.0, 23),    # 16
    (40000, 3.0, 24),    # 8, then 16 (two fields)
    (50003, 3.0, 25),    # 4, then 8 (two fields, 1024 threads, 14 words, 5 planes)
    (13000, 0.0, 7),     # sparse SBM, largest distance 20: 32 (two fields, 1024 threads, 5 planes)
    (17000, 0.0, 8),     # sparse SBM, largest distance 19: 16, then 32 (1024 threads, 18 words, 5 planes)
    (15500, 2.5, 35),    # largest distance 17: 32 (two fields, 1024 threads, 16 words, 5 planes)
])
def test_batch_width_classes_sampled(torch_cuda, n, deg, seed):
    """Every BFS launch shape, ragged last batch: the first run (7 planes)
    and the re-planned run (planes for dmax, maybe a wider batch) give the
    same matrix; sampled rows bit-exact, all histograms bit-exact (oracle
    without the matrix), labels bit-exact."""
    from paper_2305_14641_amd import qc
    torch = torch_cuda
    if deg > 0:
        g = gg.dcsbm(n, [0.5, 0.3, 0.2], deg, seed=seed)
    else:
        g = gg.sbm(n, 1, 5e-5, 5e-5, seed=seed)
    print(f"[gpu] width class n={n} nnz={g.nnz}", flush=True)
    G = qc.Graph.from_graph(g)
    dist = torch.empty((n, n), dtype=torch.int8, device="cuda")
    dmax = G.distances(dist)
    rng = np.random.default_rng(seed)
    rows = np.unique(np.concatenate([rng.choice(n, 48, replace=False), [0, n - 1, n - 2]]))
    rows = rows.astype(np.int32)
    ref_rows, _ = oracle.bfs_rows(n, g.row_ptr, g.col, rows)
    got_rows = dist[torch.as_tensor(rows.astype(np.int64), device="cuda")].cpu().numpy()
    np.testing.assert_array_equal(got_rows, ref_rows)
    dist2 = torch.empty_like(dist)
    assert G.distances(dist2) == dmax        # second run: the re-planned shape
    assert torch.equal(dist, dist2)
    del dist, dist2
    hist = G.histograms().cpu().numpy()
    ref_hist, ref_dmax = oracle.hist_all(n, g.row_ptr, g.col, hist.shape[1])
    assert dmax == ref_dmax
    np.testing.assert_array_equal(hist, ref_hist)
    sig = [1.5]
    psi, v = G.potential(sig)
    lab = G.labels(0, qc.TIE_STRICT).cpu().numpy()
    psi_c, v_c = oracle.potential_canonical(ref_hist, sig[0])
    assert rel_err(psi.cpu().numpy()[0], psi_c) <= RTOL
    assert rel_err(v.cpu().numpy()[0], v_c) <= RTOL
    ref_lab = oracle.find_centers(oracle.ggd_parent(n, g.row_ptr, g.col, v_c, 0))
    np.testing.assert_array_equal(lab, ref_lab)


def test_distance_limit(torch_cuda):
    from paper_2305_14641_amd import qc
    torch = torch_cuda
    ok = gg.path_graph(127)
    print("[gpu] distance limit", flush=True)
    G = qc.Graph.from_graph(ok)
    dist = torch.empty((127, 127), dtype=torch.int8, device="cuda")
    assert G.distances(dist) == 126
    ref, _ = oracle.distances(ok.n, ok.row_ptr, ok.col)
    np.testing.assert_array_equal(dist.cpu().numpy(), ref)
    bad = gg.path_graph(128)
    G2 = qc.Graph.from_graph(bad)
    with pytest.raises(qc.QCError) as e:
        G2.distances()
    assert e.value.status == qc.QC_E_OVERFLOW


def test_call_order_and_arguments(torch_cuda):
    from paper_2305_14641_amd import qc
    g = gg.config1()
    G = qc.Graph.from_graph(g)
    with pytest.raises(qc.QCError) as e:
        G.labels(0)
    assert e.value.status == qc.QC_E_STATE
    for bad in ([0.0], [-1.0], [float("nan")], [float("inf")]):
        with pytest.raises(qc.QCError) as e:
            G.potential(bad)
        assert e.value.status == qc.QC_E_INVAL
    G.potential([1.0, 2.0])          # runs the distances itself
    with pytest.raises(qc.QCError):
        G.labels(2)                  # sigma index out of range
    with pytest.raises(qc.QCError):
        G.labels(0, tie_mode=7)
    G.labels(1)
    G.sync()


def test_deterministic_and_repeatable(torch_cuda):
    torch = torch_cuda
    g = gg.config2()
    a = run_gpu(torch, g, gg.SIGMAS_C2)
    b = run_gpu(torch, g, gg.SIGMAS_C2)
    np.testing.assert_array_equal(a["dist"], b["dist"])
    assert a["psi"].tobytes() == b["psi"].tobytes()
    assert a["v"].tobytes() == b["v"].tobytes()
    for k in a["labels"]:
        np.testing.assert_array_equal(a["labels"][k], b["labels"][k])
    # a second qc_distances on the same handle gives the same matrix
    G = a["G"]
    d2 = torch.empty((g.n, g.n), dtype=torch.int8, device="cuda")
    G.distances(d2)
    np.testing.assert_array_equal(d2.cpu().numpy(), a["dist"])


@pytest.mark.parametrize("g", [gg.config1(), gg.random_graph(700, 0.004, 9),
                               gg.disjoint_union(gg.path_graph(90), gg.empty_graph(5),
                                                 gg.complete_graph(40)),
                               gg.dcsbm(5000, [0.5, 0.3, 0.2], 5.0, seed=41)],
                         ids=lambda g: g.name)
@pytest.mark.parametrize("env", [{"QC_SOURCE_ORDER": "identity"}, {"QC_EDGE_BANKS": "0"},
                                 {"QC_EDGE_BANKS": "64"}, {"QC_BFS_SHAPE": "0"},
                                 {"QC_BFS_SHAPE": "1"}, {"QC_BFS_SHAPE": "2"},
                                 {"QC_BFS_SHAPE": "3"}],
                         ids=lambda e: ",".join(f"{k}={v}" for k, v in e.items()))
def test_search_order_changes_nothing(torch_cuda, monkeypatch, g, env):
    """The BFS takes its sources in an order estimated from eccentricity
    bounds, and the edges of each pull group in an order that spreads the
    gathers over the LDS banks; the node order (QC_SOURCE_ORDER=identity),
    the plain rows-ascending edge order (QC_EDGE_BANKS=0), another bank
    count, or any workgroup shape of the search (QC_BFS_SHAPE, taken from
    the second search on, once the largest distance is known) must give the
    same bytes everywhere."""
    torch = torch_cuda
    print(f"[gpu] search order {g.name} n={g.n} {env}", flush=True)
    a = run_gpu(torch, g, [0.7, 2.0], repeat=2)
    for k, val in env.items():
        monkeypatch.setenv(k, val)
    b = run_gpu(torch, g, [0.7, 2.0], repeat=2)
    np.testing.assert_array_equal(a["dist"], b["dist"])
    assert a["dmax"] == b["dmax"]
    np.testing.assert_array_equal(a["hist"], b["hist"])
    assert a["v"].tobytes() == b["v"].tobytes()
    for k in a["labels"]:
        np.testing.assert_array_equal(a["labels"][k], b["labels"][k])
    check_against_oracle(g, [0.7, 2.0], b, ties=(0,), pairsum=False)


def front_plan(n, dmax):
    """Batch width and words per thread of the seen-in-registers shape: the
    widest batch whose bit fields fit 16 words per thread (4 planes, largest
    distance <= 15; 14 words are then taken as 16) or 14 (5 planes) at 1024
    threads."""
    max_nw = 16 if dmax <= 15 else 14
    for bw in (64, 32, 16, 8):
        need = -(-(-(-n * bw // 32)) // 1024)
        for nw in (4, 8, 12, 14, 16):
            if nw > max_nw:
                break
            if bw == 64 and nw % 2:
                continue
            if nw == 14 and dmax <= 15:
                continue
            if nw >= need:
                return bw, nw
    return None


@pytest.mark.parametrize("n,deg,seed", [
    (15000, 4.0, 26),   # 32 sources, 15 of 16 words per thread
    (9000, 4.0, 22),    # 64 sources would need 18 words: 32 sources
    (6000, 5.0, 21),    # 64 sources (64-bit fields)
    (7500, 4.0, 36),    # 64 sources, 16 words: 64 KB fields, edge rows packed with a bias
    (16500, 4.0, 27),   # beyond 16 words at 32 sources: 16 sources
    (13500, 2.5, 33),   # largest distance above 15: 5 planes, 14 words
])
def test_seen_in_registers_shape(torch_cuda, monkeypatch, n, deg, seed):
    """The search shape that keeps `seen` in its owners' registers (two LDS
    fields, pull from the frontier): sampled rows bit-exact, the whole
    matrix equal to the planner's own shape, histograms and labels exact."""
    from paper_2305_14641_amd import qc
    torch = torch_cuda
    g = gg.dcsbm(n, [0.5, 0.3, 0.2], deg, seed=seed)
    print(f"[gpu] seen-in-registers shape n={n} nnz={g.nnz}", flush=True)
    ref = run_gpu(torch, g, [1.5], ties=(0,), repeat=2)
    monkeypatch.setenv("QC_BFS_SHAPE", "3")
    G = qc.Graph.from_graph(g)
    dist = torch.empty((n, n), dtype=torch.int8, device="cuda")
    dmax = G.distances(dist)
    assert G.distances(dist) == dmax
    bw, nw, planes, shape = G.bfs_plan()
    assert (bw, nw, shape) == front_plan(n, dmax) + (3,), (bw, nw, planes, shape)
    assert torch.equal(dist, torch.as_tensor(ref["dist"], device="cuda"))
    rows = np.unique(np.random.default_rng(seed).choice(n, 24, replace=False)).astype(np.int32)
    ref_rows, _ = oracle.bfs_rows(n, g.row_ptr, g.col, rows)
    np.testing.assert_array_equal(dist[torch.as_tensor(rows.astype(np.int64), device="cuda")]
                                  .cpu().numpy(), ref_rows)
    del dist
    hist = G.histograms().cpu().numpy()
    np.testing.assert_array_equal(hist, ref["hist"])
    psi, v = G.potential([1.5])
    lab = G.labels(0, qc.TIE_STRICT).cpu().numpy()
    np.testing.assert_array_equal(lab, ref["labels"][(0, 0)])
    if n <= 9000:
        check_against_oracle(g, [1.5], ref, ties=(0,), pairsum=False)


def test_recheck_counts_exact_ties(torch_cuda):
    """Twin leaves have exactly equal V: their hub's decision is re-decided in
    FP64, and the count is reported."""
    from paper_2305_14641_amd import qc
    g = gg.star_graph(50)
    G = qc.Graph.from_graph(g)
    G.potential([0.5])
    lab = G.labels(0, qc.TIE_STRICT).cpu().numpy()
    assert G.recheck_count() >= 1
    assert lab[0] == 1 and (lab[1:] == np.arange(1, 51)).all()


def test_bf16_sweep_error_and_refusal(torch_cuda):
    """The BF16 matrix-core sweep: about 1e-3 relative error vs FP64 (BF16
    keeps 8 significant bits), and the descent refuses its potentials."""
    from paper_2305_14641_amd import qc
    g = gg.config2()
    sig = gg.SIGMAS_C2 + [0.25, 8.0]
    G = qc.Graph.from_graph(g)
    psi, v = G.potential(sig, precision=qc.PREC_BF16)
    hist = G.histograms().cpu().numpy()
    psi, v = psi.cpu().numpy(), v.cpu().numpy()
    worst = 0.0
    for s, sigma in enumerate(sig):
        psi_c, v_c = oracle.potential_canonical(hist, sigma)
        worst = max(worst, rel_err(psi[s], psi_c), rel_err(v[s], v_c))
    print(f"[gpu] bf16 sweep worst relative error {worst:.2e}", flush=True)
    assert worst < 1.5e-2
    with pytest.raises(qc.QCError) as e:
        G.labels(0)
    assert e.value.status == qc.QC_E_STATE
    G.potential(sig)                 # FP64 again: the descent works
    G.labels(0)
    G.sync()
