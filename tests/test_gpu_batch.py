"""The batched form (include/qc_batch.h) against the plain per-graph calls and
the oracle: bitwise-identical outputs, HIP-graph replays identical to eager
runs, and oracle parity on a subset of the batched sigma-sweep graphs."""
import numpy as np
import pytest

import oracle
from paper_2305_14641_amd import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_2305_14641_amd import qc
    assert torch.cuda.is_available()
    # a spread of sizes from the sweep's draw (every BFS width class appears)
    idx = [0, 3, 7, 12, 20, 33, 41, 50, 58, 63]
    graphs = [gg.config4_graph(i) for i in idx] + [gg.path_graph(1), gg.star_graph(30)]
    sigmas = gg.sigmas_c4()[::4]
    print(f"[gpu] batch of {len(graphs)} graphs, n={[g.n for g in graphs]}", flush=True)
    return torch, qc, graphs, sigmas


@pytest.mark.parametrize("tie", [0, 1])
def test_batch_equals_plain_and_oracle(setup, tie):
    torch, qc, graphs, sigmas = setup
    handles = [qc.Graph.from_graph(g) for g in graphs]
    b = qc.Batch(handles, sigmas, tie_mode=tie, hipgraph=True)
    psi, v, lab = b.outputs()
    runs = []
    for r in range(3):      # capture, then replays with eager work in between
        b.run(psi, v, lab)
        torch.cuda.synchronize()
        runs.append((psi.cpu().numpy().copy(), v.cpu().numpy().copy(), lab.cpu().numpy().copy()))
        _ = torch.ones(1000, device="cuda").sum().item()
    for r in runs[1:]:
        for a, c in zip(runs[0], r):
            assert a.tobytes() == c.tobytes()
    psi_b, v_b, lab_b = runs[0]
    for i, (g, G) in enumerate(zip(graphs, handles)):
        o0, o1 = b.offsets[i], b.offsets[i + 1]
        p_, v_ = G.potential(sigmas)
        assert p_.cpu().numpy().tobytes() == np.ascontiguousarray(psi_b[:, o0:o1]).tobytes()
        assert v_.cpu().numpy().tobytes() == np.ascontiguousarray(v_b[:, o0:o1]).tobytes()
        for s in range(len(sigmas)):
            l_ = G.labels(s, tie).cpu().numpy()
            np.testing.assert_array_equal(l_, lab_b[s, o0:o1])
    # oracle parity on the graphs small enough for a quick full check
    for i, g in enumerate(graphs):
        if g.n > 6000:
            continue
        o0, o1 = b.offsets[i], b.offsets[i + 1]
        dist, dmax = oracle.distances(g.n, g.row_ptr, g.col)
        hist = oracle.hist_rows(dist, dmax + 1)
        for s, sigma in enumerate(sigmas):
            psi_c, v_c = oracle.potential_canonical(hist, sigma)
            np.testing.assert_allclose(psi_b[s, o0:o1], psi_c, rtol=1e-6, atol=0)
            np.testing.assert_allclose(v_b[s, o0:o1], v_c, rtol=1e-6, atol=0)
            lab_ref = oracle.find_centers(oracle.ggd_parent(g.n, g.row_ptr, g.col, v_c, tie))
            np.testing.assert_array_equal(lab_b[s, o0:o1], lab_ref)
    b.close()


def test_batch_without_hipgraph_and_fp32c(setup):
    torch, qc, graphs, sigmas = setup
    handles = [qc.Graph.from_graph(g) for g in graphs[:5]]
    b1 = qc.Batch(handles, sigmas, hipgraph=False)
    o1 = b1.outputs()
    b1.run(*o1)
    b2 = qc.Batch(handles, sigmas, hipgraph=False, fp32c=True)
    o2 = b2.outputs()
    b2.run(*o2)
    torch.cuda.synchronize()
    # FP32C and FP64ACC give identical labels
    np.testing.assert_array_equal(o2[2].cpu().numpy(), o1[2].cpu().numpy())
    # FP32C against the oracle's FP64 values to 1e-6 (psi and V) and its
    # labels in both tie modes
    b3 = qc.Batch(handles, sigmas, tie_mode=qc.TIE_MERGE, hipgraph=False, fp32c=True)
    o3 = b3.outputs()
    b3.run(*o3)
    torch.cuda.synchronize()
    psi2, v2, lab2 = (x.cpu().numpy() for x in o2)
    lab3 = o3[2].cpu().numpy()
    for i, g in enumerate(graphs[:5]):
        o0, o1_ = b2.offsets[i], b2.offsets[i + 1]
        hist, _ = oracle.hist_all(g.n, g.row_ptr, g.col, handles[i].histograms_k())
        for s, sigma in enumerate(sigmas):
            psi_c, v_c = oracle.potential_canonical(hist, sigma)
            np.testing.assert_allclose(psi2[s, o0:o1_], psi_c, rtol=1e-6, atol=0)
            np.testing.assert_allclose(v2[s, o0:o1_], v_c, rtol=1e-6, atol=0)
            for tie, lab in ((qc.TIE_STRICT, lab2), (qc.TIE_MERGE, lab3)):
                ref = oracle.find_centers(oracle.ggd_parent(g.n, g.row_ptr, g.col, v_c, tie))
                np.testing.assert_array_equal(lab[s, o0:o1_], ref, err_msg=f"graph {i} sigma {sigma} tie {tie}")
    b3.close()


@pytest.mark.parametrize("S", [1, 5, 7])
def test_batch_sigma_counts(setup, S):
    """Sigma counts that are not a multiple of four: the potential sums four
    sigmas at a time and then one by one, the descent decides groups of four
    sigmas (its last group partly padding), the resident V interleaves
    groups of four; all must match the oracle."""
    torch, qc, graphs, sigmas = setup
    gs = [graphs[1], graphs[3], graphs[-1]]
    sig = list(np.geomspace(0.4, 5.0, S))
    handles = [qc.Graph.from_graph(g) for g in gs]
    b = qc.Batch(handles, sig, hipgraph=False)
    psi, v, lab = b.outputs()
    b.run(psi, v, lab)
    torch.cuda.synchronize()
    psi, v, lab = psi.cpu().numpy(), v.cpu().numpy(), lab.cpu().numpy()
    for i, g in enumerate(gs):
        o0, o1 = b.offsets[i], b.offsets[i + 1]
        dist, dmax = oracle.distances(g.n, g.row_ptr, g.col)
        hist = oracle.hist_rows(dist, dmax + 1)
        for s, sigma in enumerate(sig):
            psi_c, v_c = oracle.potential_canonical(hist, sigma)
            np.testing.assert_allclose(psi[s, o0:o1], psi_c, rtol=1e-6, atol=0)
            np.testing.assert_allclose(v[s, o0:o1], v_c, rtol=1e-6, atol=0)
            ref = oracle.find_centers(oracle.ggd_parent(g.n, g.row_ptr, g.col, v_c, 0))
            np.testing.assert_array_equal(lab[s, o0:o1], ref, err_msg=f"S={S} sigma={sigma}")
    b.close()


def test_batch_autotune_changes_no_output(setup):
    """QC_BATCH_AUTOTUNE times the batch's searches under each planning
    policy and the histogram and jumping shapes, and keeps the fastest; the
    outputs are bitwise those of the planner's shapes."""
    torch, qc, graphs, sigmas = setup
    ha = [qc.Graph.from_graph(g) for g in graphs]
    hb = [qc.Graph.from_graph(g) for g in graphs]
    ba = qc.Batch(ha, sigmas, hipgraph=True, autotune=True)
    bb = qc.Batch(hb, sigmas, hipgraph=True)
    oa, ob = ba.outputs(), bb.outputs()
    for _ in range(2):
        ba.run(*oa)
        bb.run(*ob)
    torch.cuda.synchronize()
    for x, y in zip(oa, ob):
        assert x.cpu().numpy().tobytes() == y.cpu().numpy().tobytes()
    tiles = ba.stage_tiles()
    assert tiles["hist_waves"][32] in (4, 8, 16) and tiles["jump"] in ("lds", "global")
    assert (tiles["bfs_widest"], tiles["bfs_front_first"]) in ((32, True), (64, True), (16, True),
                                                                (32, False))
    # every graph follows the kept policy
    for G in ha:
        assert G.bfs_plan()[0] <= tiles["bfs_widest"]
    assert bb.stage_tiles()["bfs_widest"] == 32 and bb.stage_tiles()["bfs_front_first"]
    # the tuned plan stays with the graph: its own calls agree too
    d = torch.empty((graphs[3].n, graphs[3].n), dtype=torch.int8, device="cuda")
    ha[3].distances(d)
    dist, _ = oracle.distances(graphs[3].n, graphs[3].row_ptr, graphs[3].col)
    np.testing.assert_array_equal(d.cpu().numpy(), dist)
    ba.close()
    bb.close()


@pytest.mark.parametrize("env", [{"QC_HIST_VARIANT": "1"}, {"QC_HIST_VARIANT": "2"},
                                 {"QC_JUMP_VARIANT": "1"}], ids=lambda e: ",".join(f"{k}={v}" for k, v in e.items()))
def test_batch_stage_shapes_change_no_output(setup, monkeypatch, env):
    """The histogram pass in each workgroup shape and the pointer jumping in
    global memory give the bytes of the default shapes, and the batch reports
    the shapes it runs with."""
    torch, qc, graphs, sigmas = setup
    graphs = graphs + [gg.path_graph(40)]   # and a row length of 64 bins
    ha = [qc.Graph.from_graph(g) for g in graphs]
    ba = qc.Batch(ha, sigmas, hipgraph=True)
    for k, val in env.items():
        monkeypatch.setenv(k, val)
    hb = [qc.Graph.from_graph(g) for g in graphs]
    bb = qc.Batch(hb, sigmas, hipgraph=True)
    tiles = bb.stage_tiles()
    if "QC_HIST_VARIANT" in env:
        want = {32: (4, 16), 64: (2, 8), 128: (1, 4)}
        for K, w in tiles["hist_waves"].items():
            if w:
                assert w == want[K][int(env["QC_HIST_VARIANT"]) - 1]
    else:
        assert tiles["jump"] == "global"
    assert ba.stage_tiles()["jump"] == "lds"
    oa, ob = ba.outputs(), bb.outputs()
    for _ in range(2):
        ba.run(*oa)
        bb.run(*ob)
    torch.cuda.synchronize()
    for x, y in zip(oa, ob):
        assert x.cpu().numpy().tobytes() == y.cpu().numpy().tobytes()
    for G, H in zip(ha, hb):
        assert torch.equal(G.histograms(), H.histograms())
    ba.close()
    bb.close()


@pytest.mark.parametrize("form", ["default", "histograms", "all", "tail-one-launch",
                                  "tail-two-launches", "default-eager", "one-search-stream",
                                  "three-search-streams"])
def test_batch_overlapped_stages_change_no_output(setup, monkeypatch, form):
    """The stages beside the searches on the batch's second stream: the
    histograms and the later stages of the first launches' graphs beside the
    last launches (by default; one or two last launches forced), the
    histograms only, or every stage after the search; with the search
    launches on one, two (by default) or three streams (replayed as a HIP
    graph several times with other work in between, or run eagerly). Each
    gives the bytes of the serial form, and the serial form matches the
    oracle."""
    torch, qc, graphs, sigmas = setup
    hs = [qc.Graph.from_graph(g) for g in graphs]
    bs = qc.Batch(hs, sigmas, hipgraph=True, serial=True)
    assert bs.stage_tiles()["overlap"] == "none"
    overlap = {"histograms": "1", "all": "2", "tail-one-launch": "3", "tail-two-launches": "3"}
    if form in overlap:
        monkeypatch.setenv("QC_BATCH_OVERLAP", overlap[form])
    if form.startswith("tail"):
        monkeypatch.setenv("QC_BATCH_TAIL_LAUNCHES", "2" if form.endswith("launches") else "1")
    if form.endswith("search-stream") or form.endswith("search-streams"):
        monkeypatch.setenv("QC_BATCH_BFS_STREAMS", "1" if form.startswith("one") else "3")
    ho = [qc.Graph.from_graph(g) for g in graphs]
    bo = qc.Batch(ho, sigmas, hipgraph=(form != "default-eager"))
    assert bo.stage_tiles()["overlap"] == {"histograms": "histograms", "all": "all"}.get(
        form, "histograms and the tail")
    os_, oo = bs.outputs(), bo.outputs()
    bs.run(*os_)
    torch.cuda.synchronize()
    ref = [x.cpu().numpy().copy() for x in os_]
    for r in range(3):
        for x in oo:
            x.fill_(-7)
        bo.run(*oo)
        torch.cuda.synchronize()
        for x, y in zip(oo, ref):
            assert x.cpu().numpy().tobytes() == y.tobytes(), f"run {r}"
        _ = torch.ones(1000, device="cuda").sum().item()
    for G, H in zip(hs, ho):
        assert torch.equal(G.histograms(), H.histograms())
    for i, g in enumerate(graphs):
        if g.n > 3000:
            continue
        o0, o1 = bs.offsets[i], bs.offsets[i + 1]
        dist, dmax = oracle.distances(g.n, g.row_ptr, g.col)
        hist = oracle.hist_rows(dist, dmax + 1)
        for s, sigma in enumerate(sigmas):
            psi_c, v_c = oracle.potential_canonical(hist, sigma)
            np.testing.assert_allclose(ref[1][s, o0:o1], v_c, rtol=1e-6, atol=0)
            lab = oracle.find_centers(oracle.ggd_parent(g.n, g.row_ptr, g.col, v_c, 0))
            np.testing.assert_array_equal(ref[2][s, o0:o1], lab)
    bs.close()
    bo.close()


def test_batch_rejects_bad_arguments(setup):
    torch, qc, graphs, sigmas = setup
    G = qc.Graph.from_graph(graphs[-1])
    with pytest.raises(qc.QCError):
        qc.Batch([G, G], sigmas)          # a graph twice
    with pytest.raises(qc.QCError):
        qc.Batch([G], [1.0, -2.0])
    with pytest.raises(qc.QCError):
        qc.Batch([G], sigmas, tie_mode=3)


def test_batch_search_stats_count_the_searches_work(setup, monkeypatch):
    """The search kernel's own count of its work: with the sources taken in
    node order (batches of consecutive nodes), a batch pulls one level less
    than its sources' largest eccentricity (level 1 is pushed from the
    sources, and the search stops once every reachable pair is found), so
    edge visits = sum over batches of max(0, max ecc - 1) x edge entries +
    the edge entries pushed at level 1 (every node is a source once), and
    every visit gathers one bit-field word (4 bytes, or 8 for batches of 64)."""
    torch, qc, graphs, sigmas = setup
    monkeypatch.setenv("QC_SOURCE_ORDER", "identity")
    gs = [gg.config2(), gg.config1(), gg.path_graph(70)]
    handles = [qc.Graph.from_graph(g) for g in gs]
    b = qc.Batch(handles, sigmas[:2], hipgraph=True)
    psi, v, lab = b.outputs()
    for _ in range(2):
        b.run(psi, v, lab)
    visits, lds = b.search_stats()
    want_visits = want_bytes = 0
    for g, G in zip(gs, handles):
        bw = G.bfs_plan()[0]
        dist, _ = oracle.distances(g.n, g.row_ptr, g.col)
        ecc = dist.max(axis=1).astype(np.int64)
        pulled = sum(max(0, int(ecc[s0:s0 + bw].max()) - 1) for s0 in range(0, g.n, bw))
        vis = pulled * g.nnz + g.nnz
        want_visits += vis
        want_bytes += vis * (8 if bw == 64 else 4)
    assert visits == want_visits
    assert lds == want_bytes
    b.close()


def test_batch_bf16_sweep(setup):
    """The BF16 matrix-core sweep over the whole batch (one grouped launch per
    histogram row length): bitwise the per-graph BF16 potentials, within the
    BF16 error of the oracle's FP64 values (8 significant bits: a few 1e-3),
    and the batch's own run afterwards is unchanged (nothing resident is
    written)."""
    torch, qc, graphs, sigmas = setup
    sig = gg.sigmas_c4() + [1.0, 2.0]   # 34 sigmas: a second group of weight columns
    # a 40-node path adds a second row length (64 bins): a second launch
    graphs = graphs + [gg.path_graph(40)]
    handles = [qc.Graph.from_graph(g) for g in graphs]
    b = qc.Batch(handles, sig, hipgraph=True)
    psi, v, lab = b.outputs()
    b.run(psi, v, lab)
    torch.cuda.synchronize()
    lab0 = lab.cpu().numpy().copy()
    pb, vb = b.sweep_bf16()
    torch.cuda.synchronize()
    pb, vb = pb.cpu().numpy(), vb.cpu().numpy()
    for i, (g, G) in enumerate(zip(graphs, handles)):
        o0, o1 = b.offsets[i], b.offsets[i + 1]
        hist = G.histograms().cpu().numpy()
        dmax = int(np.nonzero(hist.any(axis=0))[0].max())
        for s in (0, 9, 31):
            psi_c, v_c = oracle.potential_canonical(np.ascontiguousarray(hist[:, :dmax + 1]), sig[s])
            assert np.abs(pb[s, o0:o1] / psi_c - 1).max() < 2e-2
            nz = v_c != 0      # (none on a one-node graph)
            assert np.max(np.abs(vb[s, o0:o1][nz] / v_c[nz] - 1), initial=0.0) < 2e-2
            assert (vb[s, o0:o1][~nz] == 0).all()
        p1, v1 = G.potential(sig, precision=qc.PREC_BF16)
        assert p1.cpu().numpy().tobytes() == np.ascontiguousarray(pb[:, o0:o1]).tobytes()
        assert v1.cpu().numpy().tobytes() == np.ascontiguousarray(vb[:, o0:o1]).tobytes()
    b.run(psi, v, lab)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(lab.cpu().numpy(), lab0)
    b.close()


def test_graph_shared_by_batches_of_other_launch_shapes(setup, monkeypatch):
    """One graph in two batches whose plans take different BFS launch shapes
    (so its packed edges carry different row biases): each run finds the
    edges in the other's form and re-uploads them, so a replay of the first
    batch after the second was planned gives the first run's outputs, and a
    plain call afterwards searches correctly under its own plan."""
    torch, qc, _, sigmas = setup
    g = gg.dcsbm(17000, [0.25, 0.25, 0.25, 0.25], 8.0, seed=11)
    print(f"[gpu] shared graph n={g.n}", flush=True)
    G = qc.Graph.from_graph(g)
    # the 512-thread two-field shape: 38 words per thread, a different field
    # size (and so row bias) from every plan the autotuner's policies give
    monkeypatch.setenv("QC_BFS_SHAPE", "1")
    ba = qc.Batch([G], sigmas, hipgraph=True)
    monkeypatch.delenv("QC_BFS_SHAPE")
    plan_a = G.bfs_plan()
    assert plan_a[3] == 1, plan_a
    oa = ba.outputs()
    ba.run(*oa)
    torch.cuda.synchronize()
    first = [x.cpu().numpy().copy() for x in oa]
    bb = qc.Batch([G], sigmas, hipgraph=True, autotune=True)
    plan_b = G.bfs_plan()
    assert plan_b != plan_a
    ob = bb.outputs()
    bb.run(*ob)
    ba.run(*oa)
    torch.cuda.synchronize()
    for x, y, z in zip(first, oa, ob):
        assert x.tobytes() == y.cpu().numpy().tobytes()
        assert x.tobytes() == z.cpu().numpy().tobytes()
    d = torch.empty((g.n, g.n), dtype=torch.int8, device="cuda")
    G.distances(d)
    rows = np.random.default_rng(5).choice(g.n, 24, replace=False)
    ref, _ = oracle.bfs_rows(g.n, g.row_ptr, g.col, rows)
    np.testing.assert_array_equal(d[torch.as_tensor(rows, device="cuda")].cpu().numpy(), ref)
    ba.close()
    bb.close()
