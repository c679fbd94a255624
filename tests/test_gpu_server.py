"""The serving form (include/qc_server.h): results alone and in a mix of
concurrent requests are bitwise identical and match the oracle, admission
respects the memory budget, and requests really overlap."""
import numpy as np
import pytest

import oracle
from paper_2305_14641_amd import graphgen as gg

pytestmark = pytest.mark.gpu


def requests(count):
    out = []
    for r in range(count):
        p = gg.config5_request(r)
        n = min(p["n"], 6000)  # keep the oracle quick; mixed sizes remain
        g = gg.dcsbm(n, p["fracs"], p["deg"], seed=2_000_000 + p["seed"])
        out.append((g, p["sigmas"]))
    return out


def test_server_alone_equals_mix_and_oracle():
    import torch
    from paper_2305_14641_amd import qc
    assert torch.cuda.is_available()
    reqs = requests(12)
    print(f"[gpu] server requests n={[g.n for g, _ in reqs]}", flush=True)
    # alone: one slot, one request at a time
    alone = []
    srv = qc.Server(max_slots=1, hbm_budget_bytes=4 << 30, want_potentials=True)
    for g, sig in reqs:
        rid = srv.submit(g.n, g.row_ptr, g.col, sig)
        alone.append(srv.wait(rid))
    srv.close()
    # mix: everything submitted at once on 4 slots, a budget that holds ~3
    fps = [qc.request_footprint(g.n, g.nnz, len(sig)) for g, sig in reqs]
    budget = int(sorted(fps)[-1] + sorted(fps)[-2] + sorted(fps)[-3])
    srv = qc.Server(max_slots=4, hbm_budget_bytes=budget, want_potentials=True)
    ids = [srv.submit(g.n, g.row_ptr, g.col, sig) for g, sig in reqs]
    mix = [srv.wait(i) for i in ids]
    stats = srv.stats()
    srv.close()
    assert stats["peak_bytes_in_flight"] <= budget
    assert stats["peak_requests_in_flight"] >= 2, stats
    for (g, sig), a, m in zip(reqs, alone, mix):
        assert a[0].tobytes() == m[0].tobytes()
        assert a[1].tobytes() == m[1].tobytes() and a[2].tobytes() == m[2].tobytes()
        assert m[3]["status"] == 0 and m[3]["t_done"] >= m[3]["t_admit"] >= m[3]["t_submit"]
        dist, dmax = oracle.distances(g.n, g.row_ptr, g.col)
        hist = oracle.hist_rows(dist, dmax + 1)
        assert m[3]["dmax"] == dmax
        for s, sigma in enumerate(sig):
            psi_c, v_c = oracle.potential_canonical(hist, sigma)
            np.testing.assert_allclose(m[1][s], psi_c, rtol=1e-6, atol=0)
            np.testing.assert_allclose(m[2][s], v_c, rtol=1e-6, atol=0)
            lab = oracle.find_centers(oracle.ggd_parent(g.n, g.row_ptr, g.col, v_c, 0))
            np.testing.assert_array_equal(m[0][s], lab)


def test_server_rejects_over_budget_and_bad_input():
    from paper_2305_14641_amd import qc
    g = gg.config1()
    fp = qc.request_footprint(g.n, g.nnz, 1)
    srv = qc.Server(max_slots=2, hbm_budget_bytes=fp - 1)
    with pytest.raises(qc.QCError) as e:
        srv.submit(g.n, g.row_ptr, g.col, [1.0])
    assert e.value.status == qc.QC_E_BUSY
    with pytest.raises(qc.QCError) as e:
        srv.submit(g.n, g.row_ptr, g.col, [0.0])
    assert e.value.status == qc.QC_E_INVAL
    srv.close()
    srv = qc.Server(max_slots=2, hbm_budget_bytes=fp)
    rid = srv.submit(g.n, g.row_ptr, g.col, [1.0])
    lab, _, _, info = srv.wait(rid)
    assert lab.shape == (1, g.n) and info["footprint_bytes"] == fp
    srv.close()
