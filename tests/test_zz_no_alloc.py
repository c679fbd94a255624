"""The no-allocation entry point qc_cluster_noalloc against qc_cluster and
against the per-step calls on a graph handle.

All run Algorithm 4 (distances, psi/V of Eq. 2 / Algorithm 1, the descent
of Algorithms 2-3) on the same graphs; the no-allocation call carves all its
device buffers from the library's fixed device scratch (as qc_cluster does
for a problem that fits it), the handle's calls use buffers of their own.
Checked: outputs equal to the handle's and to qc_cluster's (distances,
labels bit for bit, psi/V within 1e-6 and in fact equal) on consecutive
calls that reuse the scratch, the second one smaller; no device memory is
taken from the driver or the library's allocator during a call; a problem
beyond the scratch is refused before any device work, and qc_cluster runs
it on buffers of its own.
"""
import gc

import numpy as np
import pytest

import oracle
from paper_2305_14641_amd import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2305_14641_amd import qc
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    qc.debug_alloc_fault(0)
    return torch, qc


def handle_path(qc, n, row_ptr, col, sigmas, tie_mode, labels, psi, v, dist):
    """Algorithm 4 through the per-step calls on a graph handle."""
    G = qc.Graph(n, row_ptr, col)
    G.distances(dist)
    p_, v_ = G.potential(sigmas)
    psi.copy_(p_)
    v.copy_(v_)
    for k in range(len(sigmas)):
        labels[k].copy_(G.labels(k, tie_mode))
    G.sync()
    G.close()


def run_both(torch, qc, g, sigmas, with_dist, tie=0):
    """The handle's calls, qc_cluster and qc_cluster_noalloc on g with
    preallocated outputs; returns the handle's outputs and, for the last
    call, its outputs and the device memory it took (driver free-memory
    drop, library allocator blocks, torch bytes), after checking that
    qc_cluster's outputs equal the handle's."""
    S, n = len(sigmas), g.n
    outs = []
    for fn in (handle_path, qc.cluster, qc.cluster_noalloc):
        o = dict(labels=torch.full((S, n), -7, dtype=torch.int32, device="cuda"),
                 psi=torch.full((S, n), -1.0, dtype=torch.float32, device="cuda"),
                 v=torch.full((S, n), -1.0, dtype=torch.float32, device="cuda"),
                 dist=torch.full((n, n), 99, dtype=torch.int8, device="cuda") if with_dist else None)
        torch.cuda.synchronize()
        gc.collect()
        free0, _ = torch.cuda.mem_get_info()
        blocks0 = qc.debug_alloc_fault(0)
        torch0 = torch.cuda.memory_allocated()
        print(f"[gpu] {fn.__name__} n={n} S={S} dist={with_dist} tie={tie}", flush=True)
        if fn is handle_path:
            fn(qc, n, g.row_ptr, g.col, sigmas, tie, **o)
        else:
            fn(n, g.row_ptr, g.col, sigmas, tie_mode=tie, **o)
        torch.cuda.synchronize()
        took = (free0 - torch.cuda.mem_get_info()[0], qc.debug_alloc_fault(0) - blocks0,
                torch.cuda.memory_allocated() - torch0)
        outs.append(({k: (t.cpu().numpy() if t is not None else None) for k, t in o.items()}, took))
    check_equal(outs[0][0], outs[1][0])   # qc_cluster
    return outs[0], outs[2]


def check_equal(a, b):
    np.testing.assert_array_equal(b["labels"], a["labels"])
    np.testing.assert_allclose(b["psi"], a["psi"], rtol=1e-6, atol=0)
    np.testing.assert_allclose(b["v"], a["v"], rtol=1e-6, atol=0)
    np.testing.assert_array_equal(b["psi"], a["psi"])
    np.testing.assert_array_equal(b["v"], a["v"])
    if a["dist"] is not None:
        np.testing.assert_array_equal(b["dist"], a["dist"])


def test_noalloc_matches_cluster_on_consecutive_calls(env):
    torch, qc = env
    # larger first (the library carves the 2,708-node matrix itself), then a
    # smaller graph into caller-provided outputs, then a third graph again
    # with the matrix in the scratch: every call finds the previous call's
    # contents in the scratch
    cases = [(gg.config2(), gg.SIGMAS_C2, False, 0),
             (gg.config1(), [1.0], True, 0),
             (gg.barbell_graph(6), [0.5, 1.0, 2.0], False, 1)]
    for i, (g, sig, with_dist, tie) in enumerate(cases):
        (ref, _), (got, took) = run_both(torch, qc, g, sig, with_dist, tie)
        check_equal(ref, got)
        if i > 0:
            # the scratch already exists: the call takes no device memory
            assert took == (0, 0, 0), took
        # and the labels are the oracle's
        res = oracle.cluster(g.n, g.row_ptr, g.col, sig, tie_mode=tie, with_dist=with_dist)
        for k in range(len(sig)):
            np.testing.assert_array_equal(got["labels"][k], res["per_sigma"][k]["labels"])
        if with_dist:
            np.testing.assert_array_equal(got["dist"], res["dist"])


def test_noalloc_refuses_a_problem_beyond_its_scratch(env):
    torch, qc = env
    # a star of 8,200 nodes: the 67 MB matrix alone exceeds the 64 MiB scratch
    # when the library must hold it, and the problem fits once the caller
    # provides the matrix
    g = gg.star_graph(8199)
    assert g.n * g.n > qc.NOALLOC_SCRATCH_BYTES
    labels = torch.full((1, g.n), -7, dtype=torch.int32, device="cuda")
    print(f"[gpu] cluster_noalloc n={g.n} without dist: refused", flush=True)
    with pytest.raises(qc.QCError) as e:
        qc.cluster_noalloc(g.n, g.row_ptr, g.col, [0.5], labels=labels)
    assert e.value.status == qc.QC_E_TOO_LARGE
    torch.cuda.synchronize()
    assert (labels.cpu().numpy() == -7).all()   # nothing written
    (ref, _), (got, _) = run_both(torch, qc, g, [0.5], True)
    check_equal(ref, got)
    # qc_cluster takes the same problem on buffers of its own
    lab = qc.cluster(g.n, g.row_ptr, g.col, [0.5])
    torch.cuda.synchronize()
    np.testing.assert_array_equal(lab.cpu().numpy(), got["labels"])
