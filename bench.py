#!/usr/bin/env python3
"""Benchmark of the graph Quantum Clustering hot path on one MI355X.

Workload (default): the batched sigma sweep — 64 seeded degree-corrected SBM
graphs, N log-uniform in [1,000, 20,000], 32 widths sigma log-spaced in
[0.25, 8]. One step runs every stage for every (graph, sigma): multi-source
BFS distances (int8 N x N per graph, resident in HBM), distance histograms,
psi/V, Graph Gradient Descent parents (FP64 re-check of near ties) and
pointer jumping to labels. Inputs (CSR) are resident before timing starts.

Metric: pair-terms per second, a pair-term being one (i, j, sigma) term of the
potential sum (sum over graphs of N^2 times the number of sigmas), for the
batched form replayed as one HIP graph. Also reported: graphs/s, the plain
per-graph path on the same GPU, per-stage kernel times, the roofline of the
dominant kernel and the CPU oracle on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def bfs_bytes(g) -> float:
    """Algorithmic bytes of one graph's distance computation: the N^2 int8
    matrix written once plus the CSR read once (4(N+1) + 4 nnz)."""
    return float(g.n) * g.n + 4.0 * (g.n + 1) + 4.0 * g.nnz


def cpu_baseline(graphs, sigmas, budget_s: float) -> dict:
    """The oracle (as it stands) on the first graphs of the workload, in order
    of increasing size, until about `budget_s` seconds of CPU work."""
    import oracle
    order = sorted(range(len(graphs)), key=lambda i: graphs[i].n)
    done, terms, t_total = [], 0.0, 0.0
    for i in order:
        g = graphs[i]
        t0 = time.perf_counter()
        dist, dmax = oracle.distances(g.n, g.row_ptr, g.col)
        hist = oracle.hist_rows(dist, dmax + 1)
        for s in sigmas:
            _, v = oracle.potential_canonical(hist, s)
            oracle.find_centers(oracle.ggd_parent(g.n, g.row_ptr, g.col, v, 0))
        t_total += time.perf_counter() - t0
        terms += float(g.n) ** 2 * len(sigmas)
        done.append(g.n)
        if t_total >= budget_s:
            break
    return {
        "value": terms / t_total, "unit": "pair-terms/s", "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": (f"{len(done)} smallest of the {len(graphs)} graphs (N={min(done)}..{max(done)}), "
                   f"all {len(sigmas)} sigmas: BFS distances, histograms, canonical FP64 psi/V, "
                   f"descent labels; {t_total:.1f} s"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget-s", type=float, default=15.0)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_2305_14641_amd import graphgen as gg
    from paper_2305_14641_amd import qc

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()

    t0 = time.perf_counter()
    graphs = gg.config4()
    sigmas = gg.sigmas_c4()
    S = len(sigmas)
    log(f"generated {len(graphs)} graphs in {time.perf_counter() - t0:.1f}s")

    handles = [qc.Graph.from_graph(g) for g in graphs]
    batch = qc.Batch(handles, sigmas, tie_mode=qc.TIE_STRICT, hipgraph=True)
    psi, v, lab = batch.outputs()
    pair_terms = float(sum(float(g.n) ** 2 for g in graphs)) * S
    log(f"planned batch: total nodes {batch.total}, pair-terms/step {pair_terms:.3e}")

    if args.copy_probe_mib:
        nb = args.copy_probe_mib << 20
        a = torch.empty(nb, dtype=torch.uint8, device="cuda")
        b = torch.empty(nb, dtype=torch.uint8, device="cuda")
        a.fill_(1)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy probe: {nb} bytes read and written")
        del a, b

    # -- batched form, replayed as a HIP graph --------------------------------
    for _ in range(args.warmup):
        batch.run(psi, v, lab)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch.run(psi, v, lab)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    log(f"batched: {dt * 1e3:.2f} ms/step")
    rechecks = batch.recheck_count()

    # -- per-kernel device time: the same launches, not captured, with events --
    batch_nograph = qc.Batch(handles, sigmas, tie_mode=qc.TIE_STRICT, hipgraph=False)
    batch_nograph.run(psi, v, lab)
    torch.cuda.synchronize()
    qc.timing_enable(True)
    for _ in range(args.steps):
        batch_nograph.run(psi, v, lab)
    torch.cuda.synchronize()
    stages = {}
    for st_id, name in enumerate(qc.STAGE_NAMES):
        ms, cnt = qc.timing_read(st_id)
        stages[name] = {"ms_per_step": ms / args.steps, "launches_per_step": cnt / args.steps,
                        "avg_launch_ms": (ms / cnt) if cnt else None}
    qc.timing_enable(False)
    dom = max(stages, key=lambda k: stages[k]["ms_per_step"])
    bfs_ms = stages["bfs"]["ms_per_step"]
    bfs_launches = stages["bfs"]["launches_per_step"]
    bytes_step = sum(bfs_bytes(g) for g in graphs)
    achieved = (bytes_step / bfs_launches) / (stages["bfs"]["avg_launch_ms"] * 1e-3) / 1e9
    hist_bytes = sum(float(g.n) * g.n + 4.0 * g.n * 32 for g in graphs)
    hist_gbs = hist_bytes / (stages["hist"]["ms_per_step"] * 1e-3) / 1e9
    log(f"stages: " + ", ".join(f"{k}={v_['ms_per_step']:.3f}ms" for k, v_ in stages.items()))

    # -- plain per-graph path (one graph at a time, synchronous); its first
    # pass also checks that the batched outputs are bitwise the plain ones.
    plain = None
    if not args.no_plain:
        out_lab = torch.empty((S, max(g.n for g in graphs)), dtype=torch.int32, device="cuda")

        def plain_step(check=False):
            for i, (g, G) in enumerate(zip(graphs, handles)):
                G.distances()
                p_, v_ = G.potential(sigmas)
                for s in range(S):
                    G.labels(s, qc.TIE_STRICT, out=out_lab[s, :g.n])
                torch.cuda.synchronize()
                if check:
                    o = batch.offsets[i]
                    assert torch.equal(out_lab[:, :g.n], lab[:, o:o + g.n]), "plain != batched labels"
                    assert torch.equal(v_, v[:, o:o + g.n]), "plain != batched V"
                    assert torch.equal(p_, psi[:, o:o + g.n]), "plain != batched psi"

        plain_step(check=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.plain_steps):
            plain_step()
        torch.cuda.synchronize()
        pdt = (time.perf_counter() - t0) / args.plain_steps
        plain = {"ms_per_step": pdt * 1e3, "pair_terms_per_s": pair_terms / pdt,
                 "graphs_per_s": len(graphs) / pdt, "batched_speedup": pdt / dt,
                 "bitwise_equal_to_batched": True}
        log(f"plain: {pdt * 1e3:.2f} ms/step")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(graphs, sigmas, args.cpu_budget_s)
        log(f"cpu oracle: {cpu['value']:.3e} pair-terms/s on {cpu['cores']} threads")

    result = {
        "metric": "pair-terms/sec for psi/V (+ graphs/sec); batched vs plain at 1e-6",
        "value": pair_terms / dt,
        "unit": "pair-terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8 distances, fp64 accumulation, fp32 psi/V",
        "data": "synthetic: seeded degree-corrected SBM graphs",
        "config": {
            "workload": "batched sigma sweep: 64 DC-SBM graphs (seeds 100-163), N log-uniform "
                        "[1e3, 2e4], 2-16 blocks, mean degree 3-8; 32 sigmas geomspace(0.25, 8); "
                        "one HIP-graph replay per step",
            "graphs": len(graphs), "total_nodes": int(batch.total),
            "sum_n2": float(sum(float(g.n) ** 2 for g in graphs)), "n_sigmas": S,
            "tie_mode": "strict", "parallelism": "single GPU",
        },
        "graphs_per_s": len(graphs) / dt,
        "fp64_rechecks_per_step": rechecks,
        "stages": stages,
        "dominant_kernel": dom,
        "roofline": {
            "bound": "hbm", "kernel": "k_bfs",
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "algorithmic_bytes_per_launch": bytes_step / bfs_launches,
        },
        "hist_kernel_gbs": hist_gbs,
        "plain": plain,
        "cpu_baseline": cpu,
    }
    print(json.dumps(result))


if __name__ == "__main__":
    main()
