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
batched form replayed as one HIP graph (the stages after the search of each
search launch's graphs run on a second stream beside the next searches).
Also reported: graphs/s, the plain per-graph path on the same GPU, per-stage
kernel times (from a pass with every stage in stream order), the search's edge
visits and LDS bytes gathered, the roofline of the dominant kernel, the
smaller workloads (one 200-node graph's latency, the 2,708- and 19,717-node
graphs end to end, psi/V from a resident matrix), the serving form on the
whole 1,024-request stream (p50/p99 latency and graphs/s at several arrival
rates, against one request at a time), the fully connected dense workload,
real edge weights (shortest paths and the whole path on the 2,708- and
19,717-node graphs), and the CPU oracle on bounded samples (every core and one thread), whose
labels are compared with the GPU's.

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
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12  # vector lane-operations/s: 256 CUs x 64 lanes x 2.4 GHz
LDS_PEAK_TBS = 256 * 128 * 2.4e9 / 1e12   # LDS bytes/s: 256 CUs x 128 bytes per clock x 2.4 GHz
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix-core peak


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def bfs_bytes(g) -> float:
    """Algorithmic bytes of one graph's distance computation: the N^2 int8
    matrix written once plus the CSR read once (4(N+1) + 4 nnz)."""
    return float(g.n) * g.n + 4.0 * (g.n + 1) + 4.0 * g.nnz


PROFILE = os.path.join(ROOT, "profiles", "bench_c4_kernels_and_traffic.json")


def profiled_bfs():
    """The k_bfs entry of the committed counter summary, or None when it is
    missing or a kernel source changed since it was taken."""
    import hashlib
    if not os.path.exists(PROFILE):
        return None
    prof = json.load(open(PROFILE))
    for rel, digest in prof.get("kernel_sources_sha256", {}).items():
        path = os.path.join(ROOT, rel)
        if not os.path.exists(path) or hashlib.sha256(open(path, "rb").read()).hexdigest() != digest:
            return None
    return prof.get("k_bfs_tuned")


def profiled_traffic(launches_per_step):
    """HBM bytes per k_bfs launch measured by rocprofv3 FETCH_SIZE / WRITE_SIZE
    (scaled by a copy-kernel calibration) for the kernel sources as they are
    now: the profiled batched step's BFS bytes over this run's BFS launches per
    step (the autotuner's grouping can differ between runs); None when no such
    profile exists or a kernel source changed since."""
    prof = profiled_bfs()
    if not prof or not prof.get("hbm_bytes_per_step"):
        return None
    return prof["hbm_bytes_per_step"] / launches_per_step


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(graphs, sigmas, budget_s: float, gpu_labels=None, offsets=None,
                 threads=None) -> dict:
    """The oracle (as it stands) on the first graphs of the workload, in order
    of increasing size, until about `budget_s` seconds of CPU work, on
    `threads` threads (default: every core). When the GPU's labels of the
    same graphs are given, the oracle's labels are compared with them (after
    the timed work of each graph)."""
    import oracle
    before = oracle.num_threads()
    if threads:
        oracle.set_num_threads(threads)
    try:
        order = sorted(range(len(graphs)), key=lambda i: graphs[i].n)
        done, terms, t_total = [], 0.0, 0.0
        mismatches = 0
        for i in order:
            g = graphs[i]
            t0 = time.perf_counter()
            dist, dmax = oracle.distances(g.n, g.row_ptr, g.col)
            hist = oracle.hist_rows(dist, dmax + 1)
            labels = []
            for s in sigmas:
                _, v = oracle.potential_canonical(hist, s)
                labels.append(oracle.find_centers(oracle.ggd_parent(g.n, g.row_ptr, g.col, v, 0)))
            t_total += time.perf_counter() - t0
            if gpu_labels is not None:
                got = gpu_labels[:, offsets[i]:offsets[i + 1]]
                mismatches += int((got != np.stack(labels)).sum())
            terms += float(g.n) ** 2 * len(sigmas)
            done.append(g.n)
            if t_total >= budget_s:
                break
        cores = oracle.num_threads()
    finally:
        if threads:
            oracle.set_num_threads(before)
    out = {
        "value": terms / t_total, "unit": "pair-terms/s", "cores": cores,
        "kind": "oracle",
        "sample": (f"{len(done)} smallest of the {len(graphs)} graphs (N={min(done)}..{max(done)}), "
                   f"all {len(sigmas)} sigmas: BFS distances, histograms, canonical FP64 psi/V, "
                   f"descent labels; {t_total:.1f} s"),
        "cpu_model": cpu_model(),
    }
    if gpu_labels is not None:
        out["parity_ok"] = mismatches == 0
        out["labels_compared"] = int(sum(done) * len(sigmas))
        out["label_mismatches"] = mismatches
    return out


def _gen_request(r):
    from paper_2305_14641_amd import graphgen as gg
    g, sig = gg.config5_graph(r)
    return g.n, g.row_ptr, g.col, sig


def gen_requests(count: int) -> list:
    """The serving stream's requests, drawn in worker processes. Called before
    anything touches the GPU, so no process that has initialised it forks."""
    import concurrent.futures as cf
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 4)) as ex:
        reqs = list(ex.map(_gen_request, range(count), chunksize=4))
    log(f"generated {len(reqs)} requests in {time.perf_counter() - t0:.1f}s "
        f"(N {min(r[0] for r in reqs)}..{max(r[0] for r in reqs)})")
    return reqs


def serve(args, reqs):
    """Serving form on the request stream: open-loop Poisson arrivals, p50/p99
    latency (scheduled arrival -> labels on the host), graphs/s, and the same
    requests run one at a time."""
    import threading
    from paper_2305_14641_amd import graphgen as gg
    from paper_2305_14641_amd import qc

    budget = int(args.serve_budget_gib * (1 << 30))
    # the plain path: one request at a time through the same server (1 slot)
    srv1 = qc.Server(max_slots=1, hbm_budget_bytes=budget)
    rid = srv1.submit(*reqs[0][:3], reqs[0][3])
    srv1.wait(rid)                                   # warm-up
    t0 = time.perf_counter()
    for r in reqs:
        srv1.wait(srv1.submit(r[0], r[1], r[2], r[3]))
    plain_s = time.perf_counter() - t0
    srv1.close()
    log(f"serving, one request at a time: {len(reqs) / plain_s:.1f} graphs/s")
    results = {"requests": len(reqs), "slots": args.serve_slots,
               "budget_gib": args.serve_budget_gib,
               "sum_n2": float(sum(float(r[0]) ** 2 for r in reqs)),
               "plain_graphs_per_s": len(reqs) / plain_s, "rates": []}
    for rate in args.serve_rates:
        arrivals = gg.poisson_arrivals(len(reqs), rate, seed=77)
        srv = qc.Server(max_slots=args.serve_slots, hbm_budget_bytes=budget)
        ids = [None] * len(reqs)
        lat = [None] * len(reqs)
        start = time.perf_counter() + 0.05

        def submitter():
            for k, r in enumerate(reqs):
                delay = start + arrivals[k] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                ids[k] = srv.submit(r[0], r[1], r[2], r[3])

        th = threading.Thread(target=submitter)
        th.start()
        for k in range(len(reqs)):
            while ids[k] is None:
                time.sleep(0.0005)
            _, _, _, info = srv.wait(ids[k])
            lat[k] = info["t_done"] - (start + arrivals[k])
        th.join()
        end = time.perf_counter()
        stats = srv.stats()
        srv.close()
        lat_ms = np.sort(np.array(lat) * 1e3)
        entry = {"rate_per_s": rate, "p50_ms": float(np.percentile(lat_ms, 50)),
                 "p99_ms": float(np.percentile(lat_ms, 99)),
                 "graphs_per_s": len(reqs) / (end - start),
                 "vs_plain": (len(reqs) / (end - start)) / results["plain_graphs_per_s"], **stats}
        results["rates"].append(entry)
        log(f"rate {rate}/s: p50 {entry['p50_ms']:.1f} ms, p99 {entry['p99_ms']:.1f} ms, "
            f"{entry['graphs_per_s']:.1f} graphs/s, peak in flight {stats['peak_requests_in_flight']}")
    return results


def configs_leg(args, qc, gg, torch) -> dict:
    """The smaller workloads, each on its own: the 200-node graph's latency per
    call, the 2,708-node (4 sigmas) and 19,717-node (sigma 2) graphs end to
    end on the plain path, and psi/V from the 19,717-node graph's resident
    distance matrix (the histogram pass plus the potential kernel)."""
    out = {}

    def path(G, sigmas, dist=None):
        G.distances(dist)
        G.potential(sigmas)
        for s in range(len(sigmas)):
            G.labels(s, qc.TIE_STRICT)
        G.sync()

    # 200 nodes: one call of Algorithm 4 from host CSR (temporary handle), and
    # the same on a resident handle
    # (and through qc_cluster_noalloc, whose buffers come from the library's
    # fixed scratch instead of device allocations, into preallocated labels)
    g1 = gg.config1()
    lat_call, lat_res, lat_na = [], [], []
    G1 = qc.Graph.from_graph(g1)
    lab1 = torch.empty((len(gg.SIGMAS_C1), g1.n), dtype=torch.int32, device="cuda")
    for k in range(60):
        t0 = time.perf_counter()
        qc.cluster(g1.n, g1.row_ptr, g1.col, gg.SIGMAS_C1, qc.TIE_STRICT)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        path(G1, gg.SIGMAS_C1)
        t2 = time.perf_counter()
        qc.cluster_noalloc(g1.n, g1.row_ptr, g1.col, gg.SIGMAS_C1, qc.TIE_STRICT, labels=lab1)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        if k >= 10:
            lat_call.append((t1 - t0) * 1e3)
            lat_res.append((t2 - t1) * 1e3)
            lat_na.append((t3 - t2) * 1e3)
    G1.close()
    out["c1"] = {"workload": "SBM N=200, 4 blocks, sigma 1",
                 "call_from_host_csr_ms": {"p50": float(np.percentile(lat_call, 50)),
                                           "p99": float(np.percentile(lat_call, 99))},
                 "call_from_host_csr_noalloc_ms": {"p50": float(np.percentile(lat_na, 50)),
                                                   "p99": float(np.percentile(lat_na, 99))},
                 "resident_graph_ms": {"p50": float(np.percentile(lat_res, 50)),
                                       "p99": float(np.percentile(lat_res, 99))}}
    log(f"config 1 latency: {out['c1']['call_from_host_csr_ms']['p50']:.3f} ms per call, "
        f"{out['c1']['call_from_host_csr_noalloc_ms']['p50']:.3f} ms without allocation, "
        f"{out['c1']['resident_graph_ms']['p50']:.3f} ms on a resident graph")
    for key, g, sigmas in (("c2", gg.config2(), gg.SIGMAS_C2), ("c3", gg.config3(), gg.SIGMAS_C3)):
        G = qc.Graph.from_graph(g)
        dist = None   # the handle's own resident matrix (rows on 128-byte lines)
        for _ in range(2):
            path(G, sigmas, dist)        # the first run learns dmax and re-plans
        ts = []
        for _ in range(max(args.steps, 5)):
            t0 = time.perf_counter()
            path(G, sigmas, dist)
            ts.append((time.perf_counter() - t0) * 1e3)
        ms = float(np.median(ts))
        terms = float(g.n) ** 2 * len(sigmas)
        out[key] = {"workload": f"DC-SBM N={g.n}, {len(sigmas)} sigma(s)", "end_to_end_ms": ms,
                    "pair_terms_per_s": terms / (ms * 1e-3), "graphs_per_s": 1e3 / ms}
        if key == "c3":
            # psi/V from the resident matrix: the histogram pass over it and
            # the potential kernel, device times from the stage events
            qc.timing_enable(True)
            reps = max(args.steps, 5)
            for _ in range(reps):
                G.distances(dist)
                G.potential(sigmas)
            torch.cuda.synchronize()
            h_ms, _ = qc.timing_read(qc.STAGE_HIST)
            p_ms, _ = qc.timing_read(qc.STAGE_POTENTIAL)
            qc.timing_enable(False)
            t = (h_ms + p_ms) / reps
            out[key]["potential_from_resident_matrix"] = {
                "hist_ms": h_ms / reps, "potential_ms": p_ms / reps, "ms": t,
                "pair_terms_per_s": terms / (t * 1e-3),
                "hbm_gbs": (float(g.n) ** 2 + 8.0 * g.n * 32 + 8.0 * g.n * len(sigmas)) / (t * 1e-3) / 1e9}
        log(f"{key}: {ms:.3f} ms end to end, {terms / (ms * 1e-3):.3e} pair-terms/s")
        del dist
        G.close()
    return out


def quality_sweep(qc, gg, torch) -> dict:
    """Section 4.2's measures of the GPU labels against the planted blocks of
    the 64 sweep graphs, for each of the 32 widths (a synthetic analogue of
    the paper's sensitivity study), as means and spreads over the graphs."""
    from paper_2305_14641_amd import quality
    graphs = gg.config4()
    sigmas = gg.sigmas_c4()
    handles = [qc.Graph.from_graph(g) for g in graphs]
    b = qc.Batch(handles, sigmas, tie_mode=qc.TIE_STRICT, hipgraph=False)
    psi, v, lab = b.outputs()
    b.run(psi, v, lab)
    torch.cuda.synchronize()
    lab = lab.cpu().numpy()
    rows = []
    for s, sigma in enumerate(sigmas):
        per = []
        for i, g in enumerate(graphs):
            o0, o1 = b.offsets[i], b.offsets[i + 1]
            per.append(quality.scores(g.row_ptr, g.col, g.blocks, lab[s, o0:o1]))
        keys = ["modularity", "nmi", "ari", "fmi"]
        row = {"sigma": sigma}
        for k in keys:
            vals = np.array([p_[k] for p_ in per])
            row[k] = float(vals.mean())
            row[k + "_std"] = float(vals.std())
        cl = np.array([p_["clusters"] / g.n for p_, g in zip(per, graphs)])
        row["clusters_per_node"] = float(cl.mean())
        rows.append(row)
        log(f"sigma {sigma:6.3f}: Q {row['modularity']:.3f} NMI {row['nmi']:.3f} "
            f"ARI {row['ari']:.3f} FMI {row['fmi']:.3f} clusters/node {row['clusters_per_node']:.4f}")
    b.close()
    return {"metric": "clustering quality vs planted blocks across the sigma sweep",
            "config": {"workload": "64 DC-SBM graphs (seeds 100-163), 32 sigmas geomspace(0.25, 8), "
                                   "strict ties; GPU labels"},
            "rows": rows}


DENSE_PROFILE = os.path.join(ROOT, "profiles", "k_dense_fully_connected_n20000.json")


def dense_profile(kernel: str):
    """Counter figures per launch of one dense-kernel instance from the
    committed summary, while the kernel source is unchanged since then."""
    import hashlib
    try:
        prof = json.load(open(DENSE_PROFILE))
        src = os.path.join(ROOT, "paper_2305_14641_amd", "csrc", "qc_dense.hip")
        if hashlib.sha256(open(src, "rb").read()).hexdigest() != prof["kernel_source_sha256"]:
            return None
        return prof["kernels"][kernel]
    except (OSError, KeyError, ValueError):
        return None


def bfs_alu(stages):
    """Vector-ALU view of k_bfs: VALU lane-operations per second (counted
    wavefront instructions x 64 lanes, from the committed counter summary)
    against the issue rate of 256 CUs x 64 lanes x 2.4 GHz."""
    prof = profiled_bfs()
    if not prof or not prof.get("valu_wave_instructions_per_step"):
        return None
    ops = prof["valu_wave_instructions_per_step"] * 64 / (stages["bfs"]["ms_per_step"] * 1e-3) / 1e12
    return {"bound": "alu", "kernel": "k_bfs", "achieved": ops, "peak": VALU_PEAK_TOPS,
            "unit": "T VALU lane-ops/s", "frac": ops / VALU_PEAK_TOPS,
            "valu_wave_instructions_per_step": prof["valu_wave_instructions_per_step"],
            "lds_wave_instructions_per_step": prof.get("lds_wave_instructions_per_step")}


def real_leg(args, qc, torch) -> dict:
    """Shortest paths under real edge weights (qc_distances_real: one
    workgroup per source, binary32 path sums) and the whole real-weighted
    path (qc_cluster_real) on the 2,708- and 19,717-node graphs with seeded
    uniform weights in [0.5, 4). Kernel times from the library's stage
    events; call times include the CSR upload and the final wait."""
    from paper_2305_14641_amd import graphgen as gg
    out = {"workload": "config-2 and config-3 graphs, edge weights uniform in [0.5, 4) (seeded)"}
    for name, g, S in (("c2", gg.config2(), 4), ("c3", gg.config3(), 1)):
        w = gg.real_edge_weights(g, seed=5)
        n = g.n
        d = torch.empty((n, n), dtype=torch.float32, device="cuda")
        qc.distances_real(n, g.row_ptr, g.col, w, out=d)
        torch.cuda.synchronize()
        reps = 3
        qc.timing_enable(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            qc.distances_real(n, g.row_ptr, g.col, w, out=d)
        call_ms = (time.perf_counter() - t0) / reps * 1e3
        k_ms, k_n = qc.timing_read(qc.STAGE_SSSP)
        qc.timing_enable(False)
        k_ms /= max(k_n, 1)
        sig = list(np.geomspace(0.5, 4.0, S)) if S > 1 else [1.0]
        lab = torch.empty((S, n), dtype=torch.int32, device="cuda")
        qc.cluster_real(n, g.row_ptr, g.col, w, sig, dist=d, labels=lab)
        t0 = time.perf_counter()
        for _ in range(reps):
            qc.cluster_real(n, g.row_ptr, g.col, w, sig, dist=d, labels=lab)
        cl_ms = (time.perf_counter() - t0) / reps * 1e3
        out[name] = {"n": n, "nnz": g.nnz, "sssp_kernel_ms": k_ms, "distances_call_ms": call_ms,
                     "sources_per_s": n / (k_ms * 1e-3),
                     "pair_lengths_per_s": float(n) * n / (k_ms * 1e-3),
                     "output_gbs": 4.0 * n * n / (k_ms * 1e-3) / 1e9,
                     "cluster_call_ms": cl_ms, "n_sigmas": S,
                     "pair_terms_per_s_end_to_end": float(n) * n * S / (cl_ms * 1e-3)}
        log(f"real {name}: sssp {k_ms:.2f} ms ({n / (k_ms * 1e-3):.3e} sources/s), "
            f"distances call {call_ms:.2f} ms, cluster ({S} sigma) {cl_ms:.2f} ms")
        if name == "c3" and not args.no_cpu_baseline:
            import oracle
            src = np.arange(0, n, max(1, n // 256), dtype=np.int32)[:256]
            t0 = time.perf_counter()
            oracle.real_rows(n, g.row_ptr, g.col, w, src)
            dt = time.perf_counter() - t0
            out[name]["cpu_oracle"] = {"sources_per_s": src.shape[0] / dt,
                                       "cores": oracle.num_threads(),
                                       "sample": f"{src.shape[0]} sources, binary32 Dijkstra"}
        del d, lab
    torch.cuda.empty_cache()
    return out


def dense_leg(args, qc, torch) -> dict:
    """Algorithm 1 on a fully connected graph with float distances (the
    paper's GPU experiment shape): one pass for one width (HBM-bound) and for
    eight widths (ALU-bound), timed with HIP events on the launch stream."""
    from paper_2305_14641_amd import graphgen as gg
    n = args.dense_n
    t0 = time.perf_counter()
    d = torch.as_tensor(gg.dense_points(n, dim=16, clusters=8, seed=3)).cuda()
    log(f"dense: generated {n} x {n} matrix in {time.perf_counter() - t0:.1f}s")
    out = {"workload": f"fully connected: {n} points of an 8-cluster Gaussian mixture in 16-D, "
                       "Euclidean float32 distances", "n": n}
    for S in (1, 8):
        sig = list(np.geomspace(0.5, 8.0, S)) if S > 1 else [2.0]
        psi = torch.empty((S, n), dtype=torch.float64, device="cuda")
        v = torch.empty_like(psi)
        for _ in range(2):
            qc.potential_dense(d, sig, psi=psi, v=v)
        torch.cuda.synchronize()
        # back-to-back launches on the current stream (the launch stream),
        # bracketed by one pair of HIP events
        reps = max(args.steps, 3)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            qc.potential_dense(d, sig, psi=psi, v=v)
        e1.record()
        torch.cuda.synchronize()
        per = e0.elapsed_time(e1) / reps
        launches = (S + 7) // 8
        terms = float(n) * n * S
        alg = 4.0 * n * n * launches
        gbs = alg / (per * 1e-3) / 1e9
        prof = dense_profile(f"k_dense<{min(S, 8)}, true>")
        traffic = (prof["hbm_read_bytes_per_launch"] + prof["hbm_write_bytes_per_launch"]) if prof else None
        hbm = {"bound": "hbm", "kernel": f"k_dense<{min(S, 8)}>", "achieved": gbs,
               "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "traffic": traffic,
               "algorithmic_bytes_per_launch": 4.0 * n * n}
        alu = None
        if prof:
            # VALU lane-operations per second against the vector issue rate
            # (256 CUs x 64 lanes x 2.4 GHz, no packed math)
            ops = prof["valu_wave_instructions_per_launch"] * 64 * launches / (per * 1e-3) / 1e12
            alu = {"bound": "alu", "kernel": f"k_dense<{min(S, 8)}>", "achieved": ops,
                   "peak": VALU_PEAK_TOPS, "unit": "T VALU lane-ops/s", "frac": ops / VALU_PEAK_TOPS,
                   "valu_wave_instructions_per_launch": prof["valu_wave_instructions_per_launch"]}
        out[f"s{S}"] = {"ms": per, "launches": launches, "pair_terms_per_s": terms / (per * 1e-3),
                        "roofline": hbm if S == 1 else (alu or hbm), "other_bound": alu if S == 1 else hbm}
        log(f"dense S={S}: {per:.3f} ms, {terms / (per * 1e-3):.3e} pair-terms/s, {gbs:.0f} GB/s")
        del psi, v
    if not args.no_cpu_baseline:
        import oracle
        rows = d[:256].cpu().numpy()
        t0 = time.perf_counter()
        oracle.potential_dense(rows, 2.0)
        dt = time.perf_counter() - t0
        out["cpu_oracle"] = {"pair_terms_per_s": rows.size / dt, "cores": oracle.num_threads(),
                             "sample": "first 256 rows, one width"}
    del d
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget-s", type=float, default=15.0)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the planner's BFS launch shapes (no timing at set-up)")
    ap.add_argument("--no-dense", action="store_true",
                    help="skip the fully connected (dense float distance) leg")
    ap.add_argument("--dense-n", type=int, default=20000)
    ap.add_argument("--no-real", action="store_true",
                    help="skip the real edge weight leg (shortest paths, whole path)")
    ap.add_argument("--quality", action="store_true",
                    help="sigma-sweep quality study: label quality vs the planted blocks")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    ap.add_argument("--serve-requests", type=int, default=1024,
                    help="requests of the serving stream the serving leg runs (0: no serving leg)")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving leg and print its result")
    ap.add_argument("--serve-rates", type=float, nargs="+", default=[10, 50, 200, 500])
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the smaller workloads (latency, end to end, resident matrix)")
    ap.add_argument("--cpu-1t-budget-s", type=float, default=6.0)
    ap.add_argument("--no-bf16", action="store_true",
                    help="skip the BF16 matrix-core sweep variant")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU: --gpus must be 1"}))
        sys.exit(2)
    # the serving stream is drawn in worker processes before anything
    # touches the GPU
    reqs = gen_requests(args.serve_requests) if args.serve_requests > 0 and not args.quality else None
    if args.serve_only:
        import torch
        torch.cuda.set_device(0)
        res = serve(args, reqs)
        print(json.dumps({"metric": "serving: p50/p99 latency and graphs/s on the request stream",
                          "config": {"workload": "serving: Poisson stream of DC-SBM clustering "
                                                 "requests, N log-uniform [500, 5e4], 1-8 sigmas"},
                          **res}))
        return

    import torch
    from paper_2305_14641_amd import graphgen as gg
    from paper_2305_14641_amd import qc

    assert torch.cuda.is_available(), "bench needs a GPU"
    if args.quality:
        print(json.dumps(quality_sweep(qc, gg, torch)))
        return
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()

    t0 = time.perf_counter()
    graphs = gg.config4()
    sigmas = gg.sigmas_c4()
    S = len(sigmas)
    log(f"generated {len(graphs)} graphs in {time.perf_counter() - t0:.1f}s")

    handles = [qc.Graph.from_graph(g) for g in graphs]
    for G in handles:
        G.distances()       # learns dmax: the planner's final choice
    planned = [G.bfs_plan() for G in handles]
    t0 = time.perf_counter()
    batch = qc.Batch(handles, sigmas, tie_mode=qc.TIE_STRICT, hipgraph=True,
                     autotune=not args.no_autotune)
    tuned = [G.bfs_plan() for G in handles]
    log(f"batch set-up {time.perf_counter() - t0:.2f}s; autotuner changed the BFS plan of "
        f"{sum(a != b for a, b in zip(planned, tuned))} of {len(handles)} graphs")
    from collections import Counter
    log("BFS plans (batch width, words, planes, shape): "
        + ", ".join(f"{k}x{c}" for k, c in sorted(Counter(tuned).items())))
    stage_tiles = batch.stage_tiles()
    log(f"stage tiles: {stage_tiles}")
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
    edge_visits, lds_gathered = batch.search_stats()
    lab_host = lab.cpu().numpy()

    # -- per-kernel device time: the same launches, not captured, with events,
    #    every stage in stream order (the timed steps above run the stages
    #    after the search beside the searches, where a kernel's duration
    #    would include the GPU it shares) --
    batch_nograph = qc.Batch(handles, sigmas, tie_mode=qc.TIE_STRICT, hipgraph=False, serial=True)
    batch_nograph.run(psi, v, lab)
    torch.cuda.synchronize()
    qc.timing_enable(True)
    for _ in range(args.steps):
        batch_nograph.run(psi, v, lab)
    torch.cuda.synchronize()
    stages = {}
    for st_id, name in enumerate(qc.STAGE_NAMES[:qc.STAGE_DENSE]):
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
    # (zero when every graph's search makes its histograms itself)
    hist_ms = stages["hist"]["ms_per_step"]
    hist_gbs = hist_bytes / (hist_ms * 1e-3) / 1e9 if hist_ms > 0 else None
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

    # -- BF16 matrix-core sweep variant over the whole batch: time, matrix-core
    #    rate and error against the FP64-accumulated values ---------------------
    bf16 = None
    if not args.no_bf16:
        pb, vb = batch.sweep_bf16()
        torch.cuda.synchronize()
        reps = 10
        qc.timing_enable(True)
        for _ in range(reps):
            batch.sweep_bf16(pb, vb)
        torch.cuda.synchronize()
        ms, cnt = qc.timing_read(qc.STAGE_POTENTIAL)
        qc.timing_enable(False)
        ms, cnt = ms / reps, cnt / reps
        # psi/V of the batched run are within 1e-6 of FP64, far below the BF16 error
        pr, vr = psi.double(), v.double()
        worst_psi = float(((pb.double() - pr).abs() / pr.abs()).max())
        nz = vr != 0
        worst_v = float(((vb.double() - vr).abs()[nz] / vr.abs()[nz]).max())
        # one 16x16x32 MFMA (16,384 flops) per 16-node tile, 16 weight columns
        # (8 sigmas x {psi, numerator}) and 32 histogram bins
        col_blocks = -(-2 * S // 16)
        flops = float(sum(-(-g.n // 16) * col_blocks * (G.histograms_k() // 32) * 16384
                          for g, G in zip(graphs, handles)))
        bf16 = {"potential_ms_per_step": ms, "launches_per_step": cnt,
                "fp64_potential_ms_per_step": stages["potential"]["ms_per_step"],
                "speedup_vs_fp64_potential": stages["potential"]["ms_per_step"] / ms,
                "mfma_flops_per_step": flops,
                "mfma_tflops": flops / (ms * 1e-3) / 1e12, "mfma_peak_tflops": BF16_PEAK_TFLOPS,
                "mfma_frac": flops / (ms * 1e-3) / 1e12 / BF16_PEAK_TFLOPS,
                "max_rel_err_psi": worst_psi, "max_rel_err_v": worst_v}
        log(f"bf16 sweep: {ms:.3f} ms ({cnt:.0f} launches), {bf16['mfma_tflops']:.2f} TFLOP/s, "
            f"max rel err psi {worst_psi:.2e} V {worst_v:.2e}")

    dense = None if args.no_dense else dense_leg(args, qc, torch)
    real = None if args.no_real else real_leg(args, qc, torch)
    configs = None if args.no_configs else configs_leg(args, qc, gg, torch)
    serving = serve(args, reqs) if reqs else None

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(graphs, sigmas, args.cpu_budget_s, lab_host, batch.offsets)
        log(f"cpu oracle: {cpu['value']:.3e} pair-terms/s on {cpu['cores']} threads, "
            f"labels {'equal' if cpu['parity_ok'] else 'DIFFERENT'}")
        one = cpu_baseline(graphs, sigmas, args.cpu_1t_budget_s, lab_host, batch.offsets, threads=1)
        cpu["one_thread"] = {k: one[k] for k in ("value", "cores", "sample", "parity_ok")}
        cpu["parity_ok"] = cpu["parity_ok"] and one["parity_ok"]
        log(f"cpu oracle, one thread: {one['value']:.3e} pair-terms/s")

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
        "tiles": {"bfs_plans": {f"{bw}x{nw}x{p}x{sh}": c for (bw, nw, p, sh), c
                                in sorted(Counter(tuned).items())},
                  "bfs_plan_key": "sources per batch x words per thread x planes x shape",
                  "bfs_policy": {"widest_batch": stage_tiles["bfs_widest"],
                                 "seen_in_registers_first": stage_tiles["bfs_front_first"]},
                  "hist_waves": {str(k): w for k, w in stage_tiles["hist_waves"].items() if w},
                  "jump": stage_tiles["jump"],
                  "stages_beside_searches": stage_tiles["overlap"]},
        "dominant_kernel": dom,
        "roofline": {
            "bound": "hbm", "kernel": "k_bfs",
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": profiled_traffic(bfs_launches),
            "traffic_unit": "HBM bytes per launch (rocprofv3 counters, copy-calibrated)",
            "algorithmic_bytes_per_launch": bytes_step / bfs_launches,
        },
        "bfs_alu": bfs_alu(stages),
        "bfs_search": {
            "edge_visits_per_step": edge_visits,
            "edge_visits_per_s": edge_visits / (bfs_ms * 1e-3),
            "lds_bytes_gathered_per_step": lds_gathered,
            "lds_gather_tbs": lds_gathered / (bfs_ms * 1e-3) / 1e12,
            "lds_peak_tbs": LDS_PEAK_TBS,
            "lds_gather_frac": lds_gathered / (bfs_ms * 1e-3) / 1e12 / LDS_PEAK_TBS,
            "note": "visits counted on the device (pulled levels x edge entries + pushed row "
                    "entries); time = the search's device time per step",
        },
        "hist_kernel_gbs": hist_gbs,
        "plain": plain,
        "bf16_sweep": bf16,
        "dense": dense,
        "real_weights": real,
        "configs": configs,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(result))


if __name__ == "__main__":
    main()
