"""Seeded synthetic graph workloads (stochastic block models).

This module only draws random graphs; it holds none of the clustering
arithmetic. Both the CPU oracle tests and the HIP path take their inputs
from here, so the two sides always see the same CSR for the same seed.

The datasets the paper evaluates on (Section 4.1: citation graphs of a few
thousand nodes and a few thousand edges, with a handful of classes) are not
available, so seeded stochastic-block-model graphs of the same shape stand
in for them:

* ``sbm``      plain SBM: Bernoulli edge per pair, plus a random recursive
               spanning tree so the graph is connected.
* ``dcsbm``    degree-corrected SBM: node weights theta drawn from a
               truncated Pareto (pdf ~ theta^-2.5 on [1, sqrt(N)]), a fraction
               mu of edge endpoints kept inside the block, endpoints drawn
               proportional to theta until exactly M distinct non-loop edges
               exist. No spanning tree: these graphs are disconnected, like
               the citation graphs.

Every graph is returned as a canonical undirected CSR (symmetric, sorted,
no duplicates, no self-loops), int32 ``row_ptr`` [N+1] and ``col`` [nnz].
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Graph:
    n: int
    row_ptr: np.ndarray  # int32 [n+1]
    col: np.ndarray      # int32 [nnz]
    blocks: np.ndarray   # int32 [n], planted block of each node
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)


def csr_from_edges(n: int, u: np.ndarray, v: np.ndarray):
    """Canonical symmetric CSR from an undirected edge list (u, v).

    Loops are dropped, both directions are inserted, duplicates removed,
    rows sorted by column.
    """
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    a = np.concatenate([u, v])
    b = np.concatenate([v, u])
    key = np.unique(a * n + b)
    rows = (key // n).astype(np.int64)
    cols = (key % n).astype(np.int32)
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] > np.iinfo(np.int32).max:
        raise ValueError("graph too large for int32 CSR")
    return row_ptr.astype(np.int32), cols


def csr_from_arcs(n: int, tail: np.ndarray, head: np.ndarray):
    """Canonical directed CSR (row = tail, sorted heads, no duplicates, no
    self-loops) from a list of arcs tail -> head."""
    tail = np.asarray(tail, dtype=np.int64)
    head = np.asarray(head, dtype=np.int64)
    keep = tail != head
    key = np.unique(tail[keep] * n + head[keep])
    rows = key // n
    cols = (key % n).astype(np.int32)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    return row_ptr.astype(np.int32), cols


def _largest_remainder(fracs: np.ndarray, n: int) -> np.ndarray:
    raw = fracs * n
    sizes = np.floor(raw).astype(np.int64)
    short = n - int(sizes.sum())
    order = np.argsort(-(raw - sizes), kind="stable")
    sizes[order[:short]] += 1
    return sizes


def _block_labels(rng: np.random.Generator, sizes: np.ndarray) -> np.ndarray:
    labels = np.repeat(np.arange(len(sizes), dtype=np.int32), sizes)
    rng.shuffle(labels)  # node ids carry no block order, as in real data
    return labels


def sbm(n: int, n_blocks: int, p_in: float, p_out: float, seed: int,
        spanning_tree: bool = True) -> Graph:
    """Plain SBM with equal blocks, plus a random recursive spanning tree."""
    rng = np.random.default_rng(seed)
    sizes = _largest_remainder(np.full(n_blocks, 1.0 / n_blocks), n)
    blocks = _block_labels(rng, sizes)
    iu, ju = np.triu_indices(n, k=1)
    p = np.where(blocks[iu] == blocks[ju], p_in, p_out)
    hit = rng.random(iu.shape[0]) < p
    eu, ev = [iu[hit]], [ju[hit]]
    if spanning_tree:
        perm = rng.permutation(n)
        t = np.arange(1, n)
        parent_pos = (rng.random(n - 1) * t).astype(np.int64)  # uniform in [0, t)
        eu.append(perm[1:])
        ev.append(perm[parent_pos])
    row_ptr, col = csr_from_edges(n, np.concatenate(eu), np.concatenate(ev))
    return Graph(n, row_ptr, col, blocks, name=f"sbm(n={n},seed={seed})")


def _pareto_theta(rng: np.random.Generator, n: int, exponent: float = 2.5) -> np.ndarray:
    """theta with pdf ~ theta^-exponent on [1, sqrt(n)] (inverse CDF)."""
    lo, hi = 1.0, max(math.sqrt(n), 1.0 + 1e-9)
    a = exponent - 1.0
    u = rng.random(n)
    lo_a, hi_a = lo ** (-a), hi ** (-a)
    return (lo_a - u * (lo_a - hi_a)) ** (-1.0 / a)


def dcsbm(n: int, block_fracs, mean_degree: float, seed: int, mu: float = 0.8,
          exponent: float = 2.5) -> Graph:
    """Degree-corrected SBM with exactly round(n*mean_degree/2) edges."""
    rng = np.random.default_rng(seed)
    fr = np.asarray(block_fracs, dtype=np.float64)
    fr = fr / fr.sum()
    sizes = _largest_remainder(fr, n)
    blocks = _block_labels(rng, sizes)
    theta = _pareto_theta(rng, n, exponent)
    m_target = int(round(n * mean_degree / 2.0))
    max_edges = n * (n - 1) // 2
    if m_target > max_edges:
        raise ValueError("mean degree too large for n")

    p_all = theta / theta.sum()
    cdf_all = np.cumsum(p_all)
    nb = len(sizes)
    members = [np.flatnonzero(blocks == b) for b in range(nb)]
    cdf_blk = []
    for mem in members:
        w = theta[mem]
        cdf_blk.append(np.cumsum(w / w.sum()) if len(mem) else np.zeros(0))

    keys = np.zeros(0, dtype=np.int64)
    while keys.shape[0] < m_target:
        need = m_target - keys.shape[0]
        draw = int(need * 1.3) + 64
        u = np.minimum(np.searchsorted(cdf_all, rng.random(draw)), n - 1)
        inside = rng.random(draw) < mu
        r = rng.random(draw)
        v = np.minimum(np.searchsorted(cdf_all, r), n - 1)
        bu = blocks[u]
        for b in range(nb):
            sel = np.flatnonzero(inside & (bu == b))
            if sel.size and len(members[b]):
                pos = np.minimum(np.searchsorted(cdf_blk[b], r[sel]), len(members[b]) - 1)
                v[sel] = members[b][pos]
        ok = u != v
        a = np.minimum(u, v)[ok]
        c = np.maximum(u, v)[ok]
        new = a.astype(np.int64) * n + c
        # keep first occurrences, in draw order, until the target is met
        _, first = np.unique(new, return_index=True)
        new = new[np.sort(first)]
        new = new[~np.isin(new, keys)]
        keys = np.concatenate([keys, new[:need]])
    eu = keys // n
    ev = keys % n
    row_ptr, col = csr_from_edges(n, eu, ev)
    return Graph(n, row_ptr, col, blocks,
                 name=f"dcsbm(n={n},blocks={nb},deg={mean_degree:g},seed={seed})")


def dcsbm_directed(n: int, block_fracs, mean_out_degree: float, seed: int, mu: float = 0.8,
                   exponent: float = 2.5) -> Graph:
    """Directed degree-corrected SBM (citation-like): exactly
    round(n * mean_out_degree) distinct arcs, tails drawn proportional to an
    out-weight and heads to an in-weight (both truncated Pareto), the head
    inside the tail's block with probability mu."""
    rng = np.random.default_rng(seed)
    fr = np.asarray(block_fracs, dtype=np.float64)
    fr = fr / fr.sum()
    sizes = _largest_remainder(fr, n)
    blocks = _block_labels(rng, sizes)
    t_out = _pareto_theta(rng, n, exponent)
    t_in = _pareto_theta(rng, n, exponent)
    m_target = int(round(n * mean_out_degree))
    if m_target > n * (n - 1):
        raise ValueError("mean out-degree too large for n")
    cdf_out = np.cumsum(t_out / t_out.sum())
    cdf_in = np.cumsum(t_in / t_in.sum())
    nb = len(sizes)
    members = [np.flatnonzero(blocks == b) for b in range(nb)]
    cdf_blk = [np.cumsum(t_in[m] / t_in[m].sum()) if len(m) else np.zeros(0) for m in members]
    keys = np.zeros(0, dtype=np.int64)
    while keys.shape[0] < m_target:
        need = m_target - keys.shape[0]
        draw = int(need * 1.3) + 64
        u = np.minimum(np.searchsorted(cdf_out, rng.random(draw)), n - 1)
        inside = rng.random(draw) < mu
        r = rng.random(draw)
        v = np.minimum(np.searchsorted(cdf_in, r), n - 1)
        bu = blocks[u]
        for b in range(nb):
            sel = np.flatnonzero(inside & (bu == b))
            if sel.size and len(members[b]):
                pos = np.minimum(np.searchsorted(cdf_blk[b], r[sel]), len(members[b]) - 1)
                v[sel] = members[b][pos]
        ok = u != v
        new = u[ok].astype(np.int64) * n + v[ok]
        _, first = np.unique(new, return_index=True)
        new = new[np.sort(first)]
        new = new[~np.isin(new, keys)]
        keys = np.concatenate([keys, new[:need]])
    row_ptr, col = csr_from_arcs(n, keys // n, keys % n)
    return Graph(n, row_ptr, col, blocks,
                 name=f"dcsbm_directed(n={n},blocks={nb},outdeg={mean_out_degree:g},seed={seed})")


def edge_weights(g: Graph, max_weight: int, seed: int, directed: bool = False) -> np.ndarray:
    """Seeded integer weights 1..max_weight, one per CSR entry (uint8). For an
    undirected graph both directions of an edge get the same weight."""
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    cols = g.col.astype(np.int64)
    if directed:
        return rng.integers(1, max_weight + 1, g.nnz).astype(np.uint8)
    lo, hi = np.minimum(rows, cols), np.maximum(rows, cols)
    key = lo * g.n + hi
    uniq, inv = np.unique(key, return_inverse=True)
    w = rng.integers(1, max_weight + 1, uniq.shape[0]).astype(np.uint8)
    return w[inv]


def real_edge_weights(g: Graph, seed: int, lo: float = 0.5, hi: float = 4.0,
                      directed: bool = False, dyadic: bool = False) -> np.ndarray:
    """Seeded positive real weights, one per CSR entry (float32): uniform in
    [lo, hi), or with dyadic=True multiples of 1/8 in [1/8, 4] (every path
    sum below 2^20 is then exact in float32). For an undirected graph both
    directions of an edge get the same weight."""
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    cols = g.col.astype(np.int64)

    def draw(k):
        if dyadic:
            return (rng.integers(1, 33, k) / 8.0).astype(np.float32)
        return rng.uniform(lo, hi, k).astype(np.float32)

    if directed:
        return draw(g.nnz)
    lo_, hi_ = np.minimum(rows, cols), np.maximum(rows, cols)
    uniq, inv = np.unique(lo_ * g.n + hi_, return_inverse=True)
    return draw(uniq.shape[0])[inv]


def random_digraph(n: int, p: float, seed: int) -> Graph:
    """Directed Erdos-Renyi graph: each ordered pair an arc with probability p."""
    rng = np.random.default_rng(seed)
    a = rng.random((n, n)) < p
    np.fill_diagonal(a, False)
    t, h = np.nonzero(a)
    row_ptr, col = csr_from_arcs(n, t, h)
    return Graph(n, row_ptr, col, np.zeros(n, dtype=np.int32), name=f"digraph(n={n},p={p},seed={seed})")


# ---------------------------------------------------------------------------
# The five workloads.

SIGMAS_C1 = [1.0]
SIGMAS_C2 = [0.5, 1.0, 2.0, 3.0]
SIGMAS_C3 = [2.0]


def sigmas_c4() -> list:
    return [float(x) for x in np.geomspace(0.25, 8.0, 32)]


def config1() -> Graph:
    """N=200, 4 equal blocks, p_in 0.10, p_out 0.005, spanning tree, seed 0."""
    return sbm(200, 4, 0.10, 0.005, seed=0)


def config2() -> Graph:
    """N=2,708, 7 Dirichlet(2) blocks, ~5,400 edges (mean degree 4), seed 1."""
    rng = np.random.default_rng(1)
    fr = rng.dirichlet(np.full(7, 2.0))
    return dcsbm(2708, fr, 4.0, seed=10_001)


def config3() -> Graph:
    """N=19,717, 3 blocks 40/40/20%, mean degree 4.5, seed 2."""
    return dcsbm(19717, [0.4, 0.4, 0.2], 4.5, seed=2)


def config4_params(i: int) -> dict:
    """Draw of graph i (0..63) of the batched sigma sweep, seed 100+i."""
    rng = np.random.default_rng(100 + i)
    n = int(round(math.exp(rng.uniform(math.log(1e3), math.log(2e4)))))
    nb = int(rng.integers(2, 17))
    deg = float(rng.uniform(3.0, 8.0))
    fr = rng.dirichlet(np.full(nb, 2.0))
    return dict(n=n, fracs=fr, deg=deg, seed=100 + i)


def config4_graph(i: int) -> Graph:
    p = config4_params(i)
    return dcsbm(p["n"], p["fracs"], p["deg"], seed=1_000_000 + p["seed"])


def config4() -> list:
    return [config4_graph(i) for i in range(64)]


def config5_request(r: int) -> dict:
    """Request r (0..1023) of the serving stream, seed 1000+r."""
    rng = np.random.default_rng(1000 + r)
    n = int(round(math.exp(rng.uniform(math.log(500.0), math.log(5e4)))))
    nb = int(rng.integers(2, 33))
    deg = float(rng.uniform(3.0, 10.0))
    n_sig = int(rng.integers(1, 9))
    sig = [float(x) for x in rng.uniform(0.5, 4.0, n_sig)]
    fr = rng.dirichlet(np.full(nb, 2.0))
    return dict(n=n, fracs=fr, deg=deg, sigmas=sig, seed=1000 + r)


def config5_graph(r: int) -> tuple:
    p = config5_request(r)
    g = dcsbm(p["n"], p["fracs"], p["deg"], seed=2_000_000 + p["seed"])
    return g, p["sigmas"]


def poisson_arrivals(n_req: int, rate: float, seed: int = 77) -> np.ndarray:
    """Arrival times (seconds) of a Poisson stream of n_req requests."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n_req))


def dense_points(n: int, dim: int = 8, clusters: int = 6, seed: int = 0) -> np.ndarray:
    """Fully connected workload: Euclidean distances (float32 [n, n]) between
    n points drawn around `clusters` Gaussian centres in `dim` dimensions."""
    rng = np.random.default_rng(seed)
    centres = rng.normal(0.0, 3.0, (clusters, dim))
    x = centres[rng.integers(0, clusters, n)] + rng.normal(0.0, 1.0, (n, dim))
    sq = (x * x).sum(axis=1)
    d2 = np.maximum(sq[:, None] + sq[None, :] - 2.0 * x @ x.T, 0.0)
    d = np.sqrt(d2)
    np.fill_diagonal(d, 0.0)
    return d.astype(np.float32)


# ---------------------------------------------------------------------------
# Small named graphs (ids as in the usual textbook constructions).

def path_graph(n: int) -> Graph:
    i = np.arange(n - 1)
    rp, c = csr_from_edges(n, i, i + 1)
    return Graph(n, rp, c, np.zeros(n, np.int32), name=f"path{n}")


def star_graph(leaves: int) -> Graph:
    """Centre 0 joined to leaves 1..leaves."""
    n = leaves + 1
    rp, c = csr_from_edges(n, np.zeros(leaves, np.int64), np.arange(1, n))
    return Graph(n, rp, c, np.zeros(n, np.int32), name=f"star{leaves}")


def complete_graph(n: int) -> Graph:
    iu, ju = np.triu_indices(n, k=1)
    rp, c = csr_from_edges(n, iu, ju)
    return Graph(n, rp, c, np.zeros(n, np.int32), name=f"K{n}")


def barbell_graph(m: int) -> Graph:
    """Two K_m (nodes 0..m-1 and m..2m-1) joined by the edge (m-1, m)."""
    iu, ju = np.triu_indices(m, k=1)
    u = np.concatenate([iu, iu + m, [m - 1]])
    v = np.concatenate([ju, ju + m, [m]])
    rp, c = csr_from_edges(2 * m, u, v)
    blk = np.repeat(np.arange(2, dtype=np.int32), m)
    return Graph(2 * m, rp, c, blk, name=f"barbell{m}")


def empty_graph(n: int) -> Graph:
    rp, c = csr_from_edges(n, np.zeros(0, np.int64), np.zeros(0, np.int64))
    return Graph(n, rp, c, np.zeros(n, np.int32), name=f"empty{n}")


def disjoint_union(*gs: Graph) -> Graph:
    off = 0
    us, vs, bl = [], [], []
    for g in gs:
        rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
        us.append(rows + off)
        vs.append(g.col.astype(np.int64) + off)
        bl.append(g.blocks)
        off += g.n
    rp, c = csr_from_edges(off, np.concatenate(us), np.concatenate(vs))
    return Graph(off, rp, c, np.concatenate(bl), name="+".join(g.name for g in gs))


def random_graph(n: int, p: float, seed: int) -> Graph:
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, k=1)
    hit = rng.random(iu.shape[0]) < p
    rp, c = csr_from_edges(n, iu[hit], ju[hit])
    return Graph(n, rp, c, np.zeros(n, np.int32), name=f"gnp({n},{p},{seed})")


def twin_leaves(hubs: int, leaves_per_hub: int) -> Graph:
    """Hubs 0..hubs-1 in a path, each with its own fan of leaves (exact V ties)."""
    n = hubs + hubs * leaves_per_hub
    u = list(range(hubs - 1))
    v = list(range(1, hubs))
    nxt = hubs
    for h in range(hubs):
        for _ in range(leaves_per_hub):
            u.append(h)
            v.append(nxt)
            nxt += 1
    rp, c = csr_from_edges(n, np.array(u), np.array(v))
    return Graph(n, rp, c, np.zeros(n, np.int32), name=f"twins({hubs},{leaves_per_hub})")


def long_path_with_cycle(n: int) -> Graph:
    """Path 0..n-1; used for the int8 distance limit (diameter n-1)."""
    return path_graph(n)
