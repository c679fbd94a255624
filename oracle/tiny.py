"""A second, pure-Python oracle for graphs of a few dozen nodes.

TEST INFRASTRUCTURE ONLY (see the package docstring). It exists to check the
C oracle by an independent route: Python lists, ``collections.deque`` for the
breadth-first search, ``math.exp`` per pair, Python's own ``min`` for the
descent. Too slow for anything beyond ~50 nodes.
"""
from __future__ import annotations

import math
from collections import deque


def adjacency(n, row_ptr, col):
    return [[int(c) for c in col[row_ptr[i]:row_ptr[i + 1]]] for i in range(n)]


def hop_distances(adj):
    """Section 3.1 distance read as hop count; None marks unreachable."""
    n = len(adj)
    out = []
    for s in range(n):
        d = [None] * n
        d[s] = 0
        q = deque([s])
        while q:
            u = q.popleft()
            for v in adj[u]:
                if d[v] is None:
                    d[v] = d[u] + 1
                    q.append(v)
        out.append(d)
    return out


def potential(dist, sigma):
    """Algorithm 1 per node (self included, unreachable skipped)."""
    two_s2 = 2.0 * sigma * sigma
    psi, v = [], []
    for row in dist:
        s1 = 0.0
        s2 = 0.0
        for d in row:
            if d is None:
                continue
            e = math.exp(-(d * d) / two_s2)
            s1 += d * d * e
            s2 += e
        psi.append(s2)
        v.append(s1 / s2 / two_s2)
    return psi, v


def descend(adj, v, merge=False):
    """Algorithm 2 + 3: parent = lowest neighbour if strictly lower (ties to the
    smallest id), or the (V, id) minimum over node and neighbours (merge);
    label = the node the descent ends at."""
    n = len(adj)
    parent = []
    for i in range(n):
        if merge:
            parent.append(min([i] + adj[i], key=lambda j: (v[j], j)))
        else:
            if adj[i]:
                m = min(adj[i], key=lambda j: (v[j], j))
                parent.append(m if v[m] < v[i] else i)
            else:
                parent.append(i)
    labels = []
    for i in range(n):
        x = i
        seen = 0
        while parent[x] != x:
            x = parent[x]
            seen += 1
            assert seen <= n, "cycle in descent"
        labels.append(x)
    return parent, labels
