"""Clustering quality measures of Section 4.2 (evaluation, on host labels).

* modularity Q = (1/w) sum_ij (A_ij - gamma k_i k_j / w) [c_i = c_j], w = 2|E|
* ARI  = (RI - E[RI]) / (max RI - E[RI])  (adjusted for chance)
* FMI  = TP / sqrt((TP + FP)(TP + FN))     (pairs clustered together)
* NMI  = MI / sqrt(H(true) H(pred))        (natural logarithms)

Pair counts come from the contingency table of the two labelings. These run
on the host on the labels the GPU path returns; they are not part of the hot
path.
"""
from __future__ import annotations

import numpy as np


def _contingency(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    _, ai = np.unique(a, return_inverse=True)
    _, bi = np.unique(b, return_inverse=True)
    table = np.zeros((ai.max() + 1, bi.max() + 1), dtype=np.int64)
    np.add.at(table, (ai, bi), 1)
    return table


def _comb2(x):
    x = np.asarray(x, dtype=np.float64)
    return x * (x - 1.0) / 2.0


def ari(labels_true, labels_pred) -> float:
    t = _contingency(labels_true, labels_pred)
    n = t.sum()
    sum_ij = _comb2(t).sum()
    sum_a = _comb2(t.sum(axis=1)).sum()
    sum_b = _comb2(t.sum(axis=0)).sum()
    expected = sum_a * sum_b / _comb2(n)
    maximum = 0.5 * (sum_a + sum_b)
    if maximum == expected:
        return 1.0
    return float((sum_ij - expected) / (maximum - expected))


def fmi(labels_true, labels_pred) -> float:
    t = _contingency(labels_true, labels_pred)
    tp = _comb2(t).sum()
    p = _comb2(t.sum(axis=0)).sum()   # pairs together in the prediction (TP + FP)
    q = _comb2(t.sum(axis=1)).sum()   # pairs together in the truth (TP + FN)
    if p == 0 or q == 0:
        return 0.0
    return float(tp / np.sqrt(p * q))


def _entropy(counts):
    p = counts[counts > 0] / counts.sum()
    return float(-(p * np.log(p)).sum())


def nmi(labels_true, labels_pred) -> float:
    t = _contingency(labels_true, labels_pred).astype(np.float64)
    n = t.sum()
    pij = t / n
    pi = pij.sum(axis=1, keepdims=True)
    pj = pij.sum(axis=0, keepdims=True)
    nz = pij > 0
    mi = float((pij[nz] * np.log(pij[nz] / (pi @ pj)[nz])).sum())
    h_true = _entropy(t.sum(axis=1))
    h_pred = _entropy(t.sum(axis=0))
    if h_true == 0.0 and h_pred == 0.0:
        return 1.0
    if h_true == 0.0 or h_pred == 0.0:
        return 0.0
    return float(mi / np.sqrt(h_true * h_pred))


def modularity(row_ptr, col, labels, gamma: float = 1.0) -> float:
    """Q of a partition of an undirected graph given as a symmetric CSR."""
    row_ptr = np.asarray(row_ptr)
    col = np.asarray(col)
    labels = np.asarray(labels)
    n = labels.shape[0]
    deg = np.diff(row_ptr).astype(np.float64)
    w = deg.sum()
    if w == 0:
        return 0.0
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    inside = (labels[rows] == labels[col]).sum()
    _, inv = np.unique(labels, return_inverse=True)
    deg_c = np.bincount(inv, weights=deg)
    return float(inside / w - gamma * (deg_c ** 2).sum() / (w * w))


def scores(row_ptr, col, labels_true, labels_pred) -> dict:
    return {"modularity": modularity(row_ptr, col, labels_pred),
            "nmi": nmi(labels_true, labels_pred),
            "ari": ari(labels_true, labels_pred),
            "fmi": fmi(labels_true, labels_pred),
            "clusters": int(np.unique(labels_pred).size)}
