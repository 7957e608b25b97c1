"""Application loops on aggregate results, written from the paper's
definitions (test infrastructure only: only the tests use this module).

* Ridge linear regression (Section 2, linear regression): minimise
  J(theta) = 1/(2|D|) sum_X (sum_j theta_j X_j)^2 + lambda/2 |theta|^2 with
  the label's coefficient fixed at -1, over the non-centred covariance matrix
  C = sum_X X X^T of X = [1, X_1, ..., X_n] (C[0, 0] = |D|).  Its minimiser
  solves (C_FF / |D| + lambda I) theta_F = C_F,label / |D| over the free
  indices F: batch gradient descent converges to that point.
* Mutual information of two categorical attributes (Section 2, equation (7)):
  sum over cells of delta/alpha * log(alpha * delta / (beta * gamma)), with
  alpha the total count, beta and gamma the marginals, delta the pair count.
* Chow-Liu tree: pairs taken by decreasing mutual information (equal values:
  lower pair index first), each kept when it joins two components.
* Decision-tree splits (Section 2, decision trees): for a regression tree the
  cost of a split is the variance sum y^2 - (sum y)^2 / n of both sides; for a
  classification tree the count-weighted Gini index n (1 - sum_k p_k^2) of
  both sides.  A continuous attribute's split X <= t_k puts buckets 0..k on
  the left; a categorical attribute's split X = v puts cell v on the left.
  The best split of a node is the lowest cost, then the lowest input index,
  then the lowest cell; splits with an empty side are not candidates.
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np

VARIANCE, GINI = 0, 1


def ridge_closed_form(C: np.ndarray, label: int, lam: float) -> np.ndarray:
    C = np.asarray(C, np.float64)
    n = C.shape[0]
    N = C[0, 0]
    free = [i for i in range(n) if i != label]
    A = C[np.ix_(free, free)] / N + lam * np.eye(len(free))
    b = C[free, label] / N
    theta = np.full(n, -1.0)
    theta[free] = np.linalg.solve(A, b)
    return theta


def ridge_objective(C: np.ndarray, theta: np.ndarray, label: int, lam: float) -> float:
    C = np.asarray(C, np.float64)
    th = np.asarray(theta, np.float64)
    free = np.arange(len(th)) != label
    return float(0.5 * th @ C @ th / C[0, 0] + 0.5 * lam * np.sum(th[free] ** 2))


def mutual_information(pair_counts: np.ndarray) -> float:
    d = np.asarray(pair_counts, np.float64)
    alpha = d.sum()
    if alpha == 0:
        return 0.0
    beta = d.sum(axis=1)
    gamma = d.sum(axis=0)
    total = 0.0
    for a in range(d.shape[0]):
        for b in range(d.shape[1]):
            delta = d[a, b]
            if delta > 0:
                total += delta / alpha * math.log(alpha * delta / (beta[a] * gamma[b]))
    return total


def pair_index(n: int) -> List[Tuple[int, int]]:
    return [(i, j) for i in range(n) for j in range(i + 1, n)]


def chow_liu(mi: np.ndarray) -> Tuple[List[Tuple[int, int]], float]:
    n = mi.shape[0]
    pairs = pair_index(n)
    order = sorted(range(len(pairs)), key=lambda k: (-mi[pairs[k]], k))
    comp = list(range(n))

    def root(a):
        while comp[a] != a:
            a = comp[a]
        return a

    edges, total = [], 0.0
    for k in order:
        i, j = pairs[k]
        a, b = root(i), root(j)
        if a == b:
            continue
        comp[max(a, b)] = min(a, b)
        edges.append((i, j))
        total += float(mi[i, j])
        if len(edges) == n - 1:
            break
    return edges, total


def split_cost(I: dict, cell: int, criterion: int, n_labels: int = 0) -> float:
    """Cost of one split (input I, threshold index or category `cell`), as best_splits rates it."""
    cat = I["categorical"]
    if criterion == VARIANCE:
        cnt = np.asarray(I["counts"], np.float64)
        s = np.asarray(I["sums"], np.float64)
        sel = np.zeros(len(cnt), bool)
        if cat:
            sel[cell] = True
        else:
            sel[:cell + 1] = True
        out = 0.0
        for m in (sel, ~sel):
            n = cnt[m].sum()
            out += s[m, 1].sum() - s[m, 0].sum() ** 2 / n if n > 0 else 0.0
        return float(out)
    cnt = np.asarray(I["counts"], np.float64).reshape(n_labels, -1)
    sel = np.zeros(cnt.shape[1], bool)
    if cat:
        sel[cell] = True
    else:
        sel[:cell + 1] = True
    out = 0.0
    for m in (sel, ~sel):
        h = cnt[:, m].sum(axis=1)
        out += h.sum() - (h ** 2).sum() / h.sum() if h.sum() > 0 else 0.0
    return float(out)


def best_splits(inputs: Sequence[dict], n_nodes: int, criterion: int, n_labels: int = 0):
    """inputs: dicts with node, categorical, counts (regression: [cells]; classification:
    [labels, cells]) and, for regression, sums [cells, 2] (sum y, sum y^2).  Returns per node
    (cost, input index, cell), or (0.0, -1, -1) when the node has no candidate split."""
    best = [(math.inf, -1, -1)] * n_nodes
    for k, I in enumerate(inputs):
        cat = I["categorical"]
        if criterion == VARIANCE:
            cnt = np.asarray(I["counts"], np.float64)
            s = np.asarray(I["sums"], np.float64)
            nc = len(cnt)
            N, S1, S2 = cnt.sum(), s[:, 0].sum(), s[:, 1].sum()

            def var(n, a, b):
                return b - a * a / n if n > 0 else 0.0

            for c in range(nc if cat else nc - 1):
                if cat:
                    ln, l1, l2 = cnt[c], s[c, 0], s[c, 1]
                else:
                    ln, l1, l2 = cnt[:c + 1].sum(), s[:c + 1, 0].sum(), s[:c + 1, 1].sum()
                if ln <= 0 or N - ln <= 0:
                    continue
                cost = var(ln, l1, l2) + var(N - ln, S1 - l1, S2 - l2)
                if (cost, k, c) < best[I["node"]]:
                    best[I["node"]] = (cost, k, c)
        else:
            cnt = np.asarray(I["counts"], np.float64).reshape(n_labels, -1)
            nc = cnt.shape[1]
            tot = cnt.sum(axis=1)
            N = tot.sum()
            for c in range(nc if cat else nc - 1):
                left = cnt[:, c] if cat else cnt[:, :c + 1].sum(axis=1)
                right = tot - left
                ln, rn = left.sum(), right.sum()
                if ln <= 0 or rn <= 0:
                    continue
                cost = (ln - (left ** 2).sum() / ln) + (rn - (right ** 2).sum() / rn)
                if (cost, k, c) < best[I["node"]]:
                    best[I["node"]] = (cost, k, c)
    return [(0.0, -1, -1) if b[1] < 0 else b for b in best]
