"""Pins of the application-loop oracle (oracle/apps.py) against library
routines and brute force on materialised joins: scikit-learn's mutual
information and ridge regression, SciPy's minimum spanning tree, and split
costs computed directly from the joined label values."""
import math

import numpy as np
import pytest

import oracle
from oracle import apps
from datagen import Agg, GroupBy, Query, make_batch, make_database
from datagen.configs import cat_attrs, classification_tree_batch, cont_attrs, covariance_queries, tree_level
from tests.helpers import materialize


def covariance_matrix(db, attrs, with_abs=False):
    """The oracle's covariance over [1, attrs...] as an (n+1) x (n+1) matrix (and, with_abs,
    the matching sums of |term|)."""
    qs = covariance_queries(attrs)
    res = oracle.evaluate(db, qs, n_threads=4)
    feats = [None] + list(attrs)
    n = len(feats)
    C = np.zeros((n, n))
    A = np.zeros((n, n))
    for q, r in zip(qs, res):
        if not q.aggs:
            C[0, 0] = A[0, 0] = float(r.counts[0])
            continue
        fs = q.aggs[0].terms[0][1]
        i = feats.index(fs[0])
        j = feats.index(fs[1]) if len(fs) > 1 else 0
        C[i, j] = C[j, i] = r.sums[0, 0]
        A[i, j] = A[j, i] = r.abs_sums[0, 0]
    return (C, A) if with_abs else C


def test_ridge_closed_form_equals_scikit_learn_on_the_materialised_join():
    db = make_database(1, n_fact=20_011)
    J = materialize(db)
    attrs = cont_attrs(db)
    label = attrs[3]
    C = covariance_matrix(db, attrs)
    li = 1 + attrs.index(label)
    for lam in (1e-3, 0.1):
        theta = apps.ridge_closed_form(C, li, lam)
        X = np.stack([np.ones(len(J[label]))] + [J[a] for a in attrs if a != label], axis=1)
        N = X.shape[0]
        # sklearn minimises |y - X w|^2 + alpha |w|^2: alpha = N * lambda for 1/(2N) and lambda/2
        from sklearn.linear_model import Ridge
        w = Ridge(alpha=N * lam, fit_intercept=False, solver="cholesky", tol=1e-12).fit(X, J[label]).coef_
        free = [i for i in range(len(theta)) if i != li]
        np.testing.assert_allclose(theta[free], w, rtol=1e-7, atol=1e-9)
        assert theta[li] == -1.0
        # the objective is lowest there: any perturbation raises it
        J0 = apps.ridge_objective(C, theta, li, lam)
        rng = np.random.default_rng(0)
        for _ in range(5):
            d = np.zeros_like(theta)
            d[free] = rng.normal(size=len(free)) * 1e-3
            assert apps.ridge_objective(C, theta + d, li, lam) > J0


def test_mutual_information_equals_scikit_learn_and_chow_liu_equals_scipy_mst():
    db = make_database(5)
    J = materialize(db)
    cats = sorted(cat_attrs(db))[:7]
    pairs = apps.pair_index(len(cats))
    qs = [Query(groupby=[GroupBy(cats[i]), GroupBy(cats[j])]) for i, j in pairs]
    res = oracle.evaluate(db, qs, n_threads=4)
    from sklearn.metrics import mutual_info_score
    mi = np.zeros((len(cats), len(cats)))
    for (i, j), q, r in zip(pairs, qs, res):
        da, db_ = q.groupby[0].domain(db), q.groupby[1].domain(db)
        got = apps.mutual_information(r.counts.reshape(da, db_))
        ref = mutual_info_score(J[cats[i]], J[cats[j]])
        assert abs(got - ref) <= 1e-10 * max(1.0, abs(ref))
        mi[i, j] = mi[j, i] = got
    edges, total = apps.chow_liu(mi)
    from scipy.sparse.csgraph import minimum_spanning_tree
    # a maximum spanning tree of MI is a minimum spanning tree of (max + 1 - MI) on the same pairs
    w = np.where(np.triu(np.ones_like(mi), 1) > 0, mi.max() + 1.0 - mi, 0.0)
    T = minimum_spanning_tree(w).toarray()
    ref_edges = sorted((min(i, j), max(i, j)) for i, j in zip(*np.nonzero(T)))
    assert sorted(edges) == ref_edges
    assert abs(total - sum(mi[i, j] for i, j in ref_edges)) <= 1e-12


def test_mutual_information_closed_forms():
    """Independent attributes give 0; a bijection gives the entropy of either side."""
    assert apps.mutual_information(np.outer([3, 1, 4], [2, 5])) == pytest.approx(0.0, abs=1e-15)
    p = np.array([5, 3, 2], np.float64)
    H = -sum(x / p.sum() * math.log(x / p.sum()) for x in p)
    assert apps.mutual_information(np.diag(p)) == pytest.approx(H, rel=1e-14)


def _mask(J, preds):
    m = np.ones(len(J["y"]), bool)
    for p in preds:
        x = J[p.attr]
        if x.dtype.kind == "f":
            x, t = x.astype(np.float32), np.float32(p.value)
        else:
            t = float(p.value)
        m &= {"le": x <= t, "lt": x < t, "ge": x >= t, "gt": x > t, "eq": x == t, "ne": x != t}[p.op]
    return m


def test_regression_and_classification_splits_equal_brute_force():
    """The best split per node from the oracle's histograms equals the one found
    by computing every split's cost directly from the joined label values."""
    db = make_database(3, n_fact=30_011, dims=(500, 200, 50))
    J = materialize(db)
    level = tree_level(db, n_nodes=4, seed=3)
    feats = level.features[:8] + level.features[-4:]      # continuous and categorical attributes
    qs, inputs = [], []
    for ni, preds in enumerate(level.nodes):
        for a in feats:
            qs.append(Query([GroupBy(a, level.thresholds.get(a))], list(preds), [Agg.monomial("y"), Agg.monomial("y", "y")]))
    res = oracle.evaluate(db, qs, n_threads=4)
    k = 0
    for ni in range(len(level.nodes)):
        for a in feats:
            r = res[k]
            inputs.append({"node": ni, "categorical": a not in level.thresholds, "counts": r.counts, "sums": r.sums})
            k += 1
    best = apps.best_splits(inputs, len(level.nodes), apps.VARIANCE)
    for ni, preds in enumerate(level.nodes):
        m = _mask(J, preds)
        y = J["y"][m]
        brute = (math.inf, -1, -1)
        for fi, a in enumerate(feats):
            x = J[a][m]
            if a in level.thresholds:
                cell = np.searchsorted(level.thresholds[a], x.astype(np.float32), side="left")
                cands = [(c, cell <= c) for c in range(len(level.thresholds[a]))]
            else:
                cands = [(c, x == c) for c in range(db.column(a).domain)]
            for c, left in cands:
                if left.sum() == 0 or (~left).sum() == 0:
                    continue
                cost = sum(float(np.sum(v ** 2) - np.sum(v) ** 2 / len(v)) for v in (y[left], y[~left]))
                key = (cost, ni * len(feats) + fi, c)
                if key[0] < brute[0] - 1e-9 * abs(key[0]):
                    brute = key
        assert best[ni][1:] == brute[1:], (ni, best[ni], brute)
        assert abs(best[ni][0] - brute[0]) <= 1e-9 * abs(brute[0])
    # classification on the label g3: count-weighted Gini from COUNT GROUP BY (g3, bucket)
    label = "g3"
    nl = db.column(label).domain
    cqs = [q for q in classification_tree_batch(db, label, level) if len(q.groupby) == 2]
    cres = oracle.evaluate(db, cqs, n_threads=4)
    per_node = len(cqs) // len(level.nodes)
    cin = [{"node": i // per_node, "categorical": q.groupby[1].thresholds is None, "counts": r.counts}
           for i, (q, r) in enumerate(zip(cqs, cres))]
    cbest = apps.best_splits(cin, len(level.nodes), apps.GINI, nl)
    for ni, preds in enumerate(level.nodes):
        m = _mask(J, preds)
        lab = J[label][m]
        brute = (math.inf, -1, -1)
        for qi in range(ni * per_node, (ni + 1) * per_node):
            g = cqs[qi].groupby[1]
            x = J[g.attr][m]
            if g.thresholds is not None:
                cell = np.searchsorted(g.thresholds, x.astype(np.float32), side="left")
                cands = [(c, cell <= c) for c in range(len(g.thresholds))]
            else:
                cands = [(c, x == c) for c in range(g.domain(db))]
            for c, left in cands:
                if left.sum() == 0 or (~left).sum() == 0:
                    continue
                cost = 0.0
                for side in (left, ~left):
                    h = np.bincount(lab[side], minlength=nl).astype(np.float64)
                    cost += h.sum() - (h ** 2).sum() / h.sum()
                if cost < brute[0] - 1e-9 * abs(cost):
                    brute = (cost, qi, c)
        assert cbest[ni][1:] == brute[1:], (ni, cbest[ni], brute)
