"""The application loops on the device (through the C ABI) against the
oracle's (oracle/apps.py): on the oracle's own aggregates uploaded as inputs
(the loop alone), and end to end on the engine's results.

* ridge regression by batch gradient descent over workload 1's covariance
  matrix: the parameters reach the closed-form minimiser (relative 1e-6) and
  the objective matches;
* mutual information of workload 5's 105 pair tables (relative 1e-12 on the
  same counts) and the Chow-Liu tree (the same edges);
* the best split of every node of workload 3's regression-tree level
  (variance) and of a classification-tree level (Gini): the same input and
  cell, cost within 1e-12 on the same aggregates.
"""
import numpy as np
import pytest

import oracle
from oracle import apps
from datagen import make_batch, make_database
from datagen.configs import cat_attrs, classification_tree_batch, cont_attrs, covariance_queries, tree_level
from tests.helpers import check_sums

pytestmark = pytest.mark.gpu


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(torch.device("cuda", 0))


def test_ridge_bgd_reaches_the_closed_form():
    from paper_1906_08687_amd import lmfao
    from tests.test_oracle_apps import covariance_matrix
    db = make_database(1)
    attrs = cont_attrs(db)
    li = 1 + attrs.index(attrs[3])
    C, A = covariance_matrix(db, attrs, with_abs=True)
    for lam in (1e-3, 0.1):
        ref = apps.ridge_closed_form(C, li, lam)
        theta, info = lmfao.ridge_bgd(_dev(C), li, lam, 5000, 1e-12)
        theta = theta.cpu().numpy()
        np.testing.assert_allclose(theta, ref, rtol=1e-6, atol=1e-9)
        assert abs(info[0] - apps.ridge_objective(C, ref, li, lam)) <= 1e-9 * abs(info[0])
        assert info[1] < 5000
    # end to end: the engine's covariance block (fp32 with fp64 merge) as input
    eng = lmfao.Engine(db, covariance_queries(attrs), precision="fp32")
    eng.run()
    Cg = lmfao.covariance_matrix(eng, attrs)
    check_sums(Cg.cpu().numpy(), C, A, 1e-6, "engine covariance")
    theta, _ = lmfao.ridge_bgd(Cg, li, 0.1, 5000, 1e-12)
    np.testing.assert_allclose(theta.cpu().numpy(), apps.ridge_closed_form(C, li, 0.1), rtol=1e-4, atol=1e-6)


def test_mutual_information_and_chow_liu():
    from paper_1906_08687_amd import lmfao
    db = make_database(5)
    qs = make_batch(5, db)
    cats = cat_attrs(db)
    pairs = [(i, q) for i, q in enumerate(qs) if len(q.groupby) == 2]
    ref = oracle.evaluate(db, [q for _, q in pairs])
    eng = lmfao.Engine(db, qs)
    eng.run()
    got_mi = lmfao.mutual_information(eng, [i for i, _ in pairs]).cpu().numpy()
    n = len(cats)
    mi = np.zeros((n, n))
    for k, ((i, q), r) in enumerate(zip(pairs, ref)):
        da, db_ = q.groupby[0].domain(db), q.groupby[1].domain(db)
        m = apps.mutual_information(r.counts.reshape(da, db_))
        assert abs(got_mi[k] - m) <= 1e-12 * max(1.0, abs(m)), (k, got_mi[k], m)
        a, b = cats.index(q.groupby[0].attr), cats.index(q.groupby[1].attr)
        mi[a, b] = mi[b, a] = m
    edges, total = lmfao.chow_liu(_dev(mi))
    ref_edges, ref_total = apps.chow_liu(mi)
    assert edges == ref_edges
    assert abs(total - ref_total) <= 1e-12 * ref_total


def _split_inputs_ref(level_nodes, qs, res, db, criterion):
    per_node = len(qs) // len(level_nodes)
    out = []
    for i, (q, r) in enumerate(zip(qs, res)):
        g = q.groupby[-1]
        d = {"node": i // per_node, "categorical": g.thresholds is None, "counts": r.counts}
        if criterion == apps.VARIANCE:
            d["sums"] = r.sums
        out.append(d)
    return out


@pytest.mark.parametrize("criterion", ["variance", "gini"])
def test_best_splits_of_a_tree_level(criterion):
    from paper_1906_08687_amd import lmfao
    db = make_database(3)
    level = tree_level(db, seed=3)
    if criterion == "variance":
        qs = make_batch(3, db)
        crit, nl = apps.VARIANCE, 0
    else:
        qs = [q for q in classification_tree_batch(db, "g3", level) if len(q.groupby) == 2]
        crit, nl = apps.GINI, db.column("g3").domain
    ref_res = oracle.evaluate(db, qs)
    inputs = _split_inputs_ref(level.nodes, qs, ref_res, db, crit)
    ref = apps.best_splits(inputs, len(level.nodes), crit, nl)
    eng = lmfao.Engine(db, qs)
    eng.run()

    def agree(got, rtol):
        # the chosen split is the oracle's, or one whose cost (rated by the oracle) ties with it
        # to rtol: distinct attributes can split a node's rows identically
        ties = 0
        for node, (g, r) in enumerate(zip(got, ref)):
            assert (g[1] < 0) == (r[1] < 0), (node, g, r)
            if r[1] < 0:
                continue
            assert inputs[g[1]]["node"] == node, (node, g)
            assert abs(g[0] - r[0]) <= rtol * max(1.0, abs(r[0])), (node, g, r)
            if g[1:] != r[1:]:
                ties += 1
                assert abs(apps.split_cost(inputs[g[1]], g[2], crit, nl) - r[0]) <= rtol * max(1.0, abs(r[0])), (node, g, r)
        return ties

    # the loop alone: the oracle's aggregates as its inputs
    agree(lmfao.best_splits_from_arrays(inputs, len(level.nodes), criterion, nl), 1e-12)
    # end to end on the engine's results: counts are exact, sums within 1e-6
    agree(lmfao.best_splits(eng, list(range(len(qs))), [i // (len(qs) // len(level.nodes)) for i in range(len(qs))],
                            criterion, nl), 1e-6)
