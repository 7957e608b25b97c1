"""Pins of the oracle on the batch shapes beyond the five workloads: a data
cube (Section 2, equation (6)) and a classification-tree level (equations (9)
and (10)).  Each compares answers the definitions tie together, so that a
wrong cell index, a dropped condition or a misplaced label fails:

* cube: summing a group-by over one of its dimensions gives the group-by
  without it; the empty group-by's count is the size of the join (every
  foreign key resolves), and its sums match a numpy sum over the joined
  measure columns;
* classification tree: summing COUNT GROUP BY (label, X) over the label gives
  COUNT GROUP BY X; for one node every split attribute's buckets add up to
  the same count, which equals a direct count of the rows satisfying the
  node's conditions on the materialised join.
"""
import numpy as np

import oracle
from datagen import make_database
from datagen.configs import classification_tree_batch, data_cube_batch, tree_level
from tests.helpers import materialize

CUBE_DIMS = ["c0", "c1", "c4"]           # one categorical attribute of the fact and of two dimensions
CUBE_MEASURES = ["f1", "f2", "d1_1", "d2_1", "d4_1"]


def _grid(db, q, res):
    doms = [g.domain(db) for g in q.groupby]
    return res.counts.reshape(doms or [1]), res.sums.reshape((doms or [1]) + [res.sums.shape[1]])


def test_data_cube_is_marginally_consistent():
    db = make_database(2, n_fact=20_011)
    qs = data_cube_batch(CUBE_DIMS, CUBE_MEASURES)
    assert len(qs) == 2 ** len(CUBE_DIMS)
    ref = oracle.evaluate(db, qs)
    by_mask = {}
    for q, r in zip(qs, ref):
        mask = sum(1 << CUBE_DIMS.index(g.attr) for g in q.groupby)
        by_mask[mask] = (q, r)
    for mask, (q, r) in by_mask.items():
        cnt, sm = _grid(db, q, r)
        for i in range(len(CUBE_DIMS)):
            if (mask >> i) & 1:
                continue
            q2, r2 = by_mask[mask | (1 << i)]
            cnt2, sm2 = _grid(db, q2, r2)
            axis = sum(1 for j in range(i) if (mask >> j) & 1)    # position of dimension i in q2's group-by
            np.testing.assert_array_equal(cnt2.sum(axis=axis), cnt.reshape(cnt2.sum(axis=axis).shape))
            np.testing.assert_allclose(sm2.sum(axis=axis), sm.reshape(sm2.sum(axis=axis).shape), rtol=1e-12, atol=1e-9)
    q0, r0 = by_mask[0]
    assert int(r0.counts[0]) == db.relations[0].n_rows
    J = materialize(db)
    for k, m in enumerate(CUBE_MEASURES):
        assert np.isclose(r0.sums[0, k], float(np.sum(J[m].astype(np.float64))), rtol=1e-12)


def test_classification_tree_counts_split_by_label_and_attribute():
    db = make_database(3, n_fact=10_007)
    level = tree_level(db, n_nodes=4, seed=3)
    label = "g3"
    qs = classification_tree_batch(db, label, level)
    feats = [a for a in level.features if a != label]
    assert len(qs) == 2 * len(level.nodes) * len(feats)
    ref = oracle.evaluate(db, qs)
    J = materialize(db)
    dom_label = db.column(label).domain
    for n, preds in enumerate(level.nodes):
        keep = np.ones(len(J[label]), bool)
        for p in preds:
            x = J[p.attr]
            t = np.float32(p.value) if x.dtype.kind == "f" else float(p.value)
            keep &= {"le": x <= t, "gt": x > t, "eq": x == t, "ne": x != t}[p.op]
        node_count = int(keep.sum())
        for j, a in enumerate(feats):
            i = 2 * (n * len(feats) + j)
            with_label, alone = ref[i], ref[i + 1]
            assert [g.attr for g in qs[i].groupby] == [label, a] and [g.attr for g in qs[i + 1].groupby] == [a]
            per = with_label.counts.reshape(dom_label, -1)
            np.testing.assert_array_equal(per.sum(axis=0), alone.counts)
            assert int(alone.counts.sum()) == node_count
            # the label's class totals equal a direct count on the join
            np.testing.assert_array_equal(per.sum(axis=1), np.bincount(J[label][keep], minlength=dom_label))


def test_planner_derives_coarser_tables_of_the_batches():
    """Which tables the planner derives after the scan instead of updating
    per row, on the batch shapes: the cube's lattice leaves one scanned table;
    a tree level's COUNT GROUP BY bucket comes from the label-split counts;
    the mutual-information marginals come from the pair counts; workload 2's
    SUM(x) GROUP BY c tables stay scanned (the pair counts carry no sums)."""
    from datagen import make_batch
    from tests.test_abi import _plan_db
    db = make_database(2, n_fact=20_011)
    st = _plan_db(db, data_cube_batch(CUBE_DIMS, CUBE_MEASURES)).stats()
    assert (st["tables"], st["derived_tables"]) == (7, 6)
    assert _plan_db(db, make_batch(2, db)).stats()["derived_tables"] == 0
    db3 = make_database(3, n_fact=10_007)
    qs = classification_tree_batch(db3, "g3", tree_level(db3, n_nodes=4, seed=3))
    st = _plan_db(db3, qs).stats()
    assert st["derived_tables"] * 2 == st["tables"] == len(qs)
    db5 = make_database(5)
    st = _plan_db(db5, make_batch(5, db5)).stats()
    assert (st["tables"], st["derived_tables"]) == (120, 15)
