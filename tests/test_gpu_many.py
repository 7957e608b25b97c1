"""Parity of many-to-many joins (count-weighted views) with the oracle.

A Yelp-like star (Section 4): Review facts joined with User and Business on
unique keys and with Category and Attribute on the repeated key
``business`` (0 to 2 * mean rows per business; businesses with none do not
join).  The engine evaluates the many-to-many children as count-weighted
views: per key their row count, fp32 means and fp64 within-key scatter; each
fact row stands for the product of its children's counts; covariance entries
of two attributes of one such child are completed from the scatter.  Counts
compare bit for bit, sums under tests/helpers.check_sums at 1e-6 (the FP32
covariance block; grouped tables are fp64 in every precision).
"""
import numpy as np
import pytest

import oracle
from datagen.configs import cont_attrs, covariance_queries, many_to_many_batch, many_to_many_database
from tests.helpers import compare_results

pytestmark = pytest.mark.gpu

RTOL = 1e-6


@pytest.mark.parametrize("n_fact,mean_cat,mean_attr,seed", [(200_003, 3, 2, 11), (61_001, 12, 1, 12), (3_001, 1, 1, 13)])
def test_many_to_many_star_parity(n_fact, mean_cat, mean_attr, seed):
    from paper_1906_08687_amd.lmfao import Engine
    db = many_to_many_database(n_fact=n_fact, n_users=5_000, n_business=2_000, mean_cat=mean_cat,
                               mean_attr=mean_attr, seed=seed)
    qs = many_to_many_batch(db)
    print("case: many-to-many star, relations %s, %d queries" % ([r.n_rows for r in db.relations], len(qs)), flush=True)
    ref = oracle.evaluate(db, qs)
    assert int(ref[[i for i, q in enumerate(qs) if not (q.groupby or q.where or q.aggs)][0]].counts[0]) > n_fact
    for sched in ("batched", "plain"):
        eng = Engine(db, qs, precision="fp32", schedule=sched)
        eng.run()
        compare_results(eng.results(), ref, qs, RTOL, "many-to-many fp32 %s" % sched)
        eng.run()   # a second execution starts from cleared per-key sums and weights
        compare_results(eng.results(), ref, qs, RTOL, "many-to-many fp32 %s, second run" % sched)


def test_many_to_many_tables_in_bf16_plans():
    """Without a covariance block the grouped tables (fp64) run in any precision."""
    from paper_1906_08687_amd.lmfao import Engine
    db = many_to_many_database(n_fact=100_003, seed=14)
    qs = many_to_many_batch(db)[len(covariance_queries(cont_attrs(db))):]
    ref = oracle.evaluate(db, qs)
    eng = Engine(db, qs, precision="bf16x6", schedule="batched")
    eng.run()
    compare_results(eng.results(), ref, qs, RTOL, "many-to-many tables bf16x6")


def test_weight_beyond_exact_range_is_reported():
    """One business with 70,000 category and 70,000 attribute rows: a review of
    it joins 4.9e9 tuples, beyond the weights the root scan counts exactly;
    sync reports TOO_LARGE instead of returning wrapped counts."""
    import torch
    from datagen import Column, Relation
    from paper_1906_08687_amd.lmfao import Engine, LmfaoError
    db = many_to_many_database(n_fact=5_000, n_users=100, n_business=1, mean_cat=1, mean_attr=1, seed=15)
    for name in ("Category", "Attribute"):
        r = db.rel(name)
        n = 70_000
        cols = [Column("business", "key_many", np.zeros(n, np.int32), 1)]
        cols += [Column(c.attr, "cont", np.full(n, 0.5, np.float32)) for c in r.columns if c.kind == "cont"]
        db.relations[db.index(name)] = Relation(name, cols)
    qs = [q for q in many_to_many_batch(db) if not q.groupby and not q.where and not q.aggs]
    eng = Engine(db, qs, precision="fp32", schedule="batched")
    with pytest.raises(LmfaoError) as e:
        eng.run()
        eng.results()
    assert e.value.code == "TOO_LARGE"
    torch.cuda.synchronize()
