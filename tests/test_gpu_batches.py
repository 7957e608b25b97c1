"""Parity with the oracle on the batch shapes beyond the five workloads: a
three-dimensional data cube with five measures over workload 2's schema
(Section 2, equation (6): one group-by per subset of the dimensions), and a
classification-tree level over workload 3's schema (equations (9) and (10):
per node and split attribute, COUNT GROUP BY (label, bucket) and COUNT GROUP
BY bucket).  Both run on the general root scan (grouped tables; no
covariance block), in the batched and the plain schedule, with the coarser
tables derived from finer ones after the scan and with every table scanned.

Counts are bit-exact; sums follow tests/helpers.check_sums at 1e-6.
"""
import pytest

import oracle
from datagen import make_database
from datagen.configs import classification_tree_batch, data_cube_batch, tree_level
from tests.test_batches import CUBE_DIMS, CUBE_MEASURES
from tests.test_gpu_parity import compare

pytestmark = pytest.mark.gpu

_cache = {}


def _batch(name):
    if name not in _cache:
        if name == "cube":
            db = make_database(2, n_fact=100_003)
            qs = data_cube_batch(CUBE_DIMS, CUBE_MEASURES)
        else:
            db = make_database(3, n_fact=30_011)
            qs = classification_tree_batch(db, "g3", tree_level(db, n_nodes=8, seed=3))
        _cache[name] = (db, qs, oracle.evaluate(db, qs))
    return _cache[name]


@pytest.mark.parametrize("rollup", [True, False], ids=["derived", "scanned"])
@pytest.mark.parametrize("schedule", ["batched", "batched-no-codes", "plain"])
@pytest.mark.parametrize("name", ["cube", "classification_tree"])
def test_batch_parity(name, schedule, rollup):
    from paper_1906_08687_amd.lmfao import Engine
    db, qs, ref = _batch(name)
    print("case: %s %s rollup=%s, %d fact rows, %d queries" % (name, schedule, rollup, db.relations[0].n_rows, len(qs)),
          flush=True)
    codes = schedule != "batched-no-codes"
    eng = Engine(db, qs, precision="fp32", schedule=schedule.split("-")[0], rollup=rollup, row_codes=codes)
    st = eng.ctx.stats()
    assert (st["derived_tables"] > 0) == rollup
    if name == "classification_tree" and schedule != "plain":
        assert st["strided_families"] >= 1      # the per-node tables use the strided LDS layout
        assert st["code_scan"] == int(codes)
    eng.run()
    compare(eng.results(), ref, qs, 1e-6, "%s %s" % (name, schedule))


@pytest.mark.parametrize("name", ["cube", "classification_tree"])
def test_derived_tables_match_scanned_tables(name):
    """Summing a finer table after the scan gives the same counts as updating
    the coarser table per row, and sums equal up to the order of fp64
    additions."""
    import numpy as np
    from paper_1906_08687_amd.lmfao import Engine
    db, qs, _ = _batch(name)
    print("case: %s derived vs scanned" % name, flush=True)
    res = []
    for rollup in (True, False):
        eng = Engine(db, qs, precision="fp32", schedule="batched", rollup=rollup)
        eng.run()
        res.append(eng.results())
    for a, b in zip(*res):
        np.testing.assert_array_equal(a.counts, b.counts)
        np.testing.assert_allclose(a.sums, b.sums, rtol=1e-9, atol=1e-6)


def test_classification_tree_every_tile_candidate_agrees():
    """Every tile candidate of the tree level (tables in global memory, greedy
    LDS, LDS partitions; the partitioned ones replayed from per-row codes)
    gives the oracle's counts."""
    from paper_1906_08687_amd.lmfao import Engine
    db, qs, ref = _batch("classification_tree")
    eng = Engine(db, qs, precision="fp32", schedule="batched")
    assert eng.ctx.stats()["code_scan"] == 1
    seen = set()
    for i, cfg in enumerate(eng.ctx.candidates()):
        print("case: classification_tree candidate %d %s" % (i, cfg), flush=True)
        eng.ctx.select_candidate(i)
        eng._bind()
        seen.add(eng.ctx.stats()["code_scan"])
        eng.run()
        compare(eng.results(), ref, qs, 1e-6, "candidate %s" % cfg)
    assert seen == {0, 1}


def test_classification_tree_over_32_nodes_uses_two_mask_columns():
    """40 nodes are 40 filters: the per-row codes carry the filter mask in two
    columns (bits 0-31 and 32-63); counts still match the oracle."""
    from datagen import make_database
    from paper_1906_08687_amd.lmfao import Engine
    db = make_database(3, n_fact=30_011)
    qs = classification_tree_batch(db, "g3", tree_level(db, n_nodes=40, seed=5))
    ref = oracle.evaluate(db, qs)
    print("case: classification_tree 40 nodes, %d queries" % len(qs), flush=True)
    eng = Engine(db, qs, precision="fp32", schedule="batched")
    st = eng.ctx.stats()
    assert st["filters"] == 40 and st["code_scan"] == 1
    eng.run()
    compare(eng.results(), ref, qs, 1e-6, "classification_tree 40 nodes")


def test_tree_levels_of_two_kinds_share_one_code_scan():
    """A classification-tree level and a regression-tree level over the same
    nodes: two strided families (counts; counts with SUM(y), SUM(y^2)) whose
    key cells and y value come from one set of per-row codes."""
    from datagen import make_database
    from datagen.configs import batch3
    from paper_1906_08687_amd.lmfao import Engine
    db = make_database(3, n_fact=30_011)
    level = tree_level(db, n_nodes=8, seed=3)
    qs = classification_tree_batch(db, "g3", level) + batch3(db, level)
    ref = oracle.evaluate(db, qs)
    print("case: two tree levels, %d queries" % len(qs), flush=True)
    eng = Engine(db, qs, precision="fp32", schedule="batched")
    st = eng.ctx.stats()
    assert st["code_scan"] == 1 and st["strided_families"] == 2
    eng.run()
    compare(eng.results(), ref, qs, 1e-6, "two tree levels")
