"""Parity of the dedicated covariance scan (BF16 split on MFMA) over the slot
layouts it distinguishes: fact-only tiles, a fact tile shared with record
lanes, two fact tiles, four tiles, no fact features at all, a fact without a
ragged tail, records of one to five quads (a key uniform over a tile is
gathered once, others row by row), a key that changes on nearly every row,
large dimensions beside small ones, fact keys without a dimension row, and
every tile candidate of the autotuner (also over a 40,000-row dimension).  Record buffers take both layouts: pair rows when every record has
at most two quads (facts-only-tile, whole-tiles, distinct-keys, whose first
dimension has one-quad records), quad-major otherwise.

Counts are bit-exact.  Sums are checked twice:
  * against the oracle under the tolerance rule of tests/helpers.check_sums:
    1e-5 for BF16X6, the form the benchmark runs (three pieces, every term
    down to 2^-16 of a product kept; the worst measured error is 4e-7);
    BF16X3 and BF16X4 drop up to 3 and 2 times 2^-16 of a product
    (tests/test_split_bounds.py derives it), which a sum dominated by one
    repeated dimension value keeps, and are checked against that bound (plus
    the fp32 accumulation): a 20-row dimension under Zipf keys brings
    BF16X3 to 1.2e-5;
  * against the same split computed exactly (tests/helpers.split_gram), a
    check of the kernel's fp32 accumulation alone, not of parity: within
    5e-6 * sum|terms|.
"""
import numpy as np
import pytest

import oracle
from datagen.configs import AttrSpec, RelSpec, build_database, covariance_queries, cont_attrs
from datagen.schema import Database, Relation
from tests.helpers import check_sums, materialize, split_gram

pytestmark = pytest.mark.gpu

RTOL = {"bf16x6": 1e-5, "bf16x4": 2 * 2.0 ** -16 + 4e-6, "bf16x3": 3 * 2.0 ** -16 + 4e-6}
PRODUCTS = {"bf16x3": 3, "bf16x4": 4, "bf16x6": 6}
FULL = "bf16x6"       # the split the benchmark's full form runs
ACC = 5e-6

# (name, fact rows, fact features, [(dimension rows, features)], Zipf exponent of the keys)
SHAPES = [
    ("facts-only-tile", 50_003, 15, [], 0.0),
    ("mixed-fact-tile", 70_001, 5, [(1000, 8), (300, 8)], 1.1),
    ("two-fact-tiles", 65_537, 20, [(2000, 10), (500, 12)], 0.0),
    ("four-tiles", 40_017, 30, [(800, 15), (90, 15), (7, 3)], 1.2),
    ("no-fact-features", 30_011, 0, [(500, 7), (60, 9)], 0.0),
    ("whole-tiles", 64_000, 16, [(1000, 6), (100, 6)], 1.2),
    # a 19-word record (5 quads) beside a 6-word one
    ("wide-record", 30_007, 4, [(400, 18), (50, 5)], 1.1),
    # 400k keys under 40k rows: the key changes on nearly every row
    ("distinct-keys", 40_009, 3, [(50, 2), (400_000, 5)], 0.0),
    # two large dimensions (records gathered row by row) beside two small ones whose keys stay
    # the same over runs of the sorted fact (gathered once per tile, or kept from the last one)
    ("large-and-small-dims", 120_011, 12, [(60_000, 6), (300, 6), (20_000, 4), (9, 2)], 1.1),
]


def _star(seed, n_fact, n_feat, dims, zipf):
    ds = [RelSpec("D%d" % (i + 1), rows, [AttrSpec("d%d_%d" % (i + 1, j), "cont", ("normal", 3.0, 1.0))
                                          for j in range(nf)], key="k%d" % (i + 1)) for i, (rows, nf) in enumerate(dims)]
    fact = RelSpec("F", n_fact, [AttrSpec("f%d" % j, "cont", ("normal", 1.0, 2.0)) for j in range(n_feat)],
                   children=[(d, d.key) for d in ds], zipf_s={d.key: zipf for d in ds} if zipf else {})
    return build_database(seed, fact)


def _normwise(got, ref, scale, tol, what):
    err = np.abs(np.asarray(got, np.float64) - np.asarray(ref, np.float64))
    bad = err > tol * np.asarray(scale, np.float64)
    assert not bad.any(), "%s: %d sums outside %.1e * sum|terms|, worst ratio %.3e" % (
        what, int(bad.sum()), tol, float(np.max(err / np.maximum(scale, 1e-300))))


def _check(db, qs, eng, precision, what, emulate=True):
    ref = oracle.evaluate(db, qs)
    got = eng.results()
    for i, (g, r) in enumerate(zip(got, ref)):
        assert np.array_equal(g.counts, r.counts), "%s query %d: counts differ" % (what, i)
        if qs[i].aggs:
            check_sums(g.sums, r.sums, r.abs_sums, RTOL[precision], "%s query %d vs oracle" % (what, i))
    if emulate:
        conts = cont_attrs(db)
        J = materialize(db)
        G = split_gram([J[a] for a in conts], PRODUCTS[precision])
        idx = {a: k + 1 for k, a in enumerate(conts)}
        for i, (g, r) in enumerate(zip(got, ref)):
            if not qs[i].aggs:
                continue
            attrs = qs[i].aggs[0].terms[0][1]
            a = idx[attrs[0]]
            b = idx[attrs[1]] if len(attrs) > 1 else 0
            _normwise(g.sums[0, 0], G[a, b], r.abs_sums[0, 0], ACC, "%s query %d vs split" % (what, i))


@pytest.mark.parametrize("shape", SHAPES, ids=[s[0] for s in SHAPES])
@pytest.mark.parametrize("precision", ["bf16x3", "bf16x4", "bf16x6"])
def test_dedicated_scan_parity(shape, precision):
    from paper_1906_08687_amd.lmfao import Engine
    name, n_fact, n_feat, dims, zipf = shape
    db = _star(11, n_fact, n_feat, dims, zipf)
    qs = covariance_queries(cont_attrs(db))
    print("case: %s %s, %d fact rows, %d features" % (name, precision, n_fact, len(cont_attrs(db))), flush=True)
    eng = Engine(db, qs, precision=precision, schedule="batched")
    assert eng.stats()["dedicated_scan"] == 1
    eng.run()
    _check(db, qs, eng, precision, "%s %s" % (name, precision))


def test_dedicated_scan_dangling_keys():
    """Dimension rows removed after drawing: fact keys that lose their row do
    not join (their records read as zeros)."""
    from paper_1906_08687_amd.lmfao import Engine
    db = _star(12, 20_011, 6, [(700, 5), (40, 4)], 1.1)
    rels = list(db.relations)
    d1 = rels[1]
    keep = (d1.col("k1").data % 5) != 2
    cols = []
    for c in d1.columns:
        cols.append(type(c)(c.attr, c.kind, c.data[keep], c.domain))
    rels[1] = Relation(d1.name, cols)
    db = Database(rels, db.edges)
    qs = covariance_queries(cont_attrs(db))
    eng = Engine(db, qs, precision=FULL, schedule="batched")
    assert eng.stats()["dedicated_scan"] == 1
    eng.run()
    _check(db, qs, eng, FULL, "dangling", emulate=False)
    assert int(eng.results()[0].counts[0]) < 20_011


@pytest.mark.parametrize("dims", [[(3000, 6), (200, 6), (20, 6)], [(40_000, 6), (200, 6), (20, 6)]],
                         ids=["small-dims", "large-dim"])
def test_dedicated_scan_every_candidate_agrees(dims):
    from paper_1906_08687_amd.lmfao import Engine
    db = _star(13, 90_001, 16, dims, 1.2)
    qs = covariance_queries(cont_attrs(db))
    eng = Engine(db, qs, precision=FULL, schedule="batched")
    cands = eng.ctx.candidates()
    assert len(cands) >= 6
    counts0 = None
    for i, cfg in enumerate(cands):
        print("case: candidate %d %s" % (i, cfg), flush=True)
        eng.ctx.select_candidate(i)
        assert eng.stats()["dedicated_scan"] == 1
        eng._bind()
        eng.run()
        _check(db, qs, eng, FULL, "candidate %d" % i)
        c0 = int(eng.results()[0].counts[0])
        counts0 = c0 if counts0 is None else counts0
        assert c0 == counts0


def test_dedicated_scan_is_deterministic_across_runs_and_graph_replays():
    """Every wave writes its own partial and the merge sums them in a fixed order: repeated
    executions, eager and replayed from the captured graph, give bitwise-identical sums."""
    import torch
    from paper_1906_08687_amd.lmfao import Engine
    db = _star(14, 77_777, 16, [(5000, 6), (300, 6)], 1.2)
    qs = covariance_queries(cont_attrs(db))
    eng = Engine(db, qs, precision=FULL, schedule="batched")
    eng.run()                                   # eager (null stream)
    first = [r.sums.copy() for r in eng.results()]
    stream = torch.cuda.Stream()
    for rep in range(3):                        # the first captures the graph, then replays
        eng.run(stream)
        torch.cuda.synchronize()
        got = eng.results()
        for i, (g, f) in enumerate(zip(got, first)):
            assert np.array_equal(g.sums, f), "replay %d query %d differs" % (rep, i)
