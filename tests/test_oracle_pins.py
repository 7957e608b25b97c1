"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these retypes the oracle's formulas: each compares it with another
route to the same quantity (an exact rational brute force over the cross
product, closed forms, numpy library routines on an independently
materialised join, invariants, and a hand-computed fixture).
"""
import json
import math
import os
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle
from datagen import Agg, Column, Database, GroupBy, Pred, Query, Relation, make_batch, make_database
from datagen import rng as R
from datagen.configs import cat_attrs, cont_attrs, tree_level, zipf_cdf
from tests.helpers import materialize

HERE = os.path.dirname(os.path.abspath(__file__))


# --------------------------------------------------------------------------
# the seeded generator (shared input module) against its numpy restatement
# --------------------------------------------------------------------------

def test_rng_native_matches_numpy_restatement():
    g = R.native()
    for seed, name in [(1, "F.x1"), (4, "D1.d1_3"), (123456789, "thresholds.x1")]:
        key = g.key(seed, name)
        assert key == R.ref_key(seed, name)
        assert np.array_equal(g.u64(key, 1000), R.ref_u64(key, 1000))
        assert np.array_equal(g.unit(key, 1000), R.ref_unit(key, 1000))
        a, b = g.normal_f32(key, 1000, 100.0, 1.0), R.ref_normal_f32(key, 1000, 100.0, 1.0)
        assert np.max(np.abs(a.view(np.int32).astype(np.int64) - b.view(np.int32).astype(np.int64))) <= 1
        assert np.array_equal(g.uniform_i32(key, 1000, 3, 17), R.ref_uniform_i32(key, 1000, 3, 17))
        cdf = zipf_cdf(50, 1.2)
        assert np.array_equal(g.from_cdf_i32(key, 5000, cdf), R.ref_from_cdf_i32(key, 5000, cdf))


def test_rng_distributions():
    g = R.native()
    x = g.normal_f32(g.key(9, "n"), 200_000, 0.0, 1.0).astype(np.float64)
    assert abs(x.mean()) < 0.01 and abs(x.std() - 1.0) < 0.01
    k = g.from_cdf_i32(g.key(9, "z"), 200_000, zipf_cdf(100, 1.2))
    freq = np.bincount(k, minlength=100) / 200_000.0
    p = np.arange(1, 101, dtype=np.float64) ** -1.2
    p /= p.sum()
    assert np.max(np.abs(freq - p)) < 0.005


def test_radix_sort_and_fact_order():
    g = R.native()
    v = g.u64(g.key(3, "s"), 100_001) >> np.uint64(7)
    assert np.array_equal(g.sort_u64(v.copy()), np.sort(v))
    db = make_database(2)
    F = db.relations[0]
    # foreign keys sorted lexicographically, smallest dimension first (Section 3.5 attribute order)
    dims = sorted([(db.rel(n).n_rows, k) for n, k in [("D1", "k1"), ("D2", "k2"), ("D3", "k3"), ("D4", "k4")]])
    keys = [F.col(k).data for _, k in dims]
    assert np.array_equal(np.lexsort(keys[::-1]), np.arange(F.n_rows))


# --------------------------------------------------------------------------
# exact brute force over the cross product (tiny inputs)
# --------------------------------------------------------------------------

def _tiny_db(rnd: random.Random):
    """2-5 relations, <= 7 rows each, keys from a tiny range (non-unique and
    dangling keys included), tree shaped as a random star/snowflake."""
    m = rnd.randint(2, 5)
    rels, edges = [], []
    keyname = {}
    for r in range(m):
        n = rnd.randint(1, 7)
        cols = []
        if r > 0:
            p = rnd.randrange(r)
            edges.append((p, r))
            keyname[r] = "k%d" % r
            cols.append(Column(keyname[r], "key", np.array([rnd.randrange(3) for _ in range(n)], np.int32), 3))
        rels.append((n, cols))
    for p, c in edges:
        n, cols = rels[p]
        cols.append(Column(keyname[c], "key", np.array([rnd.randrange(3) for _ in range(n)], np.int32), 3))
    out = []
    for r, (n, cols) in enumerate(rels):
        for j in range(rnd.randint(1, 2)):
            vals = [rnd.choice([-2.5, -1.0, 0.0, 0.5, 1.25, 3.0, 1e3 + 0.125, 7.0 / 3.0]) for _ in range(n)]
            cols.append(Column("x%d_%d" % (r, j), "cont", np.array(vals, np.float32)))
        cols.append(Column("c%d" % r, "cat", np.array([rnd.randrange(3) for _ in range(n)], np.int32), 3))
        out.append(Relation("R%d" % r, cols))
    return Database(out, edges)


def _tiny_queries(db, rnd: random.Random):
    conts = cont_attrs(db)
    cats = cat_attrs(db)
    qs = [Query()]
    for _ in range(6):
        gb = []
        if rnd.random() < 0.6:
            gb.append(GroupBy(rnd.choice(cats)))
        if rnd.random() < 0.4:
            gb.append(GroupBy(rnd.choice(conts), np.array([-1.0, 0.5, 3.0], np.float32)))
        where = []
        if rnd.random() < 0.5:
            where.append(Pred(rnd.choice(conts), rnd.choice(["le", "lt", "ge", "gt", "eq", "ne"]),
                              rnd.choice([0.0, 0.5, 1.25])))
        if rnd.random() < 0.3:
            where.append(Pred(rnd.choice(cats), rnd.choice(["eq", "ne"]), rnd.randrange(3)))
        aggs = [Agg.monomial(), Agg.monomial(rnd.choice(conts)),
                Agg.monomial(rnd.choice(conts), rnd.choice(conts)),
                Agg([(2.0, (rnd.choice(conts),)), (-0.5, (rnd.choice(conts), rnd.choice(conts)))])]
        qs.append(Query(gb, where, aggs))
    return qs


@pytest.mark.parametrize("seed", range(12))
def test_oracle_equals_exact_brute_force(seed):
    rnd = random.Random(seed)
    db = _tiny_db(rnd)
    qs = _tiny_queries(db, rnd)
    got = oracle.evaluate(db, qs, n_threads=3)
    exact = oracle.brute_force(db, qs)
    for q, g, (cnt, sums, abs_sums) in zip(qs, got, exact):
        assert list(g.counts) == cnt
        for cell in range(len(cnt)):
            for a in range(len(q.aggs)):
                ref = float(sums[cell][a])      # correctly rounded exact value
                assert abs(g.sums[cell, a] - ref) <= 2 * math.ulp(max(abs(ref), 1e-300)) or g.sums[cell, a] == ref
                # the conditioning scale sum |term|: every term is exact in fp64 and non-negative, so a
                # plain fp64 sum of n terms is within (n - 1) ulp of the exact value
                aref = float(abs_sums[cell][a])
                n_terms = cnt[cell] * len(q.aggs[a].terms)
                assert abs(g.abs_sums[cell, a] - aref) <= max(n_terms, 2) * math.ulp(max(aref, 1e-300))


def test_oracle_golden_moo_example():
    """Hand-computed results on the Section 3.5 schema (composite join key
    (date, store) with duplicates: bag semantics)."""
    fx = json.load(open(os.path.join(HERE, "golden", "moo_example.json")))
    names = list(fx["relations"])
    rels = []
    for name in names:
        cols = []
        for attr, vals in fx["relations"][name].items():
            kind = fx["kinds"][attr]
            dt = np.float32 if kind == "cont" else np.int32
            cols.append(Column(attr, kind, np.array(vals, dt), fx["domains"].get(attr, 0)))
        rels.append(Relation(name, cols))
    db = Database(rels, [(names.index(p), names.index(c)) for p, c in fx["edges"]])
    qs = []
    for q in fx["queries"]:
        qs.append(Query([GroupBy(g) for g in q["groupby"]], [Pred(a, op, v) for a, op, v in q["where"]],
                        [Agg.monomial(*a) for a in q["aggs"]]))
    for q, spec, res in zip(qs, fx["queries"], oracle.evaluate(db, qs, n_threads=2)):
        assert list(res.counts) == spec["counts"]
        assert np.array_equal(res.sums, np.array(spec["sums"], np.float64))
    # the brute force agrees on the same fixture
    for spec, (cnt, sums, _) in zip(fx["queries"], oracle.brute_force(db, qs)):
        assert cnt == spec["counts"]
        assert [[float(s) for s in row] for row in sums] == spec["sums"]


# --------------------------------------------------------------------------
# closed forms and library routines on the generated workloads
# --------------------------------------------------------------------------

def test_count_is_fact_size_and_dim_sums_by_bincount():
    db = make_database(1)
    F = db.relations[0]
    qs = [Query(), Query(aggs=[Agg.monomial("y2")]), Query(aggs=[Agg.monomial("z1", "y3")])]
    res = oracle.evaluate(db, qs, n_threads=4)
    # every foreign key resolves against a dense key, so |J| = |F|
    assert int(res[0].counts[0]) == F.n_rows
    # SUM over a dimension attribute = sum_k cnt_F(k) * y(k), exact with fsum
    cnt = np.bincount(F.col("a").data, minlength=db.rel("D1").n_rows).astype(np.float64)
    y = db.rel("D1").col("y2").data.astype(np.float64)
    ref = math.fsum(cnt * y)
    assert abs(res[1].sums[0, 0] - ref) <= 2 * math.ulp(ref)
    J = materialize(db)
    ref2 = math.fsum(J["z1"] * J["y3"])          # fp32*fp32 products are exact in fp64
    assert abs(res[2].sums[0, 0] - ref2) <= 2 * math.ulp(abs(ref2))


def test_abs_sums_equal_fsum_of_absolute_terms():
    """Sum |term| (the scale of the tolerance rule) on workload 1's materialised join:
    each term coeff * prod x on its own, not |aggregate| per tuple.  The mixed-sign
    aggregate separates the two (|2 x1 - 0.5 x2 y1| <= |2 x1| + |0.5 x2 y1|)."""
    db = make_database(1, n_fact=30_011)
    J = materialize(db)
    mixed = Agg([(2.0, ("x1",)), (-0.5, ("x2", "y1"))])
    qs = [Query(aggs=[Agg.monomial("x1", "z1"), mixed, Agg.monomial()]),
          Query([GroupBy("c")], [Pred("z2", "gt", 0.0)], [mixed, Agg([(3.0, ())])])]
    res = oracle.evaluate(db, qs, n_threads=4)
    t1 = np.abs(2.0 * J["x1"])
    t2 = np.abs(-0.5 * J["x2"] * J["y1"])           # products of two fp32 values are exact in fp64
    n = len(J["x1"])
    for got, ref in [(res[0].abs_sums[0, 0], math.fsum(np.abs(J["x1"] * J["z1"]))),
                     (res[0].abs_sums[0, 1], math.fsum(np.concatenate([t1, t2]))),
                     (res[0].abs_sums[0, 2], float(n))]:
        assert abs(got - ref) <= n * math.ulp(ref)
    partial = math.fsum(np.abs(2.0 * J["x1"] - 0.5 * J["x2"] * J["y1"]))
    assert res[0].abs_sums[0, 1] > partial * (1 + 1e-3)
    m = J["z2"].astype(np.float32) > np.float32(0.0)
    for v in range(db.column("c").domain):
        sel = m & (J["c"] == v)
        ref = math.fsum(np.concatenate([t1[sel], t2[sel]]))
        assert abs(res[1].abs_sums[v, 0] - ref) <= n * math.ulp(max(ref, 1e-300))
        assert res[1].abs_sums[v, 1] == 3.0 * sel.sum()


def test_covariance_matches_fsum_and_is_symmetric_psd():
    db = make_database(1)
    J = materialize(db)
    conts = cont_attrs(db)
    qs = [Query(aggs=[Agg.monomial(conts[i], conts[j]) for j in range(len(conts))]) for i in range(len(conts))]
    res = oracle.evaluate(db, qs, n_threads=4)
    G = np.array([r.sums[0] for r in res])
    for i in range(len(conts)):
        for j in range(len(conts)):
            ref = math.fsum(J[conts[i]] * J[conts[j]])
            assert abs(G[i, j] - ref) <= 2 * math.ulp(abs(ref))
    assert np.array_equal(G, G.T)
    X = np.stack([np.ones_like(J[conts[0]])] + [J[c] for c in conts], axis=1)
    Aug = np.zeros((len(conts) + 1, len(conts) + 1))
    Aug[1:, 1:] = G
    Aug[0, 0] = len(J[conts[0]])
    Aug[0, 1:] = Aug[1:, 0] = [oracle.evaluate(db, [Query(aggs=[Agg.monomial(c)])])[0].sums[0, 0] for c in conts]
    np.testing.assert_allclose(Aug, X.T @ X, rtol=1e-12)
    assert np.linalg.eigvalsh(Aug).min() > -1e-9 * np.abs(Aug).max()


def test_groupby_counts_and_pair_marginals():
    db = make_database(2)
    J = materialize(db)
    cats = sorted(cat_attrs(db))
    dom = {c: db.column(c).domain for c in cats}
    qs = [Query(groupby=[GroupBy(c)], aggs=[Agg.monomial("f1"), Agg.monomial("s2")]) for c in cats]
    qs += [Query(groupby=[GroupBy(cats[0]), GroupBy(cats[3])])]
    res = oracle.evaluate(db, qs, n_threads=4)
    n = len(J["f1"])
    for c, r in zip(cats, res):
        assert np.array_equal(r.counts, np.bincount(J[c], minlength=dom[c]).astype(np.uint64))
        assert int(r.counts.sum()) == n
        for a, attr in enumerate(["f1", "s2"]):
            for v in range(dom[c]):
                ref = math.fsum(J[attr][J[c] == v])
                assert abs(r.sums[v, a] - ref) <= 2 * math.ulp(abs(ref)) + 1e-300
    pair = res[-1].counts.reshape(dom[cats[0]], dom[cats[3]])
    assert np.array_equal(pair.sum(axis=1), res[0].counts)
    assert np.array_equal(pair.sum(axis=0), res[3].counts)
    flat = J[cats[0]] * dom[cats[3]] + J[cats[3]]
    assert np.array_equal(res[-1].counts, np.bincount(flat, minlength=dom[cats[0]] * dom[cats[3]]).astype(np.uint64))


def _mask(J, preds):
    m = np.ones(len(J["y"]), bool)
    for p in preds:
        x = J[p.attr]
        if p.attr.startswith(("x", "u", "v", "w")):
            x = x.astype(np.float32)
            t = np.float32(p.value)
        else:
            t = float(p.value)
        m &= {"le": x <= t, "lt": x < t, "ge": x >= t, "gt": x > t, "eq": x == t, "ne": x != t}[p.op]
    return m


def test_regression_tree_level_invariants():
    db = make_database(3)
    J = materialize(db)
    level = tree_level(db)
    nodes = level.nodes[:6]
    feats = level.features
    qs = []
    for preds in nodes:
        for a in feats:
            qs.append(Query([GroupBy(a, level.thresholds.get(a))], list(preds),
                            [Agg.monomial("y"), Agg.monomial("y", "y")]))
    res = oracle.evaluate(db, qs, n_threads=4)
    for ni, preds in enumerate(nodes):
        m = _mask(J, preds)
        for fi, a in enumerate(feats):
            r = res[ni * len(feats) + fi]
            # every attribute's buckets partition the node's tuples
            assert int(r.counts.sum()) == int(m.sum())
            if a in level.thresholds:
                # bucket = #{t_k < x}: np.searchsorted(..., side="left") is that count
                b = np.searchsorted(level.thresholds[a], J[a][m].astype(np.float32), side="left")
                assert np.array_equal(r.counts, np.bincount(b, minlength=21).astype(np.uint64))
            # per-cell variance numerator sum y^2 - (sum y)^2 / n is non-negative
            n = r.counts.astype(np.float64)
            with np.errstate(divide="ignore", invalid="ignore"):
                var = np.where(n > 0, r.sums[:, 1] - r.sums[:, 0] ** 2 / np.maximum(n, 1), 0.0)
            assert np.all(var >= -1e-9 * np.maximum(r.sums[:, 1], 1.0))
    # adding a conjunct never increases a count
    extra = Pred("x1", "le", 0.0)
    q0 = Query([GroupBy("g1")], list(nodes[0]), [])
    q1 = Query([GroupBy("g1")], list(nodes[0]) + [extra], [])
    r0, r1 = oracle.evaluate(db, [q0, q1])
    assert np.all(r1.counts <= r0.counts)


def test_bucket_and_predicate_boundaries():
    """x equal to a threshold falls in the bucket of that threshold (x <= t_k
    <=> bucket <= k), and strict/non-strict predicates differ exactly there."""
    F = Relation("F", [Column("x", "cont", np.array([-1.0, 0.5, 0.5, 1.0, 2.0, 9.0], np.float32)),
                       Column("c", "cat", np.array([0, 1, 1, 0, 1, 0], np.int32), 2)])
    db = Database([F], [])
    th = np.array([0.5, 1.0, 2.0], np.float32)
    qs = [Query([GroupBy("x", th)]), Query(where=[Pred("x", "le", 0.5)]), Query(where=[Pred("x", "lt", 0.5)]),
          Query(where=[Pred("x", "gt", 1.0)]), Query(where=[Pred("x", "ge", 1.0)]),
          Query([GroupBy("c")], [Pred("c", "ne", 1)], [Agg.monomial("x")])]
    r = oracle.evaluate(db, qs)
    assert list(r[0].counts) == [3, 1, 1, 1]
    assert [int(q.counts[0]) for q in r[1:5]] == [3, 1, 2, 3]
    assert list(r[5].counts) == [3, 0] and r[5].sums[0, 0] == 9.0 and r[5].sums[1, 0] == 0.0


def test_integer_predicates_against_real_constants():
    """1[c op v] on an integer attribute compares c with the real number v:
    c >= 2.5 is c >= 3, c < 2.5 is c <= 2, c = 2.5 never holds, c != 2.5 always
    does, and constants beyond the int32 range hold for all or no rows."""
    F = Relation("F", [Column("c", "cat", np.array([0, 1, 2, 3, 4, 2, 3, 9], np.int32), 10)])
    db = Database([F], [])
    c = F.col("c").data
    cases = [("ge", 2.5, c >= 3), ("gt", 2.5, c >= 3), ("le", 2.5, c <= 2), ("lt", 2.5, c <= 2),
             ("eq", 2.5, c < -1), ("ne", 2.5, c >= 0), ("ge", -0.5, c >= 0), ("lt", 3.0, c <= 2),
             ("le", 1e12, c >= 0), ("gt", -1e12, c >= 0), ("lt", -1e12, c < -1), ("ge", 3e9, c < -1),
             ("eq", 3.0, c == 3), ("ne", 3.0, c != 3)]
    res = oracle.evaluate(db, [Query(where=[Pred("c", op, v)]) for op, v, _ in cases])
    for (op, v, m), r in zip(cases, res):
        assert int(r.counts[0]) == int(m.sum()), (op, v)
    exact = oracle.brute_force(db, [Query(where=[Pred("c", op, v)]) for op, v, _ in cases])
    assert [e[0][0] for e in exact] == [int(m.sum()) for _, _, m in cases]


def test_thread_count_does_not_change_results():
    db = make_database(4, n_fact=20_011)
    qs = make_batch(4, db)[:60]
    a = oracle.evaluate(db, qs, n_threads=1)
    b = oracle.evaluate(db, qs, n_threads=7)
    for x, y in zip(a, b):
        assert np.array_equal(x.counts, y.counts)
        np.testing.assert_allclose(x.sums, y.sums, rtol=4e-16, atol=0)


def test_aggregate_count_formulas():
    """Section 2: (n+1)(n+2)/2 aggregates for linear regression over n
    attributes; n(n-1)/2 pairs for Chow-Liu; d*n*(p+1)*c for trees."""
    for k, n in [(1, 9), (4, 40)]:
        db = make_database(k) if k == 1 else make_database(4, n_fact=1000, dims=(10, 10, 10, 10))
        qs = [q for q in make_batch(k, db) if not q.groupby]
        assert len(qs) == (n + 1) * (n + 2) // 2
    db = make_database(5, n_fact=1000, dims=(10, 10, 10))
    pairs = [q for q in make_batch(5, db) if len(q.groupby) == 2]
    assert len(pairs) == 15 * 14 // 2
    db = make_database(3, n_fact=1000, dims=(10, 10, 10))
    qs = make_batch(3, db)
    assert len(qs) == 32 * 30
    # RT: 32 nodes x 30 attributes x (COUNT + 2 sums) grouped by bucket
    assert sum(len(q.aggs) + 1 for q in qs) == 32 * 30 * 3


def test_polynomial_moments_match_the_gram_of_the_monomial_vector():
    """Degree-2 polynomial regression (Section 2): the batch's aggregates are the
    entries of U^T U for U = [1, x_i, x_i x_j] over the materialised join
    (numpy, math.fsum), ((C^2 + C) / 2 of them for C = C(n+2, 2))."""
    from datagen.configs import polynomial_queries
    db = make_database(1, n_fact=4_001)
    J = materialize(db)
    attrs = cont_attrs(db)[:4]
    qs = polynomial_queries(attrs)
    C = math.comb(len(attrs) + 2, 2)
    assert len(qs) == (C * C + C) // 2
    res = oracle.evaluate(db, qs, n_threads=4)
    cols = [np.ones(len(J[attrs[0]]))] + [J[a] for a in attrs]
    cols += [J[attrs[i]] * J[attrs[j]] for i in range(len(attrs)) for j in range(i, len(attrs))]
    k = 0
    for a in range(len(cols)):
        for b in range(a, len(cols)):
            r = res[k]
            prod = cols[a] * cols[b]
            if not qs[k].aggs:
                assert int(r.counts[0]) == len(prod)
            else:
                ref = math.fsum(prod)
                # the oracle forms each product of up to four fp32 values in fp64 (rounded once or twice)
                assert abs(r.sums[0, 0] - ref) <= 1e-14 * math.fsum(np.abs(prod)) + 1e-300
                assert abs(r.abs_sums[0, 0] - math.fsum(np.abs(prod))) <= 1e-12 * r.abs_sums[0, 0]
            k += 1


def test_oracle_many_to_many_star_matches_brute_force_and_closed_form_count():
    """A Yelp-like star whose Category and Attribute children repeat the join
    key (bag semantics of the natural join): the oracle equals the exact
    brute force on every query of the many-to-many batch, and the size of the
    join is sum over reviews of (categories x attributes of the business), a
    closed form from per-key row counts."""
    from datagen.configs import many_to_many_batch, many_to_many_database
    db = many_to_many_database(n_fact=60, n_users=6, n_business=5, mean_cat=2, mean_attr=1, seed=3)
    qs = many_to_many_batch(db)
    got = oracle.evaluate(db, qs, n_threads=2)
    exact = oracle.brute_force(db, qs)
    for q, g, (cnt, sums, _) in zip(qs, got, exact):
        assert list(g.counts) == cnt
        for cell in range(len(cnt)):
            for a in range(len(q.aggs)):
                ref = float(sums[cell][a])
                assert abs(g.sums[cell, a] - ref) <= 2 * math.ulp(max(abs(ref), 1e-300))
    b = db.rel("Review").col("business").data
    n_cat = np.bincount(db.rel("Category").col("business").data, minlength=5)
    n_att = np.bincount(db.rel("Attribute").col("business").data, minlength=5)
    count = [i for i, q in enumerate(qs) if not q.groupby and not q.where and not q.aggs]
    total = int(np.sum(n_cat[b].astype(np.int64) * n_att[b]))
    assert total > 0 and int(got[count[0]].counts[0]) == total
