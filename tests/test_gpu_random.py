"""Parity over the held-out random star/snowflake batches and over values
that sit exactly on thresholds and predicate constants.

The random batches are the cost model's evaluation set (workloads 150-199 of
``random_workload``: 2-6 relations in star or snowflake shape, mixed
covariance entries, grouped sums, pairwise counts and filtered sums; and
workloads 150-169 of ``random_covariance_workload``: covariance-only stars
on the dedicated BF16 scan, values N(100, 1)).  Every aggregate of every
batch is compared with the oracle: counts bit for bit, sums under
tests/helpers.check_sums at 1e-6 (fp32 with fp64 merge) and 1e-5 (bf16 hi+lo
split).  Each batch runs in the launch configuration the benchmark times
(bf16x6, batched schedule captured in a hipGraph, tiles chosen by the
learned cost model judged by timing, else by the autotuner) and in the plain
form (fp32, one launch per view), and the mixed batches also batched in fp32.
"""
import os

import numpy as np
import pytest

import oracle
from datagen import Agg, Column, Database, GroupBy, Pred, Query, Relation
from datagen.configs import random_covariance_workload, random_workload
from tests.helpers import compare_results

pytestmark = pytest.mark.gpu

RTOL = {"fp32": 1e-6, "bf16x6": 1e-5}


def _bench_engine(db, qs, precision, stream):
    from paper_1906_08687_amd import costmodel
    from paper_1906_08687_amd.lmfao import Engine
    eng = Engine(db, qs, precision=precision, schedule="batched")
    eng.run(stream)
    if os.path.exists(costmodel.WEIGHTS):
        eng.ctx.choose_learned_verified(costmodel.WEIGHTS, stream, 4, 3)
    else:
        eng.ctx.autotune(stream, None, 2)
    eng._bind()
    eng.run(stream)
    return eng


@pytest.mark.parametrize("j", range(150, 200))
def test_random_batch_parity(j):
    import torch
    from paper_1906_08687_amd.lmfao import Engine
    db, qs = random_workload(j, max_rows=2_000_000)
    print("case: random batch %d, relations %s, %d queries" % (j, [r.n_rows for r in db.relations], len(qs)),
          flush=True)
    ref = oracle.evaluate(db, qs)
    stream = torch.cuda.Stream()
    eng = _bench_engine(db, qs, "bf16x6", stream)
    compare_results(eng.results(), ref, qs, RTOL["bf16x6"], "random %d bf16x6 batched" % j)
    for sched in ("batched", "plain"):
        eng = Engine(db, qs, precision="fp32", schedule=sched)
        eng.run()
        compare_results(eng.results(), ref, qs, RTOL["fp32"], "random %d fp32 %s" % (j, sched))


@pytest.mark.parametrize("j", range(150, 170))
def test_random_covariance_parity(j):
    import torch
    from paper_1906_08687_amd.lmfao import Engine
    db, qs = random_covariance_workload(j, max_rows=8_000_000, min_rows=100_000)
    print("case: random covariance star %d, relations %s, %d queries" %
          (j, [r.n_rows for r in db.relations], len(qs)), flush=True)
    ref = oracle.evaluate(db, qs)
    stream = torch.cuda.Stream()
    eng = _bench_engine(db, qs, "bf16x6", stream)
    assert eng.stats()["dedicated_scan"] == 1
    compare_results(eng.results(), ref, qs, RTOL["bf16x6"], "covariance %d bf16x6" % j)
    eng = Engine(db, qs, precision="fp32", schedule="plain")
    eng.run()
    compare_results(eng.results(), ref, qs, RTOL["fp32"], "covariance %d fp32 plain" % j)


def _ties_database(n_fact=50_021):
    """Values drawn from a small set that holds every threshold and predicate
    constant exactly, on the fact and on both dimensions (one reached through
    the other: a snowflake)."""
    rng = np.random.default_rng(77)
    vals = np.array([-1.0, 0.0, 0.5, 1.0, 1.5, 2.5, 4.0], np.float32)
    F = Relation("F", [Column("k1", "key", np.sort(rng.integers(0, 300, n_fact)).astype(np.int32), 300),
                       Column("fx", "cont", rng.choice(vals, n_fact)),
                       Column("fy", "cont", rng.choice(vals, n_fact)),
                       Column("fc", "cat", rng.integers(0, 5, n_fact).astype(np.int32), 5)])
    D1 = Relation("D1", [Column("k1", "key", np.arange(300, dtype=np.int32), 300),
                         Column("k2", "key", rng.integers(0, 40, 300).astype(np.int32), 40),
                         Column("dx", "cont", rng.choice(vals, 300)),
                         Column("dc", "cat", rng.integers(0, 4, 300).astype(np.int32), 4)])
    D2 = Relation("D2", [Column("k2", "key", np.arange(40, dtype=np.int32), 40),
                         Column("sx", "cont", rng.choice(vals, 40)),
                         Column("sc", "cat", rng.integers(0, 3, 40).astype(np.int32), 3)])
    return Database([F, D1, D2], [(0, 1), (1, 2)])


def _ties_queries():
    th = np.array([0.0, 0.5, 1.5, 4.0], np.float32)      # every threshold is a value of the data
    qs = [Query()]
    for a in ("fx", "dx", "sx"):
        qs.append(Query([GroupBy(a, th)], [], [Agg.monomial("fy"), Agg.monomial(a, "fy")]))
    for op in ("le", "lt", "ge", "gt", "eq", "ne"):
        for a, v in (("fx", 0.5), ("dx", 1.0), ("sx", 2.5)):
            qs.append(Query([], [Pred(a, op, v)], [Agg.monomial("fy")]))
        qs.append(Query([GroupBy("dx", th)], [Pred("fx", op, 1.5), Pred("sx", op, 0.0)], [Agg.monomial("dx")]))
    for a, v in (("fc", 2), ("dc", 1), ("sc", 0)):
        for op in ("eq", "ne", "le", "gt"):
            qs.append(Query([GroupBy("fc")], [Pred(a, op, v)], [Agg.monomial("sx")]))
    # real constants on integer attributes: c >= 2.5 is c >= 3, c = 1.5 never holds, and
    # constants beyond the int32 range hold for every or for no row
    for a, op, v in (("fc", "ge", 2.5), ("dc", "lt", 1.5), ("sc", "eq", 0.5), ("fc", "ne", 3.25),
                     ("dc", "le", 1e12), ("sc", "gt", -1e12), ("fc", "lt", -3e9), ("k1", "gt", 149.5)):
        qs.append(Query([GroupBy("dc")], [Pred(a, op, v)], [Agg.monomial("fx")]))
    return qs


@pytest.mark.parametrize("precision,schedule", [("fp32", "batched"), ("fp32", "plain"), ("bf16x6", "batched")])
def test_values_equal_to_thresholds_and_constants(precision, schedule):
    """x = t falls in the bucket of t (x <= t_k <=> bucket <= k), and each
    comparison operator differs from its strict or non-strict twin exactly on
    such ties; categorical constants compare as integers."""
    from paper_1906_08687_amd.lmfao import Engine
    db = _ties_database()
    qs = _ties_queries()
    ref = oracle.evaluate(db, qs)
    # the data really puts rows in every bucket up to the last threshold (none lie above it)
    assert all(int(r.counts[:4].min()) > 0 and int(r.counts[4]) == 0 for r in ref[1:4])
    eng = Engine(db, qs, precision=precision, schedule=schedule)
    eng.run()
    compare_results(eng.results(), ref, qs, RTOL[precision], "ties %s %s" % (precision, schedule))
