"""Parity at the full workload sizes, in the launch configuration the
benchmark times (bf16x6 on MFMA where a covariance block exists, batched
schedule in a hipGraph, tiles ranked by the learned cost model with its top
four and the heuristic choice judged by timing if its weights are in the
tree, else chosen by the exhaustive autotuner), and the plain fp32 form
beside it.

The oracle evaluates a seeded sample of the batch's queries over the whole
join (every cell of each sampled query): counts bit-exact, sums under the
tolerance rule of tests/helpers.check_sums.
"""
import os

import numpy as np
import pytest

import oracle
from datagen import make_batch, make_database
from tests.helpers import check_sums

pytestmark = pytest.mark.gpu

RTOL = {"fp32": 1e-6, "bf16x6": 1e-5}
SAMPLE = 12


def _bench_engine(db, qs, cols, precision):
    """The engine as the benchmark's full form configures it."""
    import torch
    from paper_1906_08687_amd import costmodel
    from paper_1906_08687_amd.lmfao import Engine
    stream = torch.cuda.Stream()
    eng = Engine(db, qs, precision=precision, schedule="batched", columns=cols)
    eng.run(stream)
    if os.path.exists(costmodel.WEIGHTS):
        eng.ctx.choose_learned_verified(costmodel.WEIGHTS, stream, 4, 10)
    else:
        eng.ctx.autotune(stream, None, 2)
    eng._bind()
    eng.run(stream)
    return eng


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_full_size_sampled_parity(k):
    import torch
    from paper_1906_08687_amd.lmfao import Engine, upload_columns
    db = make_database(k, "full")
    qs = make_batch(k, db)
    rng = np.random.default_rng(100 + k)
    sample = sorted(set([0] + list(rng.choice(np.arange(1, len(qs)), min(SAMPLE, len(qs) - 1), replace=False))))
    print("case: workload %d full size, %d fact rows, queries %s" % (k, db.relations[0].n_rows, sample), flush=True)
    ref = oracle.evaluate(db, [qs[i] for i in sample])
    cols = upload_columns(db, torch.device("cuda", 0))
    has_gram = any(not q.groupby and not q.where and q.aggs for q in qs)
    forms = [("bf16x6" if has_gram else "fp32", None), ("fp32", "plain")]
    for precision, sched in forms:
        if sched == "plain":
            eng = Engine(db, qs, precision="fp32", schedule="plain", columns=cols)
            eng.run()
        else:
            eng = _bench_engine(db, qs, cols, precision)
        got = eng.results()
        what = "workload %d %s %s" % (k, precision, sched or "batched")
        for i, r in zip(sample, ref):
            g = got[i]
            assert np.array_equal(g.counts, r.counts), "%s query %d: counts differ" % (what, i)
            if qs[i].aggs:
                check_sums(g.sums, r.sums, r.abs_sums, RTOL[precision], "%s query %d" % (what, i))
        # a COUNT without WHERE sums to the fact size over its cells (every key resolves)
        if not qs[0].where:
            assert int(got[0].counts.sum()) == db.relations[0].n_rows
        del eng
        torch.cuda.empty_cache()
