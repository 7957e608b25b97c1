"""lmfao_bind_scratch, the binding that allocates nothing: the workspace is the
library's static per-GPU scratch array.  Its results must equal those of
lmfao_bind with a caller's workspace (the same plan and kernels): counts bit
for bit, sums within the parity tolerance (1e-5 for the bf16 split forms,
1e-6 for fp32).  Two bindings in a row, the second with a smaller input,
check that nothing from the first call leaks into the second; a binding by
another context makes the first one's executions fail with STATE until it
is bound again; a plan whose workspace exceeds the array is refused."""
import numpy as np
import pytest

import oracle
from datagen import make_batch, make_database
from tests.helpers import check_sums

pytestmark = pytest.mark.gpu


def _same(a, b, scale, rtol, what):
    """a against b: counts equal, sums under the tolerance rule with the oracle's sum |term|."""
    for i, (x, y, o) in enumerate(zip(a, b, scale)):
        assert np.array_equal(x.counts, y.counts), "%s query %d: counts differ" % (what, i)
        if x.sums.size:
            check_sums(x.sums, y.sums, o.abs_sums, rtol, "%s query %d" % (what, i))


def _pair(k, n_fact, precision, **kw):
    from paper_1906_08687_amd.lmfao import Engine
    db = make_database(k, n_fact=n_fact, **kw)
    qs = make_batch(k, db)
    orc = oracle.evaluate(db, qs)
    ref = Engine(db, qs, precision=precision, schedule="batched")
    ref.run()
    eng = Engine(db, qs, precision=precision, schedule="batched", columns=ref.cols, scratch=True)
    return ref, eng, orc


def test_scratch_binding_matches_caller_workspace_twice_second_smaller():
    import torch
    from paper_1906_08687_amd.lmfao import LmfaoError
    # first call: the covariance batch (dedicated BF16 scan), 300k fact rows
    ref1, eng1, o1 = _pair(4, 300_007, "bf16x6")
    assert eng1.ctx.workspace_size() <= 64 << 20
    eng1.run()
    _same(eng1.results(), ref1.results(), o1, 1e-5, "scratch, covariance 300k")
    # second call: a smaller input (grouped tables, filters, fp32 general scan), 60k fact rows
    ref2, eng2, o2 = _pair(2, 60_013, "fp32", dims=(1_000, 200, 5_000, 100), n_sub=20)
    assert eng2.ctx.workspace_size() < eng1.ctx.workspace_size()
    eng2.run()
    _same(eng2.results(), ref2.results(), o2, 1e-6, "scratch, snowflake 60k")
    # replayed from a captured graph on a stream: still equal
    s = torch.cuda.Stream()
    for _ in range(2):
        eng2.ctx.execute(s)
        eng2.ctx.sync()
        _same(eng2.results(), ref2.results(), o2, 1e-6, "scratch, snowflake 60k, graph")
    # the first context's descriptors were overwritten by the second binding
    with pytest.raises(LmfaoError) as e:
        eng1.ctx.execute()
    assert e.value.code == "STATE"
    eng1._bind()
    eng1.run()
    _same(eng1.results(), ref1.results(), o1, 1e-5, "scratch, covariance 300k, bound again")


def test_scratch_binding_refuses_a_workspace_above_its_size():
    from paper_1906_08687_amd.lmfao import Engine, LmfaoError
    db = make_database(4, n_fact=100_000, dims=(2_000_000, 1_000, 100, 10))
    qs = make_batch(4, db)
    with pytest.raises(LmfaoError) as e:
        Engine(db, qs, precision="bf16x6", scratch=True)
    assert e.value.code == "WORKSPACE"
