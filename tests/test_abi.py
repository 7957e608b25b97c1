"""The C ABI without a GPU: every declared symbol is exported, planning is
host-only and deterministic, and every documented error path returns its
status code.  Column pointers here are placeholders: planning never reads
device memory, and binding without a device is refused."""
import ctypes
import os
import re

import pytest

from paper_1906_08687_amd import lmfao

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lmfao.h")
FAKE = 0x100000          # a placeholder device address, never dereferenced on the host


def _lib():
    if not os.path.exists(lmfao.LIB_PATH):
        pytest.skip("liblmfao.so not built")
    return lmfao.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lmfao_\w+)\s*\(", text)))


def test_header_declares_exactly_the_binding_symbols():
    assert declared_functions() == sorted(lmfao.SYMBOLS)


def test_library_exports_every_declared_symbol():
    lib = _lib()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_library_loads_only_from_the_tree_and_fails_loudly_when_missing(tmp_path):
    with pytest.raises(ImportError):
        saved = lmfao._lib
        lmfao._lib = None
        try:
            lmfao.load(str(tmp_path / "missing.so"))
        finally:
            lmfao._lib = saved


# --------------------------------------------------------------------------
# a small star schema built from placeholder pointers
# --------------------------------------------------------------------------

def star(ctx, fact_rows=1000):
    """F(k1, k2, f0, f1, fc) with D1(k1, a0, a1, ac) and D2(k2, b0)."""
    ctx.add_relation("F", fact_rows, [("k1", lmfao.I32, lmfao.KEY, 50, FAKE), ("k2", lmfao.I32, lmfao.KEY, 20, FAKE),
                                      ("f0", lmfao.F32, lmfao.CONT, 0, FAKE), ("f1", lmfao.F32, lmfao.CONT, 0, FAKE),
                                      ("fc", lmfao.I32, lmfao.CAT, 7, FAKE)])
    ctx.add_relation("D1", 50, [("k1", lmfao.I32, lmfao.KEY, 50, FAKE), ("a0", lmfao.F32, lmfao.CONT, 0, FAKE),
                                ("a1", lmfao.F32, lmfao.CONT, 0, FAKE), ("ac", lmfao.I32, lmfao.CAT, 5, FAKE)])
    ctx.add_relation("D2", 20, [("k2", lmfao.I32, lmfao.KEY, 20, FAKE), ("b0", lmfao.F32, lmfao.CONT, 0, FAKE)])
    ctx.set_join_tree([(0, 1), (0, 2)])


def covariance(attrs):
    from datagen.configs import covariance_queries
    return covariance_queries(attrs)


def new_ctx():
    _lib()
    return lmfao.Context(0)


def test_plan_is_host_only_and_reports_the_batch():
    from datagen.schema import Agg, GroupBy, Pred, Query
    ctx = new_ctx()
    star(ctx)
    feats = ["f0", "f1", "a0", "a1", "b0"]
    qs = covariance(feats)
    qs += [Query(groupby=[GroupBy("ac")], aggs=[Agg.monomial("f0")]),
           Query(groupby=[GroupBy("fc"), GroupBy("ac")]),
           Query(groupby=[GroupBy("b0", [-1.0, 0.0, 1.0])], aggs=[Agg.monomial("a1")]),
           Query(where=[Pred("a0", "le", 0.5)], aggs=[Agg.monomial("f1")])]
    for q in qs:
        ctx.add_query(q)
    n = len(feats)
    for prec in ("fp32", "bf16x3", "bf16x4"):
        for sched in ("plain", "batched"):
            ctx.plan(prec, sched)
            s = ctx.stats()
            assert s["app_aggregates"] == sum(1 + len(q.aggs) for q in qs)      # one COUNT per query
            assert s["features"] == n + 1                  # the constant 1 plus the attributes
            # two child views, the covariance output, one output view per grouped table
            assert s["tables"] == 4 and s["table_cells"] == 5 + 7 * 5 + 4 + 1
            assert s["views"] == 2 + 1 + s["tables"] and s["filters"] == 1
            assert s["groups"] == 3 and s["levels"] == 2
            assert ctx.workspace_size() > 0 and ctx.result_size() > 0
            if sched == "batched":
                assert s["launches"] >= 1
    # dense output cells: the product of the group-by domains
    expect = [1] * len(covariance(feats)) + [5, 7 * 5, 4, 1]
    for qid, cells in enumerate(expect):
        nc, na, co, so = ctx.result_layout(qid)
        assert nc == cells, qid
        assert co % 8 == 0 and so % 8 == 0
    # the planner is deterministic
    a = (ctx.workspace_size(), ctx.result_size(), ctx.stats())
    ctx.plan("fp32", "plain")
    ctx.plan("bf16x4", "batched")
    assert (ctx.workspace_size(), ctx.result_size(), ctx.stats()) == a


def test_rounds_feature_counts_workgroup_rounds_and_leaves_the_plan():
    """Feature 2 plans each candidate on the side: on the dedicated covariance scan of five
    features (one 16-slot tile, 12 resident waves per CU, little LDS) a launch of g
    workgroups of w waves takes g w / (12 n_cu) rounds; the context's own plan is unchanged."""
    ctx = new_ctx()
    star(ctx, fact_rows=50_000_000)
    for q in covariance(["f0", "f1", "a0", "b0"]):
        ctx.add_query(q)
    ctx.plan("bf16x3", "batched")
    before = ctx.stats()
    assert before["dedicated_scan"] == 1
    cands = ctx.candidates()
    n_cu = cands[0][2] // 4                           # first candidate: 1 wave per workgroup, 4 per CU
    assert cands[0][:2] == [1, 1] and n_cu > 0
    feats = [ctx.candidate_features(i) for i in range(len(cands))]
    assert ctx.stats() == before
    for i, (waves, nbuf, grid, gb, policy) in enumerate(cands):
        ctx.select_candidate(i)
        launched = ctx.stats()["grid_blocks"]         # the grid as launched (whole tiles per workgroup)
        assert launched <= grid
        assert abs(feats[i][2] - launched * waves / (12 * n_cu)) < 1e-5


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_tile_candidates_are_distinct_and_featurised(precision):
    ctx = new_ctx()
    star(ctx, fact_rows=50_000_000)                  # large enough that no candidate grid is clamped
    for q in covariance(["f0", "f1", "a0", "b0"]):
        ctx.add_query(q)
    ctx.plan(precision, "batched")
    cands = ctx.candidates()
    assert len(cands) >= 4
    assert len({tuple(c) for c in cands}) == len(cands)
    for i, c in enumerate(cands):
        waves, nbuf, grid, gb, policy = c
        assert waves in (1, 2, 4) and nbuf in (1, 2) and grid > 0
        f = ctx.candidate_features(i)
        assert f.shape == (16,) and all(map(lambda v: v == v, f))
        assert f[14] == waves and f[15] == nbuf
        ctx.select_candidate(i)
        s = ctx.stats()
        assert (s["waves"], s["nbuf"]) == (waves, nbuf)
        # rows per workgroup: whole 64-row wave tiles; the grid covers the fact exactly
        rows, br, gx = 50_000_000, s["block_rows"], s["grid_blocks"]
        assert br % (64 * waves) == 0 and gx <= grid
        assert (gx - 1) * br < rows <= gx * br
        if precision == "fp32":
            assert s["gram_block"] == gb
        else:
            assert gb == 0 and s["gram_block"] == 16         # 5 features padded to one 16-wide MFMA tile


def test_bind_and_execute_need_a_device_and_a_plan():
    import torch
    if torch.cuda.is_available():
        pytest.skip("host-only error paths")
    ctx = new_ctx()
    star(ctx)
    with pytest.raises(lmfao.LmfaoError) as e:
        ctx.plan()
    assert e.value.code == "STATE"                   # no queries yet
    ctx.add_query(covariance(["f0"])[0])
    with pytest.raises(lmfao.LmfaoError) as e:
        ctx.bind(FAKE, 1 << 20, FAKE, 1 << 20)
    assert e.value.code == "STATE"                   # not planned
    ctx.plan()
    with pytest.raises(lmfao.LmfaoError) as e:
        ctx.bind(FAKE, 1 << 30, FAKE, 1 << 30)
    assert e.value.code == "HIP"                     # no device
    for call in (lambda: ctx.execute(None), lambda: ctx.sync(), lambda: ctx.time_root_group(None, 1, 1),
                 lambda: ctx.autotune(None, None, 1), lambda: ctx.choose_learned("w.bin", None),
                 lambda: ctx.choose_learned_verified("w.bin", None, 3, 1), lambda: ctx.choose_root(None, 1)):
        with pytest.raises(lmfao.LmfaoError) as e:
            call()
        assert e.value.code == "STATE"
    for k, reps in ((0, 1), (3, 0)):
        expect("INVALID_ARG", lambda: ctx.choose_learned_verified("w.bin", None, k, reps))
    expect("INVALID_ARG", lambda: ctx.choose_root(None, 0))


# --------------------------------------------------------------------------
# documented error statuses
# --------------------------------------------------------------------------

def expect(code, fn):
    with pytest.raises(lmfao.LmfaoError) as e:
        fn()
    assert e.value.code == code, str(e.value)
    assert str(e.value).split(": ", 1)[1]            # a message accompanies every error


def test_relation_errors():
    ctx = new_ctx()
    expect("TYPE", lambda: ctx.add_relation("A", 10, [("x", lmfao.I32, lmfao.CONT, 0, FAKE)]))
    expect("TYPE", lambda: ctx.add_relation("A", 10, [("k", lmfao.F32, lmfao.KEY, 10, FAKE)]))
    expect("INVALID_ARG", lambda: ctx.add_relation("A", 10, [("c", lmfao.I32, lmfao.CAT, 0, FAKE)]))
    expect("INVALID_ARG", lambda: ctx.add_relation("A", 10, [("x", lmfao.F32, lmfao.CONT, 0, 0)]))
    expect("INVALID_ARG", lambda: ctx.add_relation("A", 10, [("x", lmfao.F32, lmfao.CONT, 0, FAKE),
                                                             ("x", lmfao.F32, lmfao.CONT, 0, FAKE)]))
    expect("TOO_LARGE", lambda: ctx.add_relation("A", (1 << 40) + 1, [("x", lmfao.F32, lmfao.CONT, 0, FAKE)]))
    ctx.add_relation("A", 10, [("x", lmfao.F32, lmfao.CONT, 0, FAKE)])
    expect("INVALID_ARG", lambda: ctx.add_relation("A", 10, [("y", lmfao.F32, lmfao.CONT, 0, FAKE)]))
    # an empty relation needs no data pointer
    ctx.add_relation("E", 0, [("z", lmfao.F32, lmfao.CONT, 0, 0)])


def three(ctx, shared=("k1", "k2"), d2_extra=None):
    ctx.add_relation("F", 100, [("k1", lmfao.I32, lmfao.KEY, 10, FAKE), ("k2", lmfao.I32, lmfao.KEY, 10, FAKE),
                                ("x", lmfao.F32, lmfao.CONT, 0, FAKE)])
    ctx.add_relation("D1", 10, [(shared[0], lmfao.I32, lmfao.KEY, 10, FAKE), ("y", lmfao.F32, lmfao.CONT, 0, FAKE)])
    cols = [(shared[1], lmfao.I32, lmfao.KEY, 10, FAKE), ("z", lmfao.F32, lmfao.CONT, 0, FAKE)]
    if d2_extra:
        cols.append(d2_extra)
    ctx.add_relation("D2", 10, cols)


@pytest.mark.parametrize("edges,code", [
    ([(0, 1)], "NOT_ACYCLIC"),                       # m-1 edges needed
    ([(0, 1), (0, 2), (1, 2)], "NOT_ACYCLIC"),
    ([(0, 1), (2, 1)], "NOT_ACYCLIC"),               # D1 with two parents
    ([(1, 2), (2, 1)], "NOT_ACYCLIC"),               # a cycle, F unconnected
    ([(0, 1), (0, 7)], "INVALID_ARG"),
])
def test_join_tree_shape_errors(edges, code):
    ctx = new_ctx()
    three(ctx)
    expect(code, lambda: ctx.set_join_tree(edges))


def test_join_tree_attribute_errors():
    ctx = new_ctx()                                  # F-D1 share no attribute
    three(ctx, shared=("k9", "k2"))
    expect("UNSUPPORTED", lambda: ctx.set_join_tree([(0, 1), (0, 2)]))
    ctx = new_ctx()                                  # join attribute continuous in the child
    ctx.add_relation("F", 100, [("k1", lmfao.I32, lmfao.KEY, 10, FAKE), ("x", lmfao.F32, lmfao.CONT, 0, FAKE)])
    ctx.add_relation("D1", 10, [("k1", lmfao.F32, lmfao.CONT, 0, FAKE)])
    expect("TYPE", lambda: ctx.set_join_tree([(0, 1)]))
    ctx = new_ctx()                                  # y held by D1 and D2 only: running intersection fails
    three(ctx, d2_extra=("y", lmfao.F32, lmfao.CONT, 0, FAKE))
    expect("NOT_ACYCLIC", lambda: ctx.set_join_tree([(0, 1), (0, 2)]))


def test_state_errors():
    from datagen.schema import Agg, Query
    ctx = new_ctx()
    expect("STATE", lambda: ctx.set_join_tree([]))   # no relations
    three(ctx)
    expect("STATE", lambda: ctx.add_query(Query(aggs=[Agg.monomial("x")])))
    ctx.set_join_tree([(0, 1), (0, 2)])
    expect("STATE", lambda: ctx.set_join_tree([(0, 1), (0, 2)]))
    expect("STATE", lambda: ctx.add_relation("G", 1, [("w", lmfao.F32, lmfao.CONT, 0, FAKE)]))


def test_query_errors():
    from datagen.schema import Agg, GroupBy, Pred, Query
    ctx = new_ctx()
    three(ctx)
    ctx.set_join_tree([(0, 1), (0, 2)])
    expect("UNKNOWN_ATTR", lambda: ctx.add_query(Query(aggs=[Agg.monomial("nope")])))
    expect("UNKNOWN_ATTR", lambda: ctx.add_query(Query(groupby=[GroupBy("nope")])))
    expect("UNKNOWN_ATTR", lambda: ctx.add_query(Query(where=[Pred("nope", "le", 0.0)])))
    expect("TYPE", lambda: ctx.add_query(Query(groupby=[GroupBy("y")])))                  # continuous, no thresholds
    expect("TYPE", lambda: ctx.add_query(Query(aggs=[Agg.monomial("k1")])))               # key as a factor
    expect("INVALID_ARG", lambda: ctx.add_query(Query(groupby=[GroupBy("y", [1.0, 0.0])])))
    expect("INVALID_ARG", lambda: ctx.add_query(Query(groupby=[GroupBy("y", [1.0, 1.0])])))
    # a term names at most four factors: n_factors = 5 is refused before the array is read
    names = (ctypes.c_char_p * 4)(b"x", b"y", b"x", b"y")
    term = (lmfao._Term * 1)(lmfao._Term(1.0, 5, names))
    agg = (lmfao._Agg * 1)(lmfao._Agg(1, term))
    q = lmfao._Query(0, None, 0, None, 1, agg)
    qid = ctypes.c_int32()
    assert ctx.lib.lmfao_add_query(ctx.ptr, ctypes.byref(q), ctypes.byref(qid)) == -6
    ctx.add_query(Query(aggs=[Agg.monomial("x", "z")]))
    ctx.plan()


def test_marginal_derivation_is_planned_per_filter_and_chained():
    """A grouped table one component short of a same-filter table that already
    carries its sums is summed from it after the scan: one pass per derived key
    length, each adding a launch.  Tables under another filter, or whose sums
    the finer table lacks, are not derived."""
    from datagen.schema import Agg, GroupBy, Pred, Query
    ctx = new_ctx()
    star(ctx)
    filt = [Pred("a0", "le", 0.5)]
    ctx.add_query(Query(groupby=[GroupBy("fc"), GroupBy("ac")], aggs=[Agg.monomial("f0")]))
    ctx.add_query(Query(groupby=[GroupBy("ac")], aggs=[Agg.monomial("f0")]))          # from (fc, ac)
    ctx.add_query(Query(groupby=[GroupBy("fc")], where=filt, aggs=[Agg.monomial("a1")]))  # no filtered source
    ctx.add_query(Query(where=filt, aggs=[Agg.monomial("a1")]))                        # from the filtered (fc)
    ctx.add_query(Query(groupby=[GroupBy("b0", [-1.0, 0.0, 1.0]), GroupBy("fc"), GroupBy("ac")],
                        aggs=[Agg.monomial("f0")]))
    ctx.add_query(Query(groupby=[GroupBy("fc")], aggs=[Agg.monomial("f1")]))          # (fc, ac) lacks SUM(f1)
    ctx.plan("fp32", "batched", rollup=False)
    off = ctx.stats()
    ctx.plan("fp32", "batched")
    on = ctx.stats()
    assert off["derived_tables"] == 0 and off["tables"] == on["tables"] == 6
    # (fc, ac) comes from the 3-component table, (ac) from (fc, ac), the filtered sum from the
    # filtered (fc): three passes (key lengths 2, 1, 0)
    assert on["derived_tables"] == 3
    assert on["launches"] == off["launches"] + 3
    ctx.plan("fp32", "plain")
    plain = ctx.stats()
    ctx.plan("fp32", "plain", rollup=False)
    assert plain["launches"] == ctx.stats()["launches"]       # three fewer table scans, three passes


def test_plan_option_errors():
    ctx = new_ctx()
    star(ctx)
    ctx.add_query(covariance(["f0"])[1])
    o = lmfao._PlanOpts(0, 1, 0, 0, 0, 0, None, 0, 0, 0)
    for field, bad in (("precision", 4), ("precision", -1), ("schedule", 2), ("planner", 9), ("block_rows", 128),
                       ("grid_blocks", -1), ("gram_block", 5), ("scan_every_table", 2), ("no_row_codes", -1),
                       ("no_hist", 2)):
        x = lmfao._PlanOpts.from_buffer_copy(o)
        setattr(x, field, bad)
        assert ctx.lib.lmfao_plan(ctx.ptr, ctypes.byref(x)) == -1, field
    assert ctx.lib.lmfao_plan(ctx.ptr, ctypes.byref(o)) == 0


def test_plan_size_limits():
    from datagen.schema import Agg, Query
    ctx = new_ctx()
    ctx.add_relation("F", (1 << 30) + 1, [("x", lmfao.F32, lmfao.CONT, 0, FAKE)])
    ctx.set_join_tree([])
    ctx.add_query(Query(aggs=[Agg.monomial("x")]))
    expect("TOO_LARGE", lambda: ctx.plan())


def test_mlp_parameter_count_matches_reference():
    from oracle import mlp as ref
    _lib()
    for h in (1, 8, 32, 64):
        assert lmfao.mlp_param_count(h) == ref.param_count(h)


def _plan_db(db, qs, **kw):
    ctx = new_ctx()
    for r in db.relations:
        spec = []
        for c in r.columns:
            dtype = lmfao.F32 if c.kind == "cont" else lmfao.I32
            kind = {"key": lmfao.KEY, "cont": lmfao.CONT, "cat": lmfao.CAT, "key_many": lmfao.KEY_MANY}[c.kind]
            spec.append((c.attr, dtype, kind, int(c.domain), FAKE))
        ctx.add_relation(r.name, r.n_rows, spec)
    ctx.set_join_tree(db.edges)
    for q in qs:
        ctx.add_query(q)
    ctx.plan(kw.pop("precision", "fp32"), kw.pop("schedule", "batched"), **kw)
    return ctx


def test_row_codes_are_planned_for_partitioned_filtered_tables():
    """Filtered tables over several LDS partitions (a tree level's per-node
    histograms) are replayed from per-row codes: the plan adds the code scan's
    launch and a workspace region of 4 bytes per code column and row (mask,
    one cell per key, one value per summed feature).  Unfiltered tables, the
    plain schedule and no_row_codes keep the root scan's own updates."""
    from datagen import make_batch, make_database
    db = make_database(3)
    qs = make_batch(3, db)                     # COUNT, SUM(y), SUM(y^2) per node x attribute x bucket
    on = _plan_db(db, qs)
    off = _plan_db(db, qs, row_codes=False)
    s_on, s_off = on.stats(), off.stats()
    assert s_on["code_scan"] == 1 and s_off["code_scan"] == 0
    assert s_on["strided_families"] >= 1 and s_off["strided_families"] >= 1
    assert s_on["launches"] == s_off["launches"] + 1
    n_rows = db.relations[0].n_rows
    n_keys = len(qs) // 32                     # one key per attribute, shared by the 32 nodes
    cols = 1 + n_keys + 1                      # mask, cells, y
    assert on.workspace_size() - off.workspace_size() >= cols * ((n_rows + 63) // 64 * 64) * 4
    assert _plan_db(db, qs, schedule="plain").stats()["code_scan"] == 0
    db5 = make_database(5)
    assert _plan_db(db5, make_batch(5, db5)).stats()["code_scan"] == 0   # unfiltered pair counts


def test_count_tables_are_planned_beyond_the_root_scans_lds():
    """Unfiltered COUNT-only tables that the root scan cannot hold in one LDS
    partition (the 105 pair counts of the mutual-information batch) move to
    the count-table scan: one more launch, 2 bytes of workspace per component
    code and row, tables cut into LDS slices packed into partitions.  Small
    pair tables that fit the root scan's LDS (workload 1's single grouped
    table), the plain schedule and no_hist keep the root scan's updates."""
    from datagen import make_batch, make_database
    db5 = make_database(5)
    qs5 = make_batch(5, db5)
    on, off = _plan_db(db5, qs5), _plan_db(db5, qs5, hist=False)
    s_on, s_off = on.stats(), off.stats()
    assert s_on["hist_scan"] == 1 and s_off["hist_scan"] == 0 and s_off["hist_parts"] == 0
    assert s_on["launches"] == s_off["launches"] + 1
    # every pair table's cells are in some partition: at least cells / LDS-words partitions
    pair_cells = sum(q.n_cells(db5) for q in qs5 if len(q.groupby) == 2)
    assert s_on["hist_parts"] >= pair_cells // (160 * 1024 // 4)
    n_rows = db5.relations[0].n_rows
    assert on.workspace_size() - off.workspace_size() >= 15 * ((n_rows + 63) // 64 * 64) * 2
    assert _plan_db(db5, qs5, schedule="plain").stats()["hist_scan"] == 0
    db1 = make_database(1)
    assert _plan_db(db1, make_batch(1, db1)).stats()["hist_scan"] == 0


def test_scratch_binding_needs_a_plan_and_a_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("host-only error paths")
    ctx = new_ctx()
    star(ctx)
    ctx.add_query(covariance(["f0"])[0])
    expect("STATE", lambda: ctx.bind_scratch(FAKE, 1 << 20))
    ctx.plan()
    expect("HIP", lambda: ctx.bind_scratch(FAKE, 1 << 20))


def test_application_loop_argument_errors():
    """Argument checks of the application loops return before any launch."""
    lib = _lib()
    F = ctypes.c_void_p(FAKE)
    assert lib.lmfao_ridge_bgd(F, 65, 1, 0.1, 10, 1e-9, F, F, None) == -1        # more than 64 features
    assert lib.lmfao_ridge_bgd(F, 8, 0, 0.1, 10, 1e-9, F, F, None) == -1         # label 0 is the constant
    assert lib.lmfao_ridge_bgd(F, 8, 3, -1.0, 10, 1e-9, F, F, None) == -1        # negative lambda
    assert lib.lmfao_mutual_information(F, F, 3, 4096, F, None) == -6            # domain above 2048
    assert lib.lmfao_mutual_information(None, F, 3, 10, F, None) == -1
    assert lib.lmfao_chow_liu(F, 65, F, F, None) == -6
    assert lib.lmfao_chow_liu(F, 1, F, F, None) == -1
    assert lib.lmfao_best_splits(F, 4, 2, 7, 0, F, None) == -1                   # unknown criterion
    assert lib.lmfao_best_splits(F, 4, 2, 1, 0, F, None) == -1                   # Gini needs labels
    assert lib.lmfao_best_splits(F, 4, 2, 1, 17, F, None) == -6                  # at most 16 labels


def test_training_reads_the_timing_file_and_checks_its_arguments(tmp_path):
    """lmfao_train_workspace_size parses the autotuner's timing file (16 features, 5
    configuration values, milliseconds per line); malformed files and options are refused
    before anything touches a device."""
    from paper_1906_08687_amd import costmodel
    lib = _lib()
    path = os.path.join(os.path.dirname(costmodel.WEIGHTS), "timings.csv")
    n = ctypes.c_size_t()
    assert lib.lmfao_train_workspace_size(path.encode(), 32, ctypes.byref(n)) == 0
    rows = sum(1 for l in open(path) if l.strip())
    assert n.value >= rows * (16 + 1) * 4
    bad = tmp_path / "bad.csv"
    bad.write_text("1,2,3\n")
    assert lib.lmfao_train_workspace_size(str(bad).encode(), 32, ctypes.byref(n)) == -1
    neg = tmp_path / "neg.csv"
    neg.write_text(",".join(["1"] * 21 + ["-2.0"]) + "\n")
    assert lib.lmfao_train_workspace_size(str(neg).encode(), 32, ctypes.byref(n)) == -1
    assert lib.lmfao_train_workspace_size(b"/nonexistent/timings.csv", 32, ctypes.byref(n)) == -1
    o = lmfao._TrainOpts(32, 0, 1e-3, 0, 1)                       # zero epochs
    assert lib.lmfao_train_cost_model(path.encode(), str(tmp_path / "w.bin").encode(), ctypes.byref(o),
                                      ctypes.c_void_p(FAKE), 1 << 30, None, None) == -1


def test_polynomial_moments_are_planned_with_derived_products():
    """Degree-2 polynomial regression (Section 2): the covariance over [1, x, x_i x_j]
    holds every moment of degree <= 4; the plan stages each attribute and each product of
    two attributes once (1 + n + n(n+1)/2 features) and runs the general root scan."""
    from datagen import make_database
    from datagen.configs import cont_attrs, polynomial_queries
    db = make_database(1, n_fact=1000)
    attrs = cont_attrs(db)[:6]
    qs = polynomial_queries(attrs)
    c = 1 + 6 + 21
    assert len(qs) == c * (c + 1) // 2
    st = _plan_db(db, qs).stats()
    assert st["features"] == c and st["dedicated_scan"] == 0
    # nine attributes: 1 + 9 + 45 = 55 staged values, within the 64 of the covariance block
    assert _plan_db(db, polynomial_queries(cont_attrs(db)[:9])).stats()["features"] == 1 + 9 + 45


def test_many_to_many_children_plan_as_count_weighted_views():
    """A child whose join key repeats (KEY_MANY) is planned as a
    count-weighted view: FP32 covariance, grouped sums keyed by other
    relations and sums of its attributes plan at the tree root.  A query that
    groups by, filters on or (grouped) multiplies attributes of the child is
    evaluated at the child (its root, Section 3.3); one that does so for two
    such children, and a BF16 covariance block with one, are UNSUPPORTED."""
    import numpy as np
    from datagen.configs import cont_attrs, covariance_queries, many_to_many_batch, many_to_many_database
    from datagen.schema import Agg, GroupBy, Pred, Query
    db = many_to_many_database(n_fact=2000, n_users=50, n_business=40)
    qs = many_to_many_batch(db)
    ctx = _plan_db(db, qs)
    assert ctx.stats()["target_queries"] == 0
    assert all(ctx.query_root(i) == 0 for i in range(len(qs)))
    for prec in ("bf16x3", "bf16x6"):
        with pytest.raises(lmfao.LmfaoError) as e:
            _plan_db(db, qs, precision=prec)
        assert e.value.code == "UNSUPPORTED"
    # tables only: any precision (tables are summed in fp64)
    _plan_db(db, qs[len(covariance_queries(cont_attrs(db))):], precision="bf16x6")
    cat, att = db.index("Category"), db.index("Attribute")
    local = [(Query(groupby=[GroupBy("cw", np.array([0.0, 1.0], np.float32))]), cat),
             (Query(where=[Pred("aw", "gt", 0.0)], aggs=[Agg.monomial("stars")]), att),
             (Query(groupby=[GroupBy("bcat")], aggs=[Agg.monomial("cw", "cv")]), cat),
             (Query(aggs=[Agg.monomial("cw", "cv", "stars")]), cat)]
    ctx = _plan_db(db, [q for q, _ in local] + [Query(aggs=[Agg.monomial("cw", "cv")])])
    assert [ctx.query_root(i) for i in range(len(local))] == [r for _, r in local]
    assert ctx.query_root(len(local)) == 0          # ungrouped pair product: the covariance block
    assert ctx.stats()["target_queries"] == len(local)
    with pytest.raises(lmfao.LmfaoError) as e:
        _plan_db(db, [Query(groupby=[GroupBy("cw", np.array([0.0], np.float32))], where=[Pred("aw", "gt", 0.0)])])
    assert e.value.code == "UNSUPPORTED"


def test_find_roots_assigns_grouped_queries_to_their_relations():
    """The paper's root assignment (Section 3.3) on workload 2's snowflake:
    the covariance block stays at the fact; a relation's weight is the sum
    over grouped queries of the fraction of their group-by attributes it
    holds; relations become roots in decreasing weight (ties to the larger),
    each for the unassigned queries grouping by one of its attributes; S,
    below D3, passes its queries to D3.  Under the tree policy every query
    stays at the fact."""
    from datagen import make_batch, make_database
    db = make_database(2)
    qs = make_batch(2, db)
    tree = _plan_db(db, qs)
    assert tree.stats()["target_queries"] == 0
    ctx = _plan_db(db, qs, root="find")
    idx = {r.name: i for i, r in enumerate(db.relations)}
    owner = {c.attr: r.name for r in db.relations for c in r.columns if c.kind == "cat"}
    roots = [ctx.query_root(i) for i in range(len(qs))]
    # expected, from the definition: weights over grouped queries
    W = {r.name: 0.0 for r in db.relations}
    for q in qs:
        if not q.groupby and not q.where:
            continue
        for g in q.groupby:
            W[owner[g.attr]] += 1.0 / len(q.groupby)
    order = sorted(W, key=lambda n: (-W[n], -db.rel(n).n_rows))
    parent = {c: p for p, c in db.edges}
    top = lambda n: n if parent.get(idx[n]) in (None, 0) else db.relations[parent[idx[n]]].name
    for q, r in zip(qs, roots):
        if not q.groupby and not q.where:
            assert r == idx["F"]
            continue
        first = next(n for n in order if W[n] > 0 and any(owner[g.attr] == n for g in q.groupby))
        assert r == idx[top(first)], (q, r, first)
    assert ctx.stats()["target_queries"] == sum(1 for r in roots if r != idx["F"]) > 0


def test_root_assignment_falls_back_and_forced_views_are_bounded():
    """A query the paper's root assignment sends to a dimension stays at the tree root when
    its view towards that dimension would exceed 2^24 cells (the dimension's key domain times
    the query's other group-by cells); a query forced to a many-to-many child by such a view
    is TOO_LARGE instead."""
    from datagen.schema import GroupBy, Query
    big = 1 << 23
    ctx = new_ctx()
    ctx.add_relation("F", 1 << 20, [("k", lmfao.I32, lmfao.KEY, big, FAKE), ("fc", lmfao.I32, lmfao.CAT, 4, FAKE)])
    ctx.add_relation("D", big, [("k", lmfao.I32, lmfao.KEY, big, FAKE), ("dc", lmfao.I32, lmfao.CAT, 9, FAKE)])
    ctx.set_join_tree([(0, 1)])
    qs = [Query(groupby=[GroupBy("dc")]), Query(groupby=[GroupBy("dc")]),
          Query(groupby=[GroupBy("dc"), GroupBy("fc")])]
    for q in qs:
        ctx.add_query(q)
    ctx.plan("fp32", "batched", root="find")
    # D carries the larger weight (2.5 against 0.5): the two dc queries go there (views of 2^23
    # cells); the (dc, fc) query's view would be 2^25 cells, so it stays at F
    assert [ctx.query_root(i) for i in range(3)] == [1, 1, 0]
    assert ctx.stats()["target_queries"] == 2
    ctx.plan("fp32", "batched", root="tree")
    assert [ctx.query_root(i) for i in range(3)] == [0, 0, 0]
    expect("INVALID_ARG", lambda: ctx.query_root(3))

    ctx = new_ctx()
    ctx.add_relation("F", 1 << 20, [("k", lmfao.I32, lmfao.KEY, big, FAKE), ("fc", lmfao.I32, lmfao.CAT, 4, FAKE)])
    ctx.add_relation("C", 1 << 24, [("k", lmfao.I32, lmfao.KEY_MANY, big, FAKE), ("cc", lmfao.I32, lmfao.CAT, 3, FAKE)])
    ctx.set_join_tree([(0, 1)])
    ctx.add_query(Query(groupby=[GroupBy("cc")]))
    ctx.plan("fp32", "batched")
    assert ctx.query_root(0) == 1
    ctx.add_query(Query(groupby=[GroupBy("cc"), GroupBy("fc")]))
    expect("TOO_LARGE", lambda: ctx.plan("fp32", "batched"))
