"""Thin Python binding of ``liblmfao.so`` (ctypes): argument marshalling only.

Every step of the evaluation runs in the library's HIP kernels; PyTorch is
used to hold device memory (columns, workspace, results) and streams.  The
binding refuses to run without the compiled library: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblmfao.so")

OK = 0
ERRORS = {-1: "INVALID_ARG", -2: "NOT_ACYCLIC", -3: "UNKNOWN_ATTR", -4: "TYPE", -5: "DOMAIN", -6: "TOO_LARGE",
          -7: "WORKSPACE", -8: "STATE", -9: "HIP", -10: "UNSUPPORTED"}
I32, F32 = 0, 1
KEY, CONT, CAT, KEY_MANY = 0, 1, 2, 3
OPS = {"le": 0, "lt": 1, "ge": 2, "gt": 3, "eq": 4, "ne": 5}
PRECISION = {"fp32": 0, "bf16x3": 1, "bf16x4": 2, "bf16x6": 3}
SCHEDULE = {"plain": 0, "batched": 1}
PLANNER = {"heuristic": 0, "autotune": 1, "learned": 2}
ROOT = {"tree": 0, "find": 1}
N_FEATURES = 16


class LmfaoError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (ERRORS.get(status, str(status)), msg))
        self.status = status
        self.code = ERRORS.get(status, str(status))


class _Col(ctypes.Structure):
    _fields_ = [("attr", ctypes.c_char_p), ("dtype", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("domain", ctypes.c_int32), ("data", ctypes.c_void_p)]


class _GroupBy(ctypes.Structure):
    _fields_ = [("attr", ctypes.c_char_p), ("n_thresholds", ctypes.c_int32), ("thresholds", ctypes.c_void_p)]


class _Pred(ctypes.Structure):
    _fields_ = [("attr", ctypes.c_char_p), ("op", ctypes.c_int32), ("value", ctypes.c_double)]


class _Term(ctypes.Structure):
    _fields_ = [("coeff", ctypes.c_double), ("n_factors", ctypes.c_int32), ("factors", ctypes.c_char_p * 4)]


class _Agg(ctypes.Structure):
    _fields_ = [("n_terms", ctypes.c_int32), ("terms", ctypes.POINTER(_Term))]


class _Query(ctypes.Structure):
    _fields_ = [("n_groupby", ctypes.c_int32), ("groupby", ctypes.POINTER(_GroupBy)),
                ("n_preds", ctypes.c_int32), ("preds", ctypes.POINTER(_Pred)),
                ("n_aggs", ctypes.c_int32), ("aggs", ctypes.POINTER(_Agg))]


class _PlanOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("schedule", ctypes.c_int32), ("planner", ctypes.c_int32),
                ("block_rows", ctypes.c_int32), ("grid_blocks", ctypes.c_int32), ("gram_block", ctypes.c_int32),
                ("cost_model", ctypes.c_char_p), ("scan_every_table", ctypes.c_int32),
                ("no_row_codes", ctypes.c_int32), ("no_hist", ctypes.c_int32), ("root_policy", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("app_aggregates", ctypes.c_int32), ("inter_aggregates", ctypes.c_int32),
                ("views", ctypes.c_int32), ("groups", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("features", ctypes.c_int32), ("filters", ctypes.c_int32), ("tables", ctypes.c_int32),
                ("table_cells", ctypes.c_int64), ("launches", ctypes.c_int32), ("block_rows", ctypes.c_int32),
                ("grid_blocks", ctypes.c_int32), ("gram_block", ctypes.c_int32), ("lds_tables", ctypes.c_int32),
                ("waves", ctypes.c_int32), ("nbuf", ctypes.c_int32), ("lds_bytes", ctypes.c_int32),
                ("dedicated_scan", ctypes.c_int32), ("derived_tables", ctypes.c_int32),
                ("strided_families", ctypes.c_int32), ("code_scan", ctypes.c_int32),
                ("hist_scan", ctypes.c_int32), ("hist_parts", ctypes.c_int32), ("target_queries", ctypes.c_int32)]


# every symbol the header declares
SYMBOLS = ["lmfao_create", "lmfao_destroy", "lmfao_last_error", "lmfao_add_relation", "lmfao_set_join_tree",
           "lmfao_add_query", "lmfao_plan", "lmfao_plan_stats", "lmfao_query_root", "lmfao_choose_root", "lmfao_workspace_size", "lmfao_result_size",
           "lmfao_result_layout", "lmfao_bind", "lmfao_bind_scratch", "lmfao_execute", "lmfao_sync", "lmfao_time_root_group",
           "lmfao_candidates", "lmfao_candidate", "lmfao_candidate_features", "lmfao_select_candidate",
           "lmfao_autotune", "lmfao_choose_learned", "lmfao_choose_learned_verified", "lmfao_mlp_param_count", "lmfao_mlp_forward",
           "lmfao_mlp_scratch_floats", "lmfao_mlp_loss_grad", "lmfao_adam_step", "lmfao_mlp_train",
           "lmfao_measure_peak", "lmfao_train_workspace_size", "lmfao_train_cost_model", "lmfao_ridge_bgd", "lmfao_mutual_information", "lmfao_chow_liu", "lmfao_best_splits"]

_lib = None


def load(path: str = LIB_PATH):
    """Load the compiled engine; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("liblmfao.so is not built (run __graft_entry__.build()); "
                          "the engine has no fallback path")
    lib = ctypes.CDLL(path)
    P, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    st = ctypes.c_int32
    sig = {
        "lmfao_create": (st, [ctypes.POINTER(P), i32]),
        "lmfao_destroy": (None, [P]),
        "lmfao_last_error": (ctypes.c_char_p, [P]),
        "lmfao_add_relation": (st, [P, ctypes.c_char_p, i64, i32, P, ctypes.POINTER(i32)]),
        "lmfao_set_join_tree": (st, [P, i32, P]),
        "lmfao_add_query": (st, [P, ctypes.POINTER(_Query), ctypes.POINTER(i32)]),
        "lmfao_plan": (st, [P, ctypes.POINTER(_PlanOpts)]),
        "lmfao_plan_stats": (st, [P, ctypes.POINTER(_Stats)]),
        "lmfao_query_root": (st, [P, i32, ctypes.POINTER(i32)]),
        "lmfao_choose_root": (st, [P, P, i32, ctypes.POINTER(i32)]),
        "lmfao_workspace_size": (st, [P, ctypes.POINTER(sz)]),
        "lmfao_result_size": (st, [P, ctypes.POINTER(sz)]),
        "lmfao_result_layout": (st, [P, i32, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(sz),
                                     ctypes.POINTER(sz)]),
        "lmfao_bind": (st, [P, P, sz, P, sz]),
        "lmfao_bind_scratch": (st, [P, P, sz]),
        "lmfao_execute": (st, [P, P]),
        "lmfao_sync": (st, [P]),
        "lmfao_time_root_group": (st, [P, P, i32, i32, ctypes.POINTER(ctypes.c_double)]),
        "lmfao_candidates": (st, [P, ctypes.POINTER(i32)]),
        "lmfao_candidate": (st, [P, i32, P]),
        "lmfao_candidate_features": (st, [P, i32, P]),
        "lmfao_select_candidate": (st, [P, i32]),
        "lmfao_autotune": (st, [P, P, ctypes.c_char_p, i32, ctypes.POINTER(i32)]),
        "lmfao_choose_learned": (st, [P, ctypes.c_char_p, P, ctypes.POINTER(i32)]),
        "lmfao_choose_learned_verified": (st, [P, ctypes.c_char_p, P, i32, i32, ctypes.POINTER(i32)]),
        "lmfao_mlp_param_count": (i32, [i32]),
        "lmfao_mlp_scratch_floats": (i64, [i32, i32]),
        "lmfao_mlp_forward": (st, [i32, P, P, i32, P, P]),
        "lmfao_mlp_loss_grad": (st, [i32, P, P, P, i32, P, P, P, P]),
        "lmfao_adam_step": (st, [i32, P, P, P, P, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                 ctypes.c_float, P]),
        "lmfao_mlp_train": (st, [i32, P, P, P, P, P, i32, i32, ctypes.c_float, P, P, P, P]),
        "lmfao_measure_peak": (st, [i32, P, sz, i32, P, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]),
        "lmfao_ridge_bgd": (st, [P, i32, i32, ctypes.c_double, i32, ctypes.c_double, P, P, P]),
        "lmfao_train_workspace_size": (st, [ctypes.c_char_p, i32, ctypes.POINTER(sz)]),
        "lmfao_train_cost_model": (st, [ctypes.c_char_p, ctypes.c_char_p, P, P, sz, P, ctypes.POINTER(ctypes.c_float)]),
        "lmfao_mutual_information": (st, [P, P, i32, i32, P, P]),
        "lmfao_chow_liu": (st, [P, i32, P, P, P]),
        "lmfao_best_splits": (st, [P, i32, i32, i32, i32, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        return None
    return int(stream.cuda_stream)


def _ptr(t) -> int:
    return int(t.data_ptr())


@dataclass
class QueryResult:
    counts: np.ndarray          # uint64 [n_cells]
    sums: np.ndarray            # float64 [n_cells, n_aggs]


class Context:
    """One engine context over a database whose columns live on the device."""

    def __init__(self, device: int = 0):
        self.lib = load()
        self.ptr = ctypes.c_void_p()
        self._check(self.lib.lmfao_create(ctypes.byref(self.ptr), device))
        self.device = device
        self._keep: list = []
        self.n_queries = 0

    def close(self):
        if self.ptr:
            self.lib.lmfao_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, status: int):
        if status != OK:
            msg = self.lib.lmfao_last_error(self.ptr) if self.ptr else b""
            raise LmfaoError(status, (msg or b"").decode())

    # ---- relations, tree, queries --------------------------------------------------
    def add_relation(self, name: str, n_rows: int, cols: Sequence[tuple]) -> int:
        """cols: (attr, dtype, kind, domain, device pointer)."""
        arr = (_Col * len(cols))()
        for i, (attr, dtype, kind, domain, ptr) in enumerate(cols):
            b = attr.encode()
            self._keep.append(b)
            arr[i] = _Col(b, dtype, kind, domain, ptr)
        rid = ctypes.c_int32()
        self._check(self.lib.lmfao_add_relation(self.ptr, name.encode(), n_rows, len(cols), arr, ctypes.byref(rid)))
        return rid.value

    def set_join_tree(self, edges: Sequence[tuple]):
        flat = (ctypes.c_int32 * max(1, 2 * len(edges)))(*[v for e in edges for v in e])
        self._check(self.lib.lmfao_set_join_tree(self.ptr, len(edges), flat))

    def add_query(self, q) -> int:
        keep = self._keep
        gbs = (_GroupBy * max(1, len(q.groupby)))()
        for i, g in enumerate(q.groupby):
            b = g.attr.encode()
            keep.append(b)
            if g.thresholds is not None:
                th = np.ascontiguousarray(g.thresholds, np.float32)
                keep.append(th)
                gbs[i] = _GroupBy(b, len(th), th.ctypes.data)
            else:
                gbs[i] = _GroupBy(b, 0, None)
        preds = (_Pred * max(1, len(q.where)))()
        for i, p in enumerate(q.where):
            b = p.attr.encode()
            keep.append(b)
            preds[i] = _Pred(b, OPS[p.op], float(p.value))
        aggs = (_Agg * max(1, len(q.aggs)))()
        for i, a in enumerate(q.aggs):
            terms = (_Term * max(1, len(a.terms)))()
            for j, (coeff, facs) in enumerate(a.terms):
                names = (ctypes.c_char_p * 4)()
                for k, f in enumerate(facs[:4]):      # the library refuses more than four factors
                    b = f.encode()
                    keep.append(b)
                    names[k] = b
                terms[j] = _Term(float(coeff), len(facs), names)
            keep.append(terms)
            aggs[i] = _Agg(len(a.terms), terms)
        keep.extend([gbs, preds, aggs])
        Q = _Query(len(q.groupby), gbs, len(q.where), preds, len(q.aggs), aggs)
        qid = ctypes.c_int32()
        self._check(self.lib.lmfao_add_query(self.ptr, ctypes.byref(Q), ctypes.byref(qid)))
        self.n_queries += 1
        return qid.value

    # ---- planning --------------------------------------------------------------------
    def plan(self, precision="fp32", schedule="batched", planner="heuristic", grid_blocks=0, gram_block=0,
             rollup=True, row_codes=True, hist=True, root="tree"):
        """``root``: "tree" evaluates every query at the join tree's root, "find"
        assigns roots per query with the paper's heuristic (``root_policy``).
        ``rollup``: tables one group-by component short of another table with
        the same filter are summed from it after the scan (``scan_every_table``
        = 0); False makes the scan update every table.  ``row_codes``: filtered
        tables over several LDS partitions are updated from per-row codes when
        they qualify (``no_row_codes`` = 0).  ``hist``: unfiltered COUNT-only
        tables beyond the root scan's LDS are counted by the count-table scan
        from 16-bit component codes (``no_hist`` = 0)."""
        o = _PlanOpts(PRECISION[precision], SCHEDULE[schedule], PLANNER[planner], 0, grid_blocks, gram_block, None,
                      0 if rollup else 1, 0 if row_codes else 1, 0 if hist else 1, ROOT[root])
        self._check(self.lib.lmfao_plan(self.ptr, ctypes.byref(o)))

    def choose_root(self, stream=None, reps: int = 3) -> str:
        """Time the tree-root plan and the paper's root assignment, keep the faster ("tree" or "find")."""
        r = ctypes.c_int32()
        self._check(self.lib.lmfao_choose_root(self.ptr, _stream_handle(stream), reps, ctypes.byref(r)))
        return {v: k for k, v in ROOT.items()}[r.value]

    def query_root(self, qid: int) -> int:
        """Relation index at which query ``qid`` is evaluated."""
        r = ctypes.c_int32()
        self._check(self.lib.lmfao_query_root(self.ptr, qid, ctypes.byref(r)))
        return r.value

    def stats(self) -> dict:
        s = _Stats()
        self._check(self.lib.lmfao_plan_stats(self.ptr, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in _Stats._fields_}

    def workspace_size(self) -> int:
        v = ctypes.c_size_t()
        self._check(self.lib.lmfao_workspace_size(self.ptr, ctypes.byref(v)))
        return v.value

    def result_size(self) -> int:
        v = ctypes.c_size_t()
        self._check(self.lib.lmfao_result_size(self.ptr, ctypes.byref(v)))
        return v.value

    def result_layout(self, qid: int):
        n, a, co, so = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_size_t(), ctypes.c_size_t()
        self._check(self.lib.lmfao_result_layout(self.ptr, qid, ctypes.byref(n), ctypes.byref(a), ctypes.byref(co),
                                                 ctypes.byref(so)))
        return n.value, a.value, co.value, so.value

    def bind(self, ws_ptr: int, ws_bytes: int, res_ptr: int, res_bytes: int):
        self._check(self.lib.lmfao_bind(self.ptr, ws_ptr, ws_bytes, res_ptr, res_bytes))

    def bind_scratch(self, res_ptr: int, res_bytes: int):
        """Bind the library's static scratch array as the workspace (no allocation)."""
        self._check(self.lib.lmfao_bind_scratch(self.ptr, res_ptr, res_bytes))

    def execute(self, stream=None):
        self._check(self.lib.lmfao_execute(self.ptr, _stream_handle(stream)))

    def sync(self):
        self._check(self.lib.lmfao_sync(self.ptr))

    def time_root_group(self, stream=None, warmup=2, reps=10) -> float:
        ms = ctypes.c_double()
        self._check(self.lib.lmfao_time_root_group(self.ptr, _stream_handle(stream), warmup, reps, ctypes.byref(ms)))
        return ms.value

    def candidates(self) -> List[List[int]]:
        n = ctypes.c_int32()
        self._check(self.lib.lmfao_candidates(self.ptr, ctypes.byref(n)))
        out = []
        for i in range(n.value):
            cfg = (ctypes.c_int32 * 5)()
            self._check(self.lib.lmfao_candidate(self.ptr, i, cfg))
            out.append(list(cfg))
        return out

    def candidate_features(self, i: int) -> np.ndarray:
        f = np.zeros(N_FEATURES, np.float32)
        self._check(self.lib.lmfao_candidate_features(self.ptr, i, f.ctypes.data))
        return f

    def select_candidate(self, i: int):
        self._check(self.lib.lmfao_select_candidate(self.ptr, i))

    def autotune(self, stream=None, timing_db: Optional[str] = None, reps: int = 3) -> int:
        best = ctypes.c_int32()
        self._check(self.lib.lmfao_autotune(self.ptr, _stream_handle(stream), timing_db.encode() if timing_db else None,
                                            reps, ctypes.byref(best)))
        return best.value

    def choose_learned(self, weights: str, stream=None) -> int:
        best = ctypes.c_int32()
        self._check(self.lib.lmfao_choose_learned(self.ptr, weights.encode(), _stream_handle(stream),
                                                  ctypes.byref(best)))
        return best.value

    def choose_learned_verified(self, weights: str, stream=None, top_k: int = 3, reps: int = 3) -> int:
        best = ctypes.c_int32()
        self._check(self.lib.lmfao_choose_learned_verified(self.ptr, weights.encode(), _stream_handle(stream),
                                                           top_k, reps, ctypes.byref(best)))
        return best.value


class Engine:
    """Evaluate a query batch over a ``datagen.Database`` on one GPU.

    Columns are copied to the device once (load time is outside every
    measurement, as in the paper's protocol); the workspace and result arena
    are torch tensors bound to the context (with ``scratch``, the workspace is
    the library's static scratch array instead: lmfao_bind_scratch).
    ``rollup`` and ``row_codes`` are the plan options of ``Context.plan``
    (derived tables; tables replayed from per-row codes), both on by default.
    """

    def __init__(self, db, queries, precision="fp32", schedule="batched", planner="heuristic", device=0,
                 grid_blocks=0, gram_block=0, columns=None, rollup=True, row_codes=True, scratch=False, hist=True,
                 root="tree"):
        import torch
        self.torch = torch
        self.db = db
        self.queries = list(queries)
        self.dev = torch.device("cuda", device)
        self.ctx = Context(device)
        self.cols = columns if columns is not None else upload_columns(db, self.dev)
        for r in db.relations:
            spec = []
            for c in r.columns:
                t = self.cols[(r.name, c.attr)]
                dtype = F32 if c.kind == "cont" else I32
                kind = {"key": KEY, "cont": CONT, "cat": CAT, "key_many": KEY_MANY}[c.kind]
                spec.append((c.attr, dtype, kind, int(c.domain), _ptr(t)))
            self.ctx.add_relation(r.name, r.n_rows, spec)
        self.ctx.set_join_tree(db.edges)
        for q in self.queries:
            self.ctx.add_query(q)
        self.precision, self.schedule, self.rollup, self.row_codes = precision, schedule, rollup, row_codes
        self.scratch, self.hist, self.root = scratch, hist, root
        self.ctx.plan(precision, schedule, planner, grid_blocks, gram_block, rollup, row_codes, hist, root)
        self._bind()

    def _bind(self):
        torch = self.torch
        self.ws_bytes = self.ctx.workspace_size()
        self.res_bytes = self.ctx.result_size()
        if self.scratch:
            # the library's static scratch array is the workspace; only the results are ours
            if not hasattr(self, "res") or self.res.numel() < self.res_bytes:
                self.res = torch.empty(self.res_bytes, dtype=torch.uint8, device=self.dev)
            self.ctx.bind_scratch(_ptr(self.res), self.res.numel())
            return
        if not hasattr(self, "ws") or self.ws.numel() < self.ws_bytes + 256:
            # slack so that other tile candidates (autotuner, cost model) bind in place
            self.ws = torch.empty(self.ws_bytes + (4 << 20), dtype=torch.uint8, device=self.dev)
        if not hasattr(self, "res") or self.res.numel() < self.res_bytes:
            self.res = torch.empty(self.res_bytes, dtype=torch.uint8, device=self.dev)
        base = _ptr(self.ws)
        self.ws_base = (base + 255) // 256 * 256
        self.ctx.bind(self.ws_base, self.ws.numel() - (self.ws_base - base), _ptr(self.res), self.res.numel())

    def choose_root(self, stream=None, reps: int = 3) -> str:
        """Keep the faster of the tree-root plan and the paper's root assignment (timed whole);
        returns "tree" or "find"."""
        self.root = self.ctx.choose_root(stream, reps)
        self._bind()
        self.run(stream)
        return self.root

    def replan(self, precision=None, schedule=None, planner="heuristic", grid_blocks=0, gram_block=0):
        self.precision = precision or self.precision
        self.schedule = schedule or self.schedule
        self.ctx.plan(self.precision, self.schedule, planner, grid_blocks, gram_block, self.rollup, self.row_codes,
                      self.hist, self.root)
        self._bind()

    def run(self, stream=None):
        self.ctx.execute(stream)
        self.ctx.sync()

    def results(self) -> List[QueryResult]:
        host = self.res.cpu().numpy()
        out = []
        for qid in range(len(self.queries)):
            n, a, co, so = self.ctx.result_layout(qid)
            counts = host[co:co + 8 * n].view(np.uint64).copy()
            sums = host[so:so + 8 * n * a].view(np.float64).reshape(n, a).copy()
            out.append(QueryResult(counts, sums))
        return out

    def stats(self) -> dict:
        return self.ctx.stats()


def upload_columns(db, dev):
    import torch
    out = {}
    for r in db.relations:
        for c in r.columns:
            out[(r.name, c.attr)] = torch.from_numpy(np.ascontiguousarray(c.data)).to(dev)
    return out


# ---------------------------------------------------------------------------
# cost-model network kernels (device tensors in, device tensors out)
# ---------------------------------------------------------------------------

def _check(status: int, what: str):
    if status != OK:
        raise LmfaoError(status, what)


def mlp_param_count(hidden: int) -> int:
    return int(load().lmfao_mlp_param_count(hidden))


def mlp_forward(hidden: int, params, x, stream=None):
    """y[n] = network(x[n][16]) for fp32 device tensors."""
    import torch
    y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
    _check(load().lmfao_mlp_forward(hidden, _ptr(params), _ptr(x), x.shape[0], _ptr(y), _stream_handle(stream)),
           "mlp_forward")
    return y


def mlp_loss_grad(hidden: int, params, x, target, stream=None):
    import torch
    lib = load()
    n = x.shape[0]
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    grad = torch.empty_like(params)
    scratch = torch.empty(int(lib.lmfao_mlp_scratch_floats(hidden, n)), dtype=torch.float32, device=x.device)
    _check(lib.lmfao_mlp_loss_grad(hidden, _ptr(params), _ptr(x), _ptr(target), n, _ptr(loss), _ptr(grad),
                                   _ptr(scratch), _stream_handle(stream)), "mlp_loss_grad")
    return loss, grad


def adam_step(params, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(load().lmfao_adam_step(params.numel(), _ptr(params), _ptr(grad), _ptr(m), _ptr(v), step, lr, beta1, beta2,
                                  eps, _stream_handle(stream)), "adam_step")


def mlp_train(hidden: int, params, x, target, epochs: int, lr: float, stream=None):
    """Full-batch Adam training on the device; returns the per-step losses."""
    import torch
    lib = load()
    n = x.shape[0]
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    grad = torch.empty_like(params)
    scratch = torch.empty(int(lib.lmfao_mlp_scratch_floats(hidden, n)), dtype=torch.float32, device=x.device)
    losses = torch.empty(epochs, dtype=torch.float32, device=x.device)
    _check(lib.lmfao_mlp_train(hidden, _ptr(params), _ptr(m), _ptr(v), _ptr(x), _ptr(target), n, epochs, lr,
                               _ptr(grad), _ptr(scratch), _ptr(losses), _stream_handle(stream)), "mlp_train")
    return losses


PEAKS = {"read": 0, "lds_u32": 1, "lds_u32_spread": 2, "lds_f64": 3, "global_u64": 4}


def measure_peak(kind: str, buf, iters: int, stream=None):
    """Time one throughput probe (lmfao_measure_peak) on a device tensor ``buf``;
    returns (milliseconds, bytes read or atomics issued)."""
    load()
    ms, units = ctypes.c_double(), ctypes.c_double()
    _check(_lib.lmfao_measure_peak(PEAKS[kind], _ptr(buf), buf.numel() * buf.element_size(), iters,
                                   _stream_handle(stream), ctypes.byref(ms), ctypes.byref(units)), "measure_peak")
    return ms.value, units.value


# ---------------------------------------------------------------------------
# application loops (Section 2): argument marshalling around lmfao_ridge_bgd,
# lmfao_mutual_information, lmfao_chow_liu and lmfao_best_splits
# ---------------------------------------------------------------------------

class _SplitInput(ctypes.Structure):
    _fields_ = [("counts", ctypes.c_void_p), ("sums", ctypes.c_void_p), ("sum_stride", ctypes.c_int32),
                ("n_cells", ctypes.c_int32), ("categorical", ctypes.c_int32), ("node", ctypes.c_int32)]


class _SplitResult(ctypes.Structure):
    _fields_ = [("cost", ctypes.c_double), ("input", ctypes.c_int32), ("cell", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("pad2", ctypes.c_int32)]


SPLIT = {"variance": 0, "gini": 1}


def _sync():
    import torch
    torch.cuda.synchronize()


def _to_device_bytes(obj_bytes: bytes, dev):
    import torch
    return torch.frombuffer(bytearray(obj_bytes), dtype=torch.uint8).to(dev)


def ridge_bgd(cov, label: int, lam: float, max_iters: int = 1000, tol: float = 1e-10, stream=None):
    """Ridge regression by gradient descent on the device over the covariance matrix `cov`
    (an n x n float64 device tensor over [1, X...]); returns (theta tensor, [J, steps, |grad|])."""
    import torch
    load()
    cov = cov.contiguous()
    n = cov.shape[0]
    theta = torch.empty(n, dtype=torch.float64, device=cov.device)
    info = torch.empty(3, dtype=torch.float64, device=cov.device)
    _check(_lib.lmfao_ridge_bgd(_ptr(cov), n, label, lam, max_iters, tol, _ptr(theta), _ptr(info),
                                _stream_handle(stream)), "ridge_bgd")
    _sync()
    return theta, info.cpu().numpy()


def covariance_matrix(eng, attrs):
    """The engine's covariance block over [1, attrs...] as an n x n float64 device tensor,
    gathered from the result arena (queries of datagen.configs.covariance_queries)."""
    import torch
    feats = [None] + list(attrs)
    n = len(feats)
    res64 = eng.res.view(torch.float64)
    C = torch.zeros((n, n), dtype=torch.float64, device=eng.res.device)
    for qid, q in enumerate(eng.queries):
        if q.groupby or q.where:
            continue
        _, a, co, so = eng.ctx.result_layout(qid)
        if not q.aggs:
            C[0, 0] = eng.res[co:co + 8].view(torch.int64)[0].to(torch.float64)
            continue
        fs = q.aggs[0].terms[0][1]
        i = feats.index(fs[0])
        j = feats.index(fs[1]) if len(fs) > 1 else 0
        C[i, j] = res64[so // 8]
        C[j, i] = res64[so // 8]
    return C


def mutual_information(eng, pair_qids, stream=None):
    """Mutual information of each pairwise COUNT GROUP BY query of `eng` (device tensor)."""
    import torch
    load()
    base = _ptr(eng.res)
    ptrs, doms = [], []
    for qid in pair_qids:
        q = eng.queries[qid]
        _, _, co, _ = eng.ctx.result_layout(qid)
        ptrs.append(base + co)
        doms += [q.groupby[0].domain(eng.db), q.groupby[1].domain(eng.db)]
    dev = eng.res.device
    pt = torch.tensor(ptrs, dtype=torch.int64, device=dev)
    dt = torch.tensor(doms, dtype=torch.int32, device=dev)
    mi = torch.empty(len(ptrs), dtype=torch.float64, device=dev)
    _check(_lib.lmfao_mutual_information(_ptr(pt), _ptr(dt), len(ptrs), max(doms) if doms else 1, _ptr(mi),
                                         _stream_handle(stream)), "mutual_information")
    _sync()
    return mi


def chow_liu(mi, stream=None):
    """Chow-Liu tree of an n x n float64 device tensor of mutual informations:
    (edges as a list of (i, j) in the order taken, their total)."""
    import torch
    load()
    mi = mi.contiguous()
    n = mi.shape[0]
    edges = torch.empty(2 * (n - 1), dtype=torch.int32, device=mi.device)
    total = torch.empty(1, dtype=torch.float64, device=mi.device)
    _check(_lib.lmfao_chow_liu(_ptr(mi), n, _ptr(edges), _ptr(total), _stream_handle(stream)), "chow_liu")
    _sync()
    e = edges.cpu().numpy().reshape(-1, 2)
    return [(int(a), int(b)) for a, b in e if a >= 0], float(total.item())


def _run_splits(structs, n_nodes, criterion, n_labels, dev, stream=None):
    import torch
    load()
    arr = (_SplitInput * max(1, len(structs)))(*structs)
    din = _to_device_bytes(bytes(arr), dev)
    out = torch.empty(n_nodes * ctypes.sizeof(_SplitResult), dtype=torch.uint8, device=dev)
    _check(_lib.lmfao_best_splits(_ptr(din), len(structs), n_nodes, SPLIT[criterion], n_labels, _ptr(out),
                                  _stream_handle(stream)), "best_splits")
    _sync()
    host = (_SplitResult * n_nodes).from_buffer_copy(out.cpu().numpy().tobytes())
    return [(r.cost, r.input, r.cell) for r in host]


def best_splits(eng, qids, nodes, criterion="variance", n_labels=0, stream=None):
    """Best split per node from the engine's histograms: query qids[k] belongs to node nodes[k];
    VARIANCE queries group by the split attribute and sum y and y^2; GINI queries group by
    (label, split attribute).  Returns (cost, input k, cell) per node."""
    base = _ptr(eng.res)
    structs = []
    for qid, node in zip(qids, nodes):
        q = eng.queries[qid]
        n_cells, a, co, so = eng.ctx.result_layout(qid)
        g = q.groupby[-1]
        cells = g.domain(eng.db)
        structs.append(_SplitInput(base + co, base + so if criterion == "variance" else None, a, cells,
                                   1 if g.thresholds is None else 0, node))
    return _run_splits(structs, max(nodes) + 1 if nodes else 0, criterion, n_labels, eng.res.device, stream)


def best_splits_from_arrays(inputs, n_nodes, criterion="variance", n_labels=0, stream=None):
    """Best split per node from host histograms (dicts: node, categorical, counts, sums),
    uploaded to the device first."""
    import torch
    dev = torch.device("cuda", 0)
    keep, structs = [], []
    for I in inputs:
        c = torch.from_numpy(np.ascontiguousarray(I["counts"], dtype=np.uint64).view(np.int64)).to(dev)
        keep.append(c)
        sp, stride = None, 0
        if criterion == "variance":
            sm = np.ascontiguousarray(I["sums"], dtype=np.float64)
            st = torch.from_numpy(sm).to(dev)
            keep.append(st)
            sp, stride = _ptr(st), sm.shape[1]
        n_cells = (c.numel() if criterion == "variance" else c.numel() // n_labels)
        structs.append(_SplitInput(_ptr(c), sp, stride, n_cells, int(I["categorical"]), int(I["node"])))
    out = _run_splits(structs, n_nodes, criterion, n_labels, dev, stream)
    del keep
    return out


class _TrainOpts(ctypes.Structure):
    _fields_ = [("hidden", ctypes.c_int32), ("epochs", ctypes.c_int32), ("lr", ctypes.c_float),
                ("pad", ctypes.c_int32), ("seed", ctypes.c_uint64)]


def train_cost_model(timing_db: str, weights_out: str, hidden: int = 32, epochs: int = 4000, lr: float = 3e-3,
                     seed: int = 1, device: int = 0, stream=None) -> float:
    """lmfao_train_cost_model in a torch-allocated workspace; returns the final loss."""
    import torch
    load()
    need = ctypes.c_size_t()
    _check(_lib.lmfao_train_workspace_size(timing_db.encode(), hidden, ctypes.byref(need)), "train_workspace_size")
    ws = torch.empty(need.value + 256, dtype=torch.uint8, device=torch.device("cuda", device))
    base = (_ptr(ws) + 255) // 256 * 256
    loss = ctypes.c_float()
    o = _TrainOpts(hidden, epochs, lr, 0, seed)
    _check(_lib.lmfao_train_cost_model(timing_db.encode(), weights_out.encode(), ctypes.byref(o), base,
                                       need.value + 256 - (base - _ptr(ws)), _stream_handle(stream),
                                       ctypes.byref(loss)), "train_cost_model")
    return float(loss.value)
