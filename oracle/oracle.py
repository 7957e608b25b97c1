"""Python front end of the CPU oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module.  It marshals a ``datagen`` database and
query batch into the plain C oracle in ``oracle.c`` (the definition of the
batch, evaluated by enumerating the natural join) and returns dense results.

``brute_force`` is a second, independent statement of the same definition in
pure Python (exact rational arithmetic over the full cross product), used to
pin the C oracle on tiny inputs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from fractions import Fraction
from itertools import product
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "_oracle.so")

OP_CODES = {"le": 0, "lt": 1, "ge": 2, "gt": 3, "eq": 4, "ne": 5}
ERRORS = {-1: "invalid argument", -2: "categorical code outside its domain", -3: "out of memory"}


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Rel(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_cols", ctypes.c_int32),
                ("col_attr", ctypes.c_void_p), ("col_type", ctypes.c_void_p), ("col_data", ctypes.c_void_p)]


class _Edge(ctypes.Structure):
    _fields_ = [("parent", ctypes.c_int32), ("child", ctypes.c_int32), ("n_shared", ctypes.c_int32),
                ("parent_col", ctypes.c_void_p), ("child_col", ctypes.c_void_p)]


class _Query(ctypes.Structure):
    _fields_ = [("n_groupby", ctypes.c_int32), ("gb_attr", ctypes.c_void_p), ("gb_nthr", ctypes.c_void_p),
                ("gb_thr", ctypes.c_void_p), ("gb_dom", ctypes.c_void_p),
                ("n_preds", ctypes.c_int32), ("pred_attr", ctypes.c_void_p), ("pred_op", ctypes.c_void_p),
                ("pred_val", ctypes.c_void_p),
                ("n_aggs", ctypes.c_int32), ("agg_nterms", ctypes.c_void_p), ("term_coeff", ctypes.c_void_p),
                ("term_nfac", ctypes.c_void_p), ("fac_attr", ctypes.c_void_p),
                ("counts", ctypes.c_void_p), ("sums", ctypes.c_void_p), ("abs_sums", ctypes.c_void_p)]


@dataclass
class Result:
    """Dense result of one query: ``counts[cell]``, ``sums[cell, agg]`` and
    ``abs_sums[cell, agg]`` (the sum of |term|, the conditioning scale)."""
    counts: np.ndarray
    sums: np.ndarray
    abs_sums: np.ndarray


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        lib.oracle_evaluate.restype = ctypes.c_int
        lib.oracle_evaluate.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                        ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_int32]
        _lib = lib
    return _lib


def _arr(keep, a, dtype):
    a = np.ascontiguousarray(np.asarray(a, dtype=dtype))
    keep.append(a)
    return a.ctypes.data


def evaluate(db, queries: Sequence, n_threads: Optional[int] = None, root: int = 0,
             root_range: Optional[tuple] = None) -> List[Result]:
    """Evaluate ``queries`` over the natural join of ``db`` (see module doc)."""
    lib = _load()
    keep: list = []
    names: List[str] = []
    loc = {}
    rels = (_Rel * len(db.relations))()
    for ri, r in enumerate(db.relations):
        attrs, types, datas = [], [], []
        for ci, c in enumerate(r.columns):
            if c.attr not in loc:
                loc[c.attr] = (ri, ci)
                names.append(c.attr)
            attrs.append(names.index(c.attr))
            arr = np.ascontiguousarray(c.data)
            keep.append(arr)
            types.append(1 if arr.dtype == np.float32 else 0)
            if arr.dtype not in (np.float32, np.int32):
                raise TypeError("columns must be int32 or float32")
            datas.append(arr.ctypes.data)
        rels[ri].n_rows = r.n_rows
        rels[ri].n_cols = len(r.columns)
        rels[ri].col_attr = _arr(keep, attrs, np.int32)
        rels[ri].col_type = _arr(keep, types, np.int32)
        ptrs = (ctypes.c_void_p * max(1, len(datas)))(*datas)
        keep.append(ptrs)
        rels[ri].col_data = ctypes.cast(ptrs, ctypes.c_void_p).value
    aid = {n: i for i, n in enumerate(names)}
    edges = (_Edge * max(1, len(db.edges)))()
    for ei, (p, c) in enumerate(db.edges):
        P, C = db.relations[p], db.relations[c]
        shared = [x.attr for x in C.columns if P.has(x.attr)]
        if not shared:
            raise ValueError("join tree edge %s-%s shares no attribute" % (P.name, C.name))
        pc = [[x.attr for x in P.columns].index(a) for a in shared]
        cc = [[x.attr for x in C.columns].index(a) for a in shared]
        edges[ei].parent, edges[ei].child, edges[ei].n_shared = p, c, len(shared)
        edges[ei].parent_col = _arr(keep, pc, np.int32)
        edges[ei].child_col = _arr(keep, cc, np.int32)
    attr_rel = [loc[n][0] for n in names]
    attr_col = [loc[n][1] for n in names]
    qs = (_Query * max(1, len(queries)))()
    results = []
    for qi, q in enumerate(queries):
        Q = qs[qi]
        Q.n_groupby = len(q.groupby)
        Q.gb_attr = _arr(keep, [aid[g.attr] for g in q.groupby] or [0], np.int32)
        Q.gb_nthr = _arr(keep, [0 if g.thresholds is None else len(g.thresholds) for g in q.groupby] or [0],
                         np.int32)
        thr_ptrs = []
        for g in q.groupby:
            thr_ptrs.append(None if g.thresholds is None else _arr(keep, g.thresholds, np.float32))
        tp = (ctypes.c_void_p * max(1, len(thr_ptrs)))(*thr_ptrs)
        keep.append(tp)
        Q.gb_thr = ctypes.cast(tp, ctypes.c_void_p).value
        Q.gb_dom = _arr(keep, [g.domain(db) for g in q.groupby] or [1], np.int32)
        Q.n_preds = len(q.where)
        Q.pred_attr = _arr(keep, [aid[p.attr] for p in q.where] or [0], np.int32)
        Q.pred_op = _arr(keep, [OP_CODES[p.op] for p in q.where] or [0], np.int32)
        Q.pred_val = _arr(keep, [p.value for p in q.where] or [0.0], np.float64)
        Q.n_aggs = len(q.aggs)
        Q.agg_nterms = _arr(keep, [len(a.terms) for a in q.aggs] or [0], np.int32)
        Q.term_coeff = _arr(keep, [t[0] for a in q.aggs for t in a.terms] or [0.0], np.float64)
        Q.term_nfac = _arr(keep, [len(t[1]) for a in q.aggs for t in a.terms] or [0], np.int32)
        Q.fac_attr = _arr(keep, [aid[f] for a in q.aggs for t in a.terms for f in t[1]] or [0], np.int32)
        cells = q.n_cells(db)
        res = Result(np.zeros(cells, np.uint64), np.zeros((cells, len(q.aggs)), np.float64),
                     np.zeros((cells, len(q.aggs)), np.float64))
        Q.counts = res.counts.ctypes.data
        Q.sums = res.sums.ctypes.data
        Q.abs_sums = res.abs_sums.ctypes.data
        results.append(res)
    nt = n_threads or os.cpu_count() or 1
    b, e = root_range if root_range is not None else (0, db.relations[root].n_rows)
    rc = lib.oracle_evaluate(ctypes.addressof(rels), len(db.relations), ctypes.addressof(edges), len(db.edges),
                             root, _arr(keep, attr_rel, np.int32), _arr(keep, attr_col, np.int32), len(names),
                             ctypes.addressof(qs), len(queries), b, e, nt)
    if rc != 0:
        raise RuntimeError("oracle: " + ERRORS.get(rc, str(rc)))
    return results


# ---------------------------------------------------------------------------
# pure-Python brute force (tiny inputs only)
# ---------------------------------------------------------------------------

def _pred(x, op, t) -> bool:
    return {"le": x <= t, "lt": x < t, "ge": x >= t, "gt": x > t, "eq": x == t, "ne": x != t}[op]


def brute_force(db, queries: Sequence):
    """Exact results by the textbook definition: the natural join is the set
    of combinations of one row per relation that agree on every attribute
    name they share; aggregates are summed as exact rationals.  Returns, per
    query, (counts as a list of ints, sums as a list of lists of Fractions,
    abs_sums: the exact sum over join tuples and terms of |coeff * prod x|,
    each term taken on its own, as a list of lists of Fractions)."""
    rows = []
    for r in db.relations:
        rows.append([{c.attr: c.data[i].item() for c in r.columns} for i in range(r.n_rows)])
    kinds = {c.attr: c.kind for r in db.relations for c in r.columns}
    out = []
    joined = []
    for combo in product(*rows):
        t = {}
        ok = True
        for part in combo:
            for a, v in part.items():
                if a in t and t[a] != v:
                    ok = False
                    break
                t[a] = v
            if not ok:
                break
        if ok:
            joined.append(t)
    for q in queries:
        doms = [g.domain(db) for g in q.groupby]
        cells = int(np.prod(doms)) if doms else 1
        counts = [0] * cells
        sums = [[Fraction(0)] * len(q.aggs) for _ in range(cells)]
        abs_sums = [[Fraction(0)] * len(q.aggs) for _ in range(cells)]
        for t in joined:
            if not all(_pred(np.float32(t[p.attr]) if kinds[p.attr] == "cont" else int(t[p.attr]), p.op,
                             np.float32(p.value) if kinds[p.attr] == "cont" else float(p.value))
                       for p in q.where):
                continue
            cell = 0
            for g, d in zip(q.groupby, doms):
                if g.thresholds is None:
                    v = int(t[g.attr])
                else:
                    x = np.float32(t[g.attr])
                    v = sum(1 for th in g.thresholds if np.float32(th) < x)
                cell = cell * d + v
            counts[cell] += 1
            for ai, a in enumerate(q.aggs):
                for coeff, facs in a.terms:
                    term = Fraction(coeff)
                    for f in facs:
                        term *= Fraction(float(np.float32(t[f])))
                    sums[cell][ai] += term
                    abs_sums[cell][ai] += abs(term)
        out.append((counts, sums, abs_sums))
    return out
