"""Test helpers shared by the oracle pins and the GPU parity tests.

``materialize`` builds the natural join of a star/snowflake database whose
non-root relations have dense unique keys 0..n-1 (every generated workload)
by plain numpy gathers: one join tuple per fact row.  It is an independent
route to the join used to pin the oracle with library routines.

``check_sums`` is the tolerance rule for floating-point aggregates: with
kappa = sum|term| / |exact|, a well-conditioned result (kappa <= 2) must meet
|got - ref| <= rtol * |ref|; otherwise the normwise bound
|got - ref| <= rtol * sum|term| applies (Higham's measure for summation).
"""
from __future__ import annotations

import numpy as np


def materialize(db):
    fact = db.relations[0]
    n = fact.n_rows
    rows = {0: np.arange(n, dtype=np.int64)}
    children = {}
    for p, c in db.edges:
        children.setdefault(p, []).append(c)
    order = [0]
    i = 0
    while i < len(order):
        p = order[i]
        for c in children.get(p, []):
            P, C = db.relations[p], db.relations[c]
            shared = [x.attr for x in C.columns if P.has(x.attr)]
            assert len(shared) == 1
            key = P.col(shared[0]).data[rows[p]].astype(np.int64)
            pk = C.col(shared[0]).data
            assert np.array_equal(pk, np.arange(C.n_rows)), "dense unique keys expected"
            rows[c] = key
            order.append(c)
        i += 1
    out = {}
    for ri, r in enumerate(db.relations):
        for col in r.columns:
            if col.attr in out:
                continue
            v = col.data[rows[ri]]
            out[col.attr] = v.astype(np.float64) if col.kind == "cont" else v.astype(np.int64)
    return out


def kappa(ref, abs_sums):
    ref = np.asarray(ref, np.float64)
    a = np.asarray(abs_sums, np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        k = np.where(ref != 0, a / np.abs(ref), np.where(a == 0, 1.0, np.inf))
    return k


def sum_errors(got, ref, abs_sums):
    """Return (strict relative error, normwise error, kappa) arrays."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    a = np.asarray(abs_sums, np.float64)
    d = np.abs(got - ref)
    with np.errstate(divide="ignore", invalid="ignore"):
        strict = np.where(ref != 0, d / np.abs(ref), np.where(d == 0, 0.0, np.inf))
        normwise = np.where(a != 0, d / a, np.where(d == 0, 0.0, np.inf))
    return strict, normwise, kappa(ref, a)


def check_sums(got, ref, abs_sums, rtol, what=""):
    strict, normwise, k = sum_errors(got, ref, abs_sums)
    ok = np.where(k <= 2.0, strict <= rtol, normwise <= rtol)
    if not np.all(ok):
        bad = np.argwhere(~ok)[:5]
        msg = ["%s: %d of %d sums outside tolerance %.1e" % (what, int((~ok).sum()), ok.size, rtol)]
        g, r, s, nw, kk = (np.asarray(got).ravel(), np.asarray(ref).ravel(), strict.ravel(),
                           normwise.ravel(), k.ravel())
        for b in np.argwhere(~ok.ravel())[:5].ravel():
            msg.append("  #%d got %r ref %r strict %.3e normwise %.3e kappa %.3g" % (b, g[b], r[b], s[b], nw[b], kk[b]))
        raise AssertionError("\n".join(msg))
    return float(np.max(strict, initial=0.0)), float(np.max(normwise, initial=0.0))


def compare_results(got, ref, queries, rtol, what):
    """Counts bit for bit, sums under check_sums; returns the worst (strict,
    normwise) error over the sums that were compared."""
    worst = (0.0, 0.0)
    for i, (g, r, q) in enumerate(zip(got, ref, queries)):
        assert g.counts.shape == r.counts.shape, (what, i)
        if not np.array_equal(g.counts, r.counts):
            bad = np.argwhere(g.counts != r.counts).ravel()[:5]
            raise AssertionError("%s query %d: counts differ at cells %s: got %s ref %s" %
                                 (what, i, bad, g.counts[bad], r.counts[bad]))
        if q.aggs:
            s, n = check_sums(g.sums, r.sums, r.abs_sums, rtol, "%s query %d" % (what, i))
            worst = (max(worst[0], s), max(worst[1], n))
    return worst


def bf16_split(x):
    """x = hi + lo + d with hi = bf16(x), lo = bf16(x - hi), both round to
    nearest even (the split of the BF16 covariance forms), as exact float64."""
    def bf16(v):
        u = np.asarray(v, np.float32).view(np.uint32).astype(np.uint64)
        return (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16).astype(np.uint32).view(np.float32)
    x = np.asarray(x, np.float32)
    hi = bf16(x)
    lo = bf16((x - hi).astype(np.float32))
    return hi.astype(np.float64), lo.astype(np.float64)


def bf16_split3(x):
    """x = hi + mid + lo (+ a remainder below 2^-24 |x|): hi = bf16(x),
    mid = bf16(x - hi), lo = bf16(x - hi - mid), round to nearest even, as exact
    float64 (the split of the BF16X6 form)."""
    x = np.asarray(x, np.float32)
    hi, mid = bf16_split(x)
    r = (x.astype(np.float64) - hi - mid).astype(np.float32)     # exact: at most 8 significant bits left
    lo, _ = bf16_split(r)
    return hi, mid, lo


def split_gram(columns, products):
    """The covariance block a BF16 split form computes, over features
    [1, columns...] of the materialised join, every product exact in float64
    (8-bit significands): products = 3 (hi*hi + hi*lo + lo*hi), 4 (+ lo*lo), or
    6 (three pieces: hi*hi + hi*mid + mid*hi + mid*mid + hi*lo + lo*hi)."""
    n = len(columns[0]) if columns else 0
    X = np.stack([np.ones(n, np.float32)] + [np.asarray(c, np.float32) for c in columns], axis=1)
    if products == 6:
        H, M, L = bf16_split3(X)
        return H.T @ H + H.T @ M + M.T @ H + M.T @ M + H.T @ L + L.T @ H
    H, L = bf16_split(X)
    G = H.T @ H + H.T @ L + L.T @ H
    if products == 4:
        G += L.T @ L
    return G
