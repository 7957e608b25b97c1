"""Error bounds of the BF16 hi+lo split arithmetic, derived and checked on
the CPU (numpy emulation of the split; no GPU, no oracle).

x = hi + lo + d with hi = bf16(x), lo = bf16(x - hi), both round to nearest
even.  bf16 keeps 8 significant bits, so |lo| <= 2^-8 |x| and
|d| <= 2^-8 |lo| <= 2^-16 |x|.  For a product x*y the three-product form
hi*hi + hi*lo + lo*hi drops lo*lo + hi*dy + dx*hi (+ smaller terms): a
relative error below 3 * 2^-16 = 4.6e-5 per product.  The four-product form
keeps lo*lo and drops the d terms: below 2 * 2^-16 = 3.1e-5.  Over many
distinct values these errors average out, except that the dropped lo*lo of
a square is never negative (a bias of a few 1e-6 for three products); a sum
dominated by one repeated value (a small dimension reached through Zipf
keys) keeps that value's error.  So a sum of n products is
within eps * sum|terms| of the exact one, eps = 3 * 2^-16 or 2 * 2^-16 plus
the fp32 accumulation, and no better in the worst case.
"""
import numpy as np


def bf16(x):
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def split(x):
    x = np.asarray(x, np.float32)
    hi = bf16(x)
    lo = bf16((x - hi).astype(np.float32))
    return hi.astype(np.float64), lo.astype(np.float64)


def products(x, y):
    hx, lx = split(x)
    hy, ly = split(y)
    exact = x.astype(np.float64) * y.astype(np.float64)
    x3 = hx * hy + hx * ly + lx * hy
    return exact, x3, x3 + lx * ly


def test_split_is_exact_to_the_stated_bits():
    rng = np.random.default_rng(0)
    x = rng.normal(0, 1, 200_000).astype(np.float32) * np.float32(10) ** rng.integers(-3, 4, 200_000).astype(np.float32)
    hi, lo = split(x)
    r = (x.astype(np.float64) - hi)
    assert np.all(np.abs(lo) <= 2.0 ** -8 * np.abs(x.astype(np.float64)) + 1e-300)
    assert np.all(np.abs(r - lo) <= 2.0 ** -16 * np.abs(x.astype(np.float64)))


def test_per_product_bounds():
    rng = np.random.default_rng(1)
    x = rng.normal(3, 1, 500_000).astype(np.float32)
    y = rng.normal(-2, 5, 500_000).astype(np.float32)
    for a, b in ((x, y), (x, x), (y, y)):
        exact, x3, x4 = products(a, b)
        rel3 = np.abs(x3 - exact) / np.abs(exact)
        rel4 = np.abs(x4 - exact) / np.abs(exact)
        assert rel3.max() <= 3 * 2.0 ** -16
        assert rel4.max() <= 2 * 2.0 ** -16
        assert rel4.mean() < rel3.mean()
        # errors of distinct values average out, except the dropped lo*lo of a square: a
        # one-signed bias of about E[lo^2] / E[x^2] (a few 1e-6) that the fourth product removes
        A = np.abs(exact).sum()
        assert abs(x3.sum() - exact.sum()) <= 5e-6 * A
        assert abs(x4.sum() - exact.sum()) <= 1e-7 * A


def test_a_repeated_value_keeps_its_error():
    """A sum of one value's squares keeps the per-product error of that
    value: above 1e-5 for the worst values of either form."""
    rng = np.random.default_rng(2)
    v = rng.uniform(1, 8, 2_000_000).astype(np.float32)
    exact, x3, x4 = products(v, v)
    for approx in (x3, x4):
        worst = v[np.argmax(np.abs(approx - exact) / exact)]
        e, a3, a4 = (np.sum(t) for t in products(np.full(1000, worst), np.full(1000, worst)))
        a = a3 if approx is x3 else a4
        assert 1e-5 < abs(a - e) / e <= 3 * 2.0 ** -16


def test_three_piece_split_keeps_every_term_to_2_to_minus_16():
    """x = hi + mid + lo + r with |r| <= 2^-24 |x|; the six products hi*hi +
    hi*mid + mid*hi + mid*mid + hi*lo + lo*hi drop only terms of order 2^-24
    (mid*lo, lo*mid, lo*lo and those of r): below 4 * 2^-24 per product, so even
    a sum of one repeated value stays far inside 1e-5."""
    from tests.helpers import bf16_split3
    rng = np.random.default_rng(3)
    x = rng.normal(3, 1, 500_000).astype(np.float32) * np.float32(10) ** rng.integers(-3, 4, 500_000).astype(np.float32)
    y = rng.normal(-2, 5, 500_000).astype(np.float32)
    hx, mx, lx = bf16_split3(x)
    assert np.all(np.abs(x.astype(np.float64) - hx - mx - lx) <= 2.0 ** -24 * np.abs(x.astype(np.float64)))
    hy, my, ly = bf16_split3(y)
    exact = x.astype(np.float64) * y.astype(np.float64)
    six = hx * hy + hx * my + mx * hy + mx * my + hx * ly + lx * hy
    assert np.max(np.abs(six - exact) / np.abs(exact)) <= 4 * 2.0 ** -24
    # the worst value of the three-product form, repeated: six products stay below 1e-6
    v = rng.uniform(1, 8, 2_000_000).astype(np.float32)
    e3 = np.abs(products(v, v)[1] - v.astype(np.float64) ** 2) / v.astype(np.float64) ** 2
    w = v[np.argmax(e3)]
    h, m, l = (float(t[0]) for t in bf16_split3(np.array([w], np.float32)))
    assert e3.max() > 1e-5
    assert abs(h * h + 2 * h * m + m * m + 2 * h * l - float(w) ** 2) / float(w) ** 2 < 1e-6
