"""Range arguments of the fixed-point spreading tile, checked on the host.

The FP32 spread forms each term q wx wy wz 2^e of a tile as an exact integer
product of two int32 factors and one rounding shift (k_spread, FIX): with
b = wmax^3 sum |q| over the tile's particles,

    e  = 58 - ilogb(b)               tile scale, 2^e b <= 2^59
    ka = 30 - ilogb(wmax^2)          A = rint(wy wz 2^ka), |A| < 2^31
    eq = 30 - ilogb(|q| wmax)        B = rint(q wx 2^eq), |B| < 2^31
    s  = eq + ka - e  (>= 1)         term = (A B + 2^(s-1)) >> s

The tests evaluate these exponents exactly as the kernel does (float32
inputs, frexp-based ilogb) on extreme charge ranges and tile sizes and check
the bounds the kernel relies on: int32 factors, a shift of at least one bit
(the rounding constant), and per-tile sums far inside the int64 range, so
that no cell can overflow whatever the order of the atomics.  They also
check that the rounded terms reproduce the float products to the expected
precision.  No GPU is involved.
"""
import math

import numpy as np
import pytest


def ilogb(x):
    """floor(log2 |x|) of a positive finite float, as ilogbf computes it."""
    m, ex = math.frexp(float(x))
    return ex - 1


def exponents(q, wmax_true):
    """e, ka and per-particle (eq, s) as the kernel derives them."""
    wmax = np.float32(1.01 * wmax_true)              # the plan's margin
    wmax3 = np.float32(1.01 * wmax_true ** 3)
    qabs = np.abs(q.astype(np.float32))
    bnd = np.float32(np.float32(qabs.sum(dtype=np.float32)) * wmax3)
    e = max(-100, min(120, 58 - ilogb(max(float(bnd), 1e-30))))
    ka = 30 - ilogb(np.float32(wmax * wmax))
    eq = np.array([30 - ilogb(np.float32(a * wmax)) if a > 0 else 0 for a in qabs])
    s = np.where(qabs > 0, np.clip(eq + ka - e, 0, 63), 0)
    return e, ka, eq, s, float(bnd)


CASES = [
    ("water", lambda rng, n: rng.choice([0.834, -0.417], size=n)),
    ("ions_unit", lambda rng, n: rng.choice([1.0, -1.0], size=n)),
    ("wide_range", lambda rng, n: rng.choice([-1, 1], size=n) * 10.0 ** rng.uniform(-6, 3, size=n)),
    ("tiny", lambda rng, n: rng.choice([-1, 1], size=n) * 1e-30 * rng.uniform(0.5, 2, size=n)),
    ("huge", lambda rng, n: rng.choice([-1, 1], size=n) * 1e30 * rng.uniform(0.5, 2, size=n)),
    ("one_big_many_small", lambda rng, n: np.concatenate([[50.0], 1e-7 * rng.standard_normal(n - 1)])),
]


@pytest.mark.parametrize("wmax_true", [0.37, 1.0, 2.9])
@pytest.mark.parametrize("n", [1, 41, 770, 20000])
@pytest.mark.parametrize("name,gen", CASES, ids=[c[0] for c in CASES])
def test_exponents_keep_every_term_in_range(name, gen, n, wmax_true):
    rng = np.random.default_rng(n)
    q = np.asarray(gen(rng, n), dtype=np.float64).astype(np.float32)
    e, ka, eq, s, bnd = exponents(q, wmax_true)
    charged = np.abs(q) > 0
    # |B| = |q| w 2^eq < 2^31 and |A| = wy wz 2^ka < 2^31 for every window value
    # up to the true maximum (the plan's wmax carries 1 % on top)
    assert np.all(np.abs(q[charged]).astype(np.float64) * wmax_true * np.exp2(eq[charged]) < 2.0 ** 31)
    assert wmax_true ** 2 * 2.0 ** ka < 2.0 ** 31
    # the shift carries a rounding bit
    assert np.all(s[charged] >= 1)
    # a tile's integer sums: sum of |terms| <= 2^e b + (one rounding unit per
    # term), far below 2^63 even if every term of every particle hit one cell
    terms_bound = 2.0 ** e * bnd + 216 * n
    assert terms_bound < 2.0 ** 60


@pytest.mark.parametrize("n", [41, 770])
def test_integer_terms_reproduce_the_float_products(n):
    """The rounded integer term, scaled back by 2^-e, agrees with the product
    q wx wy wz to about two float roundings (the factors are rounded from
    float products) plus one unit of 2^-e."""
    rng = np.random.default_rng(7)
    wmax_true = 1.0
    q = rng.choice([-1, 1], size=n) * 10.0 ** rng.uniform(-3, 1, size=n)
    q = q.astype(np.float32)
    e, ka, eq, s, bnd = exponents(q, wmax_true)
    for j in range(0, n, max(1, n // 25)):
        w = rng.uniform(0, wmax_true, size=3).astype(np.float32)
        sq = np.float32(np.ldexp(np.float64(q[j]), int(eq[j])))
        B = int(np.rint(np.float32(w[0] * sq)))
        A = int(np.rint(np.float32(w[1] * np.float32(w[2] * np.float32(2.0 ** ka)))))
        sh = int(s[j])
        term = (A * B + (1 << (sh - 1))) >> sh          # Python ints: exact, floor shift
        exact = float(q[j]) * float(w[0]) * float(w[1]) * float(w[2])
        got = term * 2.0 ** -e
        assert abs(got - exact) <= 4 * 2.0 ** -24 * abs(exact) + 2.0 ** -e
