"""Pins for the oracle's double-double primitives against exact rational arithmetic.

TwoSum (Sec. 2.2): x = fl(a + b) and y with x + y = a + b exactly.
TwoProd: p = fl(a b) and e with p + e = a b exactly.
Double-double add / mul / div / sqrt: relative error a small multiple of u^2.
"""
from fractions import Fraction as F
from decimal import Decimal, getcontext

import numpy as np
import pytest

import oracle

U2 = F(1, 2 ** 104)

CASES = [
    (1.0, 1e-20), (1e16, 1.0), (1.0, -1.0 + 2 ** -52), (3.0, 4.0), (-0.0, 0.0), (0.0, -0.0),
    (2.0 ** 1000, 2.0 ** 940), (1.5, 2.0 ** -60), (-7.25, 7.25), (np.pi, np.e), (1e-300, 1e-310),
]


def _rand_pairs(seed, k):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(k) * 2.0 ** rng.integers(-40, 40, k)
    b = rng.standard_normal(k) * 2.0 ** rng.integers(-40, 40, k)
    return list(zip(a.tolist(), b.tolist()))


@pytest.mark.parametrize("a,b", CASES + _rand_pairs(1, 200))
def test_two_sum_exact(a, b):
    s, e = oracle.two_sum(a, b)
    assert s == a + b                      # x = fl(a + b)
    assert F(s) + F(e) == F(a) + F(b)      # x + y = a + b exactly


@pytest.mark.parametrize("a,b", [c for c in CASES if c[0] == 0 or c[1] == 0 or 1e-250 < abs(c[0] * c[1]) < 1e300]
                         + _rand_pairs(2, 200))
def test_two_prod_exact(a, b):
    p, e = oracle.two_prod(a, b)
    assert p == a * b
    assert F(p) + F(e) == F(a) * F(b)


def _dd(x):
    """A random double-double near x."""
    h = float(x)
    return h, h * 2.0 ** -60 * 0.37


@pytest.mark.parametrize("seed", range(40))
def test_dd_arith_error(seed):
    rng = np.random.default_rng(100 + seed)
    a = (float(rng.standard_normal()), 0.0)
    a = (a[0], a[0] * 2.0 ** -55 * float(rng.uniform(-1, 1)))
    b = (float(rng.standard_normal()) * 2.0 ** int(rng.integers(-20, 20)), 0.0)
    b = (b[0], b[0] * 2.0 ** -55 * float(rng.uniform(-1, 1)))
    Fa, Fb = F(a[0]) + F(a[1]), F(b[0]) + F(b[1])
    for op, exact in (("add", Fa + Fb), ("mul", Fa * Fb), ("div", Fa / Fb)):
        h, l = oracle.dd_op(op, a, b)
        got = F(h) + F(l)
        assert abs(got - exact) <= 16 * U2 * (abs(Fa) + abs(Fb) if op == "add" else abs(exact)), op
        assert abs(l) <= abs(h) * 2.0 ** -52  # normalised
    # sqrt through Decimal at 60 digits
    getcontext().prec = 60
    x = (abs(a[0]), abs(a[1]) if a[0] > 0 else -abs(a[1]))
    h, l = oracle.dd_op("sqrt", x)
    ref = (Decimal(x[0]) + Decimal(x[1])).sqrt()
    assert abs(Decimal(h) + Decimal(l) - ref) <= Decimal(2.0 ** -100) * ref


def test_dd_gemm_vs_fractions():
    """op(A) B in double-double against the exact rational product."""
    rng = np.random.default_rng(7)
    n = 6
    A = np.asfortranarray(rng.standard_normal((n, n)) * 2.0 ** rng.integers(-10, 10, (n, n)))
    Bh = np.asfortranarray(rng.standard_normal((n, n)))
    Bl = np.asfortranarray(Bh * 2.0 ** -54 * rng.uniform(-1, 1, (n, n)))
    for trans in (False, True):
        Ch, Cl = oracle.dd_gemm(A, Bh, None, Bl, transA=trans)
        opA = A.T if trans else A
        for i in range(n):
            for j in range(n):
                ex = sum(F(opA[i, p]) * (F(Bh[p, j]) + F(Bl[p, j])) for p in range(n))
                mag = sum(abs(F(opA[i, p]) * F(Bh[p, j])) for p in range(n))
                assert abs(F(Ch[i, j]) + F(Cl[i, j]) - ex) <= 8 * n * U2 * mag


def test_dd_gemm_catches_transpose():
    """A non-symmetric product distinguishes A B from A^T B."""
    rng = np.random.default_rng(8)
    A = np.asfortranarray(rng.standard_normal((5, 5)))
    B = np.asfortranarray(rng.standard_normal((5, 5)))
    C1, _ = oracle.dd_gemm(A, B)
    C2, _ = oracle.dd_gemm(A, B, transA=True)
    np.testing.assert_allclose(C1, A @ B, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(C2, A.T @ B, rtol=1e-13, atol=1e-13)
