"""The residue product of V (vmode 1), checked on the host without a GPU:

* the plan of refeig_host_crt_plan against exact integer arithmetic: odd, pairwise coprime
  moduli <= 255 whose product exceeds 4 npad 128^(ka1 + kx); digit weights congruent to the
  powers of 128 and in the symmetric INT8 range; y_q u_q-constants that invert M / m_q; M;
* the 34-bit limbs of each modulus's fraction y_q / m_q, exactly (integers from long division);
* the reconstruction that the GEMM's store (each slot mod m_q) and the V epilogue (the terms
  r_q u_q summed exactly in four 34-bit limbs, then scaled by M in double-word) perform,
  ported operation for operation (Dekker products stand in for fma, both exact), on random
  integer products P = sum_k a_k x_k of the planned size (|P| from 2^60 to the bound): the
  rebuilt value is within 2^-115 M of P (the limbs' truncation contributes at most
  2^-124.2 M, the double-word products with M the rest), far inside the 2^-108 M that the
  tightest column of the n = 8192 workload needs.
"""
import math
import random
from fractions import Fraction

import numpy as np
import pytest

from paper_2602_19090_amd import binding as rb


@pytest.mark.parametrize("npad,ka1,kx", [(8192, 15, 8), (1024, 10, 6), (256, 4, 3), (8192, 18, 9)])
def test_plan_constants_exact(npad, ka1, kx):
    p = rb.host_crt_plan(npad, ka1, kx)
    ms = p["moduli"]
    assert all(m % 2 == 1 and 3 <= m <= 255 for m in ms)
    assert all(math.gcd(a, b) == 1 for i, a in enumerate(ms) for b in ms[i + 1:])
    M = math.prod(ms)
    assert M > 4 * npad * 128 ** (ka1 + kx)
    assert math.prod(ms[:-1]) <= 4 * npad * 128 ** (ka1 + kx)     # no more moduli than needed
    for q, m in enumerate(ms):
        for t in range(ka1):
            w = int(p["wA"][q][t])
            assert -127 <= w <= 127 and (w - pow(128, ka1 - 1 - t, m)) % m == 0
        for t in range(kx):
            w = int(p["wX"][q][t])
            assert -127 <= w <= 127 and (w - pow(128, kx - 1 - t, m)) % m == 0
    assert len(p["U"]) == len(p["L"]) == len(ms)
    for q, U in enumerate(p["U"]):
        m = ms[q]
        y = pow(M // m, -1, m)
        Uq = sum(Fraction(float(v)) for v in U)
        assert abs(Uq - Fraction(y, m)) < Fraction(1, 2 ** 150)
        for k in range(4):
            want = (y * 2 ** (34 * (k + 1)) // m) % 2 ** 34
            assert float(p["L"][q][k]) == float(want)
    Mdd = Fraction(float(p["M"][0])) + Fraction(float(p["M"][1]))
    assert abs(Mdd - M) / M < Fraction(1, 2 ** 100)


def test_plan_refuses_more_than_28_moduli():
    with pytest.raises(ValueError):
        rb.host_crt_plan(8192, 30, 9)


def _split(a):
    c = 134217729.0 * a
    hi = c - (c - a)
    return hi, a - hi


def _two_prod(a, b):
    p = a * b
    ah, al = _split(a)
    bh, bl = _split(b)
    return p, ((ah * bh - p) + ah * bl + al * bh) + al * bl


def _two_sum(a, b):
    s = a + b
    z = s - a
    return s, (a - (s - z)) + (b - z)


def _f32(x):
    return float(np.float32(x))


def _rebuild(cs, ms, L, M):
    """The reconstruction for one element (scale 2^0): the GEMM stores each slot mod m_q
    (symmetric); the V epilogue sums r_q L[q][k] in four limbs (every product and sum an
    integer below 2^53, so float arithmetic is exact here as on the GPU)."""
    r = [c - m * round(c * (1.0 / m)) for c, m in zip(cs, ms)]
    assert all(abs(v) <= 127 for v in r)
    a = [0.0, 0.0, 0.0, 0.0]
    for q, lt in enumerate(L):
        rq = float(r[q])
        for k in range(4):
            prod = rq * float(lt[k])
            assert abs(prod) < 2.0 ** 53 and prod == Fraction(rq) * Fraction(float(lt[k]))
            a[k] = a[k] + prod
            assert abs(a[k]) < 2.0 ** 53
    for k in (3, 2, 1):
        cr = math.floor(a[k] * 2.0 ** -34)
        a[k] = a[k] - cr * 2.0 ** 34
        a[k - 1] = a[k - 1] + cr
    a[0] = a[0] - math.floor(a[0] * 2.0 ** -34) * 2.0 ** 34
    s0 = a[0] * 2.0 ** -34
    s1, e = _two_sum(a[1] * 2.0 ** -68, a[2] * 2.0 ** -102)
    s2 = e + a[3] * 2.0 ** -136
    if s0 + s1 >= 0.5:
        s0 -= 1.0
    M0, M1, M2 = (float(v) for v in M)
    ph, pl = _two_prod(s0, M0)
    q1, q1e = _two_prod(s0, M1)
    q2, q2e = _two_prod(s1, M0)
    L, Le = _two_sum(pl, q1)
    t, te = _two_sum(L, q2)
    L = t
    Le += te + (q1e + q2e) + (s1 * M1 + s2 * M0 + s0 * M2)
    h2, l2 = _two_sum(ph, L)
    l2 += Le
    s = h2 + l2
    return s, l2 - (s - h2)


@pytest.mark.parametrize("npad,ka1,kx", [(8192, 15, 8), (1024, 10, 6)])
def test_reconstruction_error_bound(npad, ka1, kx):
    K = 48
    p = rb.host_crt_plan(npad, ka1, kx)
    ms, L, M = p["moduli"], p["L"], p["M"]
    Mx = math.prod(ms)
    rng = random.Random(7)

    def sym(v, m):
        return ((v + (m - 1) // 2) % m) - (m - 1) // 2

    worst = Fraction(0)
    for trial in range(200):
        a = [rng.randint(-(128 ** ka1 - 1), 128 ** ka1 - 1) >> rng.choice([0, 0, 40, 80])
             for _ in range(K)]
        x = [rng.randint(-(128 ** kx - 1), 128 ** kx - 1) >> rng.choice([0, 20, 40])
             for _ in range(K)]
        P = sum(ai * xi for ai, xi in zip(a, x))
        cs = [sum(sym(ai, m) * sym(xi, m) for ai, xi in zip(a, x)) for m in ms]
        assert all(abs(c) < 2 ** 27 for c in cs)
        h, l = _rebuild(cs, ms, L, M)
        worst = max(worst, abs(Fraction(h) + Fraction(l) - P) / Mx)
    assert worst < Fraction(1, 2 ** 115), float(worst)
