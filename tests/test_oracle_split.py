"""Pins for the oracle's splitting, exact slice products and parameter rule.

* 7-bit digit planes: exact reconstruction (rational arithmetic), digit range,
  the truncation bound, the exponent definition and edge cases.
* int64 slice products against Python integer dot products (brute force).
* The Ozaki identity (Sec. 2.3): with enough planes the slice products
  reproduce A X exactly.
* The FP64 splitting of eq. (a)/(x): exact reconstruction, the remainder bound
  of eq. (minamihata) and exactness of slice products when alpha + beta >=
  -log2 u + log2 n.
* beta of Sec. 4.1 on hand-derived cases, and the truncation bound it implies.
"""
import json
import os
from fractions import Fraction as F

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _mat(seed, m, n, spread=20):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((m, n)) * 2.0 ** rng.integers(-spread, spread, (m, n))
    return np.asfortranarray(M)


def _edge_matrix():
    M = np.zeros((7, 6))
    M[:, 0] = [1.0, -1.0, 0.5, 2.0 ** -30, 0.0, -0.0, 0.75]                # power-of-two max
    M[:, 1] = 0.0                                                          # zero column
    M[:, 2] = [5e-324, -1e-310, 0.0, 2.0 ** -1020, 1.0, 0.0, 0.0]           # subnormals
    M[:, 3] = [np.nextafter(1.0, 0.0), -np.nextafter(1.0, 0.0), 1e-16, 0.0, 0.1, 0.2, 0.3]
    M[:, 4] = [3.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0]
    M[:, 5] = [-2.0 ** 40, 2.0 ** 39 + 1.0, 7.0, -7.0, 1.0, 0.0, 2.0 ** -13]
    return np.asfortranarray(M)


def _check_split(M, k, by_rows, ex, pl, tr):
    m, nc = M.shape
    for v in range(m if by_rows else nc):
        line = M[v, :] if by_rows else M[:, v]
        mx = np.max(np.abs(line))
        e = int(ex[v])
        if mx == 0:
            assert e == 0
        else:
            assert F(2) ** (e - 1) <= F(mx) < F(2) ** e       # e = floor(log2 max) + 1
        for t in range(len(line)):
            i, j = (v, t) if by_rows else (t, v)
            digits = [int(pl[r][i, j]) if by_rows else int(pl[r][j, i]) for r in range(k)]
            assert all(-127 <= d <= 127 for d in digits)
            a = F(M[i, j])
            assert all(d == 0 or (d > 0) == (a > 0) for d in digits)   # sign-magnitude
            val = sum(F(d) * F(2) ** (e - 7 * (r + 1)) for r, d in enumerate(digits))
            assert F(tr[i, j]) == val                                  # value of the planes
            assert abs(a - val) < F(2) ** (e - 7 * k)                  # truncation bound
            assert abs(val) <= abs(a)                                  # truncation toward 0


@pytest.mark.parametrize("by_rows", [False, True])
@pytest.mark.parametrize("k", [1, 3, 8])
def test_split_random(by_rows, k):
    M = _mat(11 + k, 9, 13)
    ex, pl, tr = oracle.split_s7(M, k, by_rows=by_rows)
    _check_split(M, k, by_rows, ex, pl, tr)
    if k == 8:   # 56 bits cover every bit of a double within 2^4 of 2^e (ulp >= 2^(e-56))
        big = np.abs(M) >= 2.0 ** (ex[:, None] - 4 if by_rows else ex[None, :] - 4)
        assert np.array_equal(tr[big], M[big])


@pytest.mark.parametrize("by_rows", [False, True])
def test_split_edges(by_rows):
    M = _edge_matrix()
    for k in (1, 2, 9):
        ex, pl, tr = oracle.split_s7(M, k, by_rows=by_rows)
        _check_split(M, k, by_rows, ex, pl, tr)


def test_split_range_error():
    """Scale exponents outside [-900, 900] are rejected (the scaled products would leave the
    normal FP64 range)."""
    M = np.asfortranarray(np.array([[1e-300, 1.0], [2e-300, 0.5]]))
    with pytest.raises(RuntimeError):
        oracle.split_s7(M, 2)


def test_split_enough_planes_is_exact():
    """Entries in [2^(e-1), 2^e) have ulp 2^(e-53) >= 2^(e-56), the grid of 8 planes,
    so 8 planes reproduce them exactly."""
    rng = np.random.default_rng(3)
    M = np.asfortranarray(rng.uniform(0.5, 1.0, (40, 5)) * rng.choice([-1, 1], (40, 5)))
    ex, pl, tr = oracle.split_s7(M, 8)
    assert np.array_equal(tr, M)


def test_slice_products_brute_force():
    rng = np.random.default_rng(4)
    m, n, K = 9, 7, 301
    Ap = rng.integers(-127, 128, (m, K)).astype(np.int8)
    Bp = rng.integers(-127, 128, (n, K)).astype(np.int8)
    C = oracle.slice_gemm_i64(Ap, Bp)
    for i in range(m):
        for j in range(n):
            assert int(C[i, j]) == sum(int(Ap[i, p]) * int(Bp[j, p]) for p in range(K))
    Ap[:] = -127; Bp[:] = -127
    C = oracle.slice_gemm_i64(Ap, Bp)
    assert np.all(C == 127 * 127 * K)


def test_ozaki_identity_exact():
    """With planes that cover every bit, sum_{r,s} 2^(e_i+e_j-7(r+s)) A^(r) X^(s) = A X exactly."""
    n = 6
    rng = np.random.default_rng(5)
    A = np.asfortranarray(rng.uniform(0.5, 1.0, (n, n)) * rng.choice([-1, 1], (n, n)))
    A = np.asfortranarray((A + A.T) / 2)
    X = np.asfortranarray(rng.uniform(0.5, 1.0, (n, n)) * rng.choice([-1, 1], (n, n)))
    k = 9
    ea, pa, ta = oracle.split_s7(A, k, by_rows=True)
    ex, px, tx = oracle.split_s7(X, k, by_rows=False)
    assert np.array_equal(ta, A) and np.array_equal(tx, X)
    acc = [[F(0)] * n for _ in range(n)]
    for r in range(k):
        for s in range(k):
            C = oracle.slice_gemm_i64(pa[r], px[s])
            for i in range(n):
                for j in range(n):
                    acc[i][j] += F(int(C[i, j])) * F(2) ** (int(ea[i]) + int(ex[j]) - 7 * (r + s + 2))
    for i in range(n):
        for j in range(n):
            assert acc[i][j] == sum(F(A[i, p]) * F(X[p, j]) for p in range(n))


# ------------------------------------------------------------------ FP64 sigma split
def _ufp(x):
    return 0.0 if x == 0 else 2.0 ** np.floor(np.log2(abs(x)))


@pytest.mark.parametrize("alpha", [10, 20, 30])
def test_sigma_split_reconstruction_and_bound(alpha):
    M = _mat(21, 8, 10, spread=6)
    slices, rem = oracle.sigma_split(M, alpha, 3, by_rows=True)
    for i in range(8):
        for j in range(10):
            assert sum(F(s[i, j]) for s in slices) + F(rem[i, j]) == F(M[i, j])
    # eq. (minamihata): |remainder after slice r| <= u * ufp(sigma^(r))
    rem_r = np.array(M)
    for s in slices:
        v = np.max(np.abs(rem_r), axis=1)
        sigma = np.array([0.75 * 2.0 ** (np.ceil(np.log2(x)) + alpha) if x > 0 else 0.0 for x in v])
        rem_r = rem_r - s
        for i in range(8):
            assert np.all(np.abs(rem_r[i]) <= 2.0 ** -53 * _ufp(sigma[i]))


def test_sigma_split_products_exact():
    """alpha + beta >= -log2 u + log2 n  =>  fl(A^(r) X^(s)) = A^(r) X^(s)."""
    n = 16
    A = _mat(31, n, n, spread=3)
    X = _mat(32, n, n, spread=3)
    alpha = beta = 29   # 58 >= 53 + 4
    As, _ = oracle.sigma_split(A, alpha, 2, by_rows=True)
    Xs, _ = oracle.sigma_split(X, beta, 2, by_rows=False)
    for Ar in As:
        for Xs_ in Xs:
            P = Ar @ Xs_
            for i in range(0, n, 5):
                for j in range(0, n, 3):
                    assert F(P[i, j]) == sum(F(Ar[i, p]) * F(Xs_[p, j]) for p in range(n))


# ------------------------------------------------------------------ beta rule
def test_beta_golden_cases():
    with open(os.path.join(GOLDEN, "beta_cases.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        n = c["n"]
        X = np.asfortranarray(np.array(c["X"], dtype=np.float64).reshape(n, n, order="F"))
        got = oracle.beta_rule(np.array(c["lam"]), X, c["delta"])
        assert got["status"] == 0
        assert got["beta"] == c["beta"], c["why"]
        assert got["kx"] == c["kx"], c["why"]


def test_beta_is_floor_of_log2():
    """2^beta <= (1/(0.75u)) sqrt(n delta g / (L S)) < 2^(beta+1), checked in rationals
    against the FP64-evaluated argument on random inputs."""
    rng = np.random.default_rng(9)
    for _ in range(50):
        n = int(rng.integers(3, 30))
        lam = np.sort(rng.uniform(-1, 1, n)) * 10.0 ** rng.integers(-6, 2)
        X = np.asfortranarray(rng.standard_normal((n, n)) * 10.0 ** rng.integers(-3, 1))
        delta = 10.0 ** rng.uniform(-15, -5)
        g = oracle.beta_rule(lam, X, delta)
        q = ((n * delta) * g["gap"]) / (g["lmax"] * g["S"])
        t = np.sqrt(q) / (0.75 * 2.0 ** -53)
        assert F(2) ** g["beta"] <= F(t) < F(2) ** (g["beta"] + 1)


def test_truncation_meets_paper_bound():
    """X^(1) from kx planes satisfies |x_ij - x1_ij| <= u * ufp(tau_j) = 2^(c_j + beta - 54),
    the bound eq. (minamihata) gives for the paper's rounding split (Sec. 3.3)."""
    import workloads
    p = workloads.make_problem(2, 128, x0="eigh")
    for delta in (1e-8, 1e-11, 1e-14):
        st = oracle.method_step(p.A, p.X0, p.D0, delta)
        for j in range(p.n):
            w = np.max(np.abs(p.X0[:, j]))
            c = int(np.ceil(np.log2(w)))
            assert np.max(np.abs(p.X0[:, j] - st.X1[:, j])) <= 2.0 ** (c + st.beta - 54)
