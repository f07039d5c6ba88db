"""Pins for the oracle's double-double refinement (Algorithm 1, Sec. 2.4).

X_true (the fixed point of the double-double iteration) is checked against
results that do not come from the oracle: closed-form 2x2 eigenvectors, a
diagonal matrix, matrices whose eigenvectors are known exactly (an exactly
representable Householder similarity), the secular-equation eigenvectors of a
diagonal-plus-rank-one matrix, the identity W = S + R D off the diagonal,
Theorem 1's bound, and the quadratic fall of the correction norm.
"""
from decimal import Decimal, getcontext
from fractions import Fraction as F

import numpy as np
import pytest

import oracle
import workloads


def _fro_max(a):
    return float(np.max(np.abs(a)))


# ---------------------------------------------------------------- 2x2 closed form
@pytest.mark.parametrize("a,b,c", [(2.0, 1.0, 2.0), (1.0, 1e-3, 0.5), (3.0, -2.5, -1.0),
                                   (1e-8, 1e-9, 3e-8), (0.7, 0.7, 0.2)])
def test_2x2_closed_form(a, b, c):
    """[[a, b], [b, c]]: lambda = (a+c)/2 -+ sqrt(((a-c)/2)^2 + b^2), x = (b, lambda - a)."""
    A = np.asfortranarray([[a, b], [b, c]])
    w, X0 = np.linalg.eigh(A)
    Xh, Xl, lh, ll, _ = oracle.refine_dd(A, np.asfortranarray(X0))
    getcontext().prec = 60
    Da, Db, Dc = Decimal(a), Decimal(b), Decimal(c)
    rad = (((Da - Dc) / 2) ** 2 + Db * Db).sqrt()
    for j, lam in enumerate([(Da + Dc) / 2 - rad, (Da + Dc) / 2 + rad]):
        x = [Db, lam - Da]
        nrm = (x[0] ** 2 + x[1] ** 2).sqrt()
        x = [x[0] / nrm, x[1] / nrm]
        got = [Decimal(Xh[i, j]) + Decimal(Xl[i, j]) for i in range(2)]
        if got[0] * x[0] + got[1] * x[1] < 0:
            x = [-x[0], -x[1]]
        for i in range(2):
            assert abs(got[i] - x[i]) < Decimal("1e-28"), (i, j)
        assert abs(Decimal(lh[j]) + Decimal(ll[j]) - lam) < Decimal("1e-28") * max(abs(lam), Decimal(1e-8))


# ---------------------------------------------------------------- diagonal
def test_diagonal_identity_fixed_point():
    """For diagonal A the eigenvectors are the unit vectors; X = I is a fixed point and a
    rotated start returns to it."""
    n = 12
    A = np.asfortranarray(np.diag(np.linspace(1.0, 2.0, n) ** 3))
    Xh = np.asfortranarray(np.eye(n)); Xl = np.zeros((n, n), order="F")
    st = oracle.refine_dd_step(A, Xh, Xl)
    assert st.emax == 0.0
    assert np.array_equal(Xh, np.eye(n)) and not Xl.any()
    np.testing.assert_array_equal(st.lam_h, np.diag(A))
    th = 1e-4
    R = np.eye(n); R[3, 3] = R[7, 7] = np.cos(th); R[3, 7] = -np.sin(th); R[7, 3] = np.sin(th)
    Xh, Xl, lh, ll, _ = oracle.refine_dd(A, np.asfortranarray(R))
    assert _fro_max(Xh - np.eye(n)) < 1e-30 and _fro_max(Xl) < 1e-30


# ---------------------------------------------------------------- exact Householder
def _exact_householder(n, m, seed):
    rng = np.random.default_rng(seed)
    v = np.zeros(n)
    idx = rng.choice(n, m, replace=False)
    v[idx] = rng.choice([-1.0, 1.0], m)
    H = np.eye(n) - (2.0 / m) * np.outer(v, v)     # entries dyadic: 2/m is a power of two
    mant = rng.choice(np.arange(513, 1024, 2), n, replace=False).astype(np.float64)
    lam = mant * 2.0 ** -rng.integers(0, 28, n).astype(np.float64)
    A = (H * lam) @ H
    # the FP64 product is exact: compare with rational arithmetic
    FH = [[F(x) for x in row] for row in H]
    for i in range(n):
        for j in range(n):
            ex = sum(FH[i][k] * F(lam[k]) * FH[k][j] for k in range(n))
            assert F(A[i, j]) == ex
    return np.asfortranarray(A), H, lam


@pytest.mark.parametrize("seed", [0, 1])
def test_exact_householder_family(seed):
    """A = H diag(lam) H with dyadic H and lam is stored exactly, so X = H and D = diag(lam)."""
    n = 24
    A, H, lam = _exact_householder(n, 16, seed)
    w, X0 = np.linalg.eigh(A)
    Xh, Xl, lh, ll, hist = oracle.refine_dd(A, np.asfortranarray(X0))
    order = np.argsort(lam)
    Xref = H[:, order]
    Xref = oracle.sign_align(Xh, Xref)
    assert _fro_max((Xh - Xref) + Xl) < 1e-28
    np.testing.assert_array_equal(lh, lam[order])


# ---------------------------------------------------------------- secular equation
@pytest.mark.parametrize("n,c", [(48, 4.0), (96, 6.0)])
def test_secular_rank_one(n, c):
    """diag(d) + rho u u^T: the refinement's fixed point equals (D - lambda I)^-1 u normalised,
    with lambda from the secular equation solved independently in double-double."""
    A, d, rho, u = workloads.diag_rank1_problem(n, seed=n, c=c)
    dh, dl, perm = oracle.exact_diag_rank1(A, rho, u)
    lam_h, lam_l, Sh, Sl = oracle.secular_rank1(dh, dl, rho, u[perm])
    # eigenvectors in the permuted basis -> original coordinates
    Xs = np.zeros((n, n)); Xs[perm, :] = Sh
    Xsl = np.zeros((n, n)); Xsl[perm, :] = Sl
    w, X0 = np.linalg.eigh(A)
    Xh, Xl, lh, ll, _ = oracle.refine_dd(A, np.asfortranarray(X0))
    s = np.sign(np.sum(Xh * Xs, axis=0))
    diff = (Xh - Xs * s) + (Xl - Xsl * s)
    gap = np.min(np.diff(lam_h))
    tol = 1e-30 * np.max(np.abs(lam_h)) / gap * 100
    assert _fro_max(diff) < max(tol, 1e-26), (_fro_max(diff), tol)
    np.testing.assert_allclose(lh, lam_h, rtol=1e-25, atol=0)


def test_secular_solver_residual():
    """The secular solver's eigenpairs satisfy A x = lambda x in double-double."""
    n = 40
    A, d, rho, u = workloads.diag_rank1_problem(n, seed=3, c=3.0)
    dh, dl, perm = oracle.exact_diag_rank1(A, rho, u)
    lam_h, lam_l, Sh, Sl = oracle.secular_rank1(dh, dl, rho, u[perm])
    X = np.zeros((n, n)); X[perm, :] = Sh
    Xl = np.zeros((n, n)); Xl[perm, :] = Sl
    Vh, Vl = oracle.dd_gemm(A, np.asfortranarray(X), None, np.asfortranarray(Xl))
    XDh, XDl = oracle.dd_gemm(np.asfortranarray(X), np.asfortranarray(np.diag(lam_h)),
                              np.asfortranarray(Xl), np.asfortranarray(np.diag(lam_l)))
    res = (Vh - XDh) + (Vl - XDl)
    assert _fro_max(res) < 1e-28 * np.max(np.abs(lam_h))
    G = X.T @ X
    assert _fro_max(G - np.eye(n)) < 1e-14


# ---------------------------------------------------------------- two starts
def test_two_starts_same_fixed_point():
    p1 = workloads.make_problem(1, 100, x0="eigh")
    p2 = workloads.make_problem(1, 100, x0="q")
    assert p1.meta["digest"] == p2.meta["digest"]
    X1, X1l, _, _, _ = oracle.refine_dd(p1.A, p1.X0)
    X2, X2l, _, _, _ = oracle.refine_dd(p2.A, p2.X0)
    X2s = oracle.sign_align(X1, X2)
    assert _fro_max(X1 - X2s) < 1e-20


# ---------------------------------------------------------------- quadratic fall
def test_quadratic_fall():
    """Theorem 1: while the error is well above the floor, max|E~| falls roughly quadratically."""
    p = workloads.make_problem(2, 256, x0="eigh")
    Xh = np.asfortranarray(p.X0.copy()); Xl = np.zeros_like(Xh, order="F")
    hist = []
    for _ in range(4):
        hist.append(oracle.refine_dd_step(p.A, Xh, Xl).emax)
    assert hist[0] > 1e-7
    for k in range(len(hist) - 1):
        if hist[k + 1] > 1e-17:  # the double-double floor here is about 1e-21
            assert np.log(hist[k + 1]) / np.log(hist[k]) > 1.6, hist


# ---------------------------------------------------------------- Theorem 1 bound
def test_theorem1_bound():
    """||E - E~|| <= 6.4 sqrt(n) ||A|| eps^2 / (gap - 14 ||A|| eps) when
    eps < min(gap / (10 sqrt(n) ||A||), 1/100)."""
    n = 10
    rng = workloads.rng_for(77)
    V = workloads.householder_vectors(rng, n, 4)
    lam = np.linspace(1.0, 2.0, n)
    A = workloads.householder_matrix(lam, V)
    w, X0 = np.linalg.eigh(A)
    Xt, Xtl, _, _, _ = oracle.refine_dd(A, np.asfortranarray(X0))
    normA = np.linalg.norm(A, 2)
    gap = np.min(np.diff(np.sort(lam)))
    for scale in (3e-5, 1e-4, 3e-4):
        Xh = np.asfortranarray(Xt + scale * rng.standard_normal((n, n)) / np.sqrt(n))
        E = np.linalg.solve(Xh, Xt) - np.eye(n)
        eps = np.linalg.norm(E, 2)
        assert eps < min(gap / (10 * np.sqrt(n) * normA), 0.01)
        st = oracle.refine_dd_step(A, Xh.copy(order="F"), np.zeros((n, n), order="F"), want_E=True)
        bound = 6.4 * np.sqrt(n) * normA * eps ** 2 / (gap - 14 * normA * eps)
        assert np.linalg.norm(E - st.E, 2) <= bound


# ---------------------------------------------------------------- W identity
def test_w_identity():
    """W = X^T (A X - X D) has w_ij = s_ij + lambda_j r_ij off the diagonal, with
    S = X^T A X and R = I - X^T X formed by separate double-double products."""
    n = 20
    p = workloads.make_problem(1, n, x0="eigh")
    rng = np.random.default_rng(5)
    X = np.asfortranarray(p.X0 + 1e-5 * rng.standard_normal((n, n)))
    st = oracle.refine_dd_step(p.A, X.copy(order="F"), np.zeros((n, n), order="F"), want_E=True)
    AXh, AXl = oracle.dd_gemm(p.A, X)
    Sh, _ = oracle.dd_gemm(X, AXh, None, AXl, transA=True)
    Gh, _ = oracle.dd_gemm(X, X, transA=True)
    R = np.eye(n) - Gh
    lam = st.lam_h
    for i in range(n):
        for j in range(n):
            if i == j:
                assert abs(st.E[i, j] - st.r[i] / 2) <= 1e-30
                continue
            w = st.E[i, j] * (lam[j] - lam[i])
            expect = Sh[i, j] + lam[j] * R[i, j]
            assert abs(w - expect) <= 1e-9 * abs(expect) + 1e-22, (i, j, w, expect)
