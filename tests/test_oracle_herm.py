"""Pins of the complex Hermitian oracle (the Hermitian extension of Algorithm 1, which
Sec. 5 names as future work) against facts that do not come from the oracle itself:

* a real symmetric A with a real X is a special case: every output equals the real
  oracle's, bit for bit (the real oracle is pinned in test_oracle_*.py);
* unitary diagonal similarity with phases in {1, i, -1, -i} (exact in FP64):
  A' = P A P^H, X' = P X must give X'_new = P X_new and the same eigenvalues. A dropped
  conjugation, a transposed operand or a wrong sign in any imaginary term breaks this;
* the fixed point agrees with LAPACK's complex Hermitian eigensolver on a well-conditioned
  matrix, and its eigenvalues with the construction;
* a 2 x 2 matrix with a closed-form eigensystem;
* the truncation of X^(1) and the beta rule on the component maxima (a reading: both parts
  of a column are cut on one grid).
"""
import numpy as np
import pytest

import oracle
import workloads


def _rough_start(p, scale, seed):
    rng = np.random.default_rng(seed)
    n = p.n
    N = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return np.asfortranarray(p.X0 + scale * N)


def _phases(n, seed):
    rng = np.random.default_rng(seed)
    return np.array([1.0, 1j, -1.0, -1j])[rng.integers(0, 4, n)]


def test_real_case_matches_real_oracle_bitwise():
    p = workloads.make_problem(2, 48, x0="eigh")
    X0 = p.X0 + 1e-6 * np.random.default_rng(1).standard_normal(p.X0.shape)
    Xh, Xl, lh, ll, r, em = oracle.herm_dd_step(p.A.astype(np.complex128), X0.astype(np.complex128))
    Rh, Rl = np.array(X0, order="F"), np.zeros_like(X0, order="F")
    ref = oracle.refine_dd_step(p.A, Rh, Rl)
    assert np.array_equal(Xh.imag, np.zeros_like(Xh.imag)) and np.array_equal(Xl.imag, 0 * Xl.imag)
    assert np.array_equal(Xh.real, Rh) and np.array_equal(Xl.real, Rl)
    assert np.array_equal(lh, ref.lam_h) and np.array_equal(ll, ref.lam_l)
    assert np.array_equal(r, ref.r) and em == ref.emax


def test_real_case_method_step_matches_real_oracle_bitwise():
    p = workloads.make_problem(1, 64, x0="eigh")
    X0 = np.asfortranarray(p.X0 + 1e-7 * np.random.default_rng(2).standard_normal(p.X0.shape))
    for delta in (1e-15, 1e-9):
        a = oracle.herm_method_step(p.A.astype(np.complex128), X0.astype(np.complex128), p.D0, delta)
        b = oracle.method_step(p.A, X0, p.D0, delta)
        assert (a.beta, a.kx) == (b.beta, b.kx)
        assert np.array_equal(a.X1.real, b.X1) and not np.any(a.X1.imag)
        assert np.array_equal(a.X_hi.real, b.X_hi) and np.array_equal(a.lam_h, b.lam_h)


@pytest.mark.parametrize("cfg,n", [(1, 40), (3, 56)])
def test_phase_equivariance(cfg, n):
    p = workloads.hermitian_problem(cfg, n)
    X0 = _rough_start(p, 1e-4, 3)
    P = _phases(n, 4)
    A2 = (P[:, None] * p.A) * np.conj(P)[None, :]
    X2 = P[:, None] * X0
    # exact: multiplication by +-1, +-i only moves and negates parts
    assert np.array_equal(np.abs(A2), np.abs(p.A)) and np.array_equal(np.abs(X2), np.abs(X0))
    Xa, Xal, la, _, ra, ea = oracle.herm_dd_step(p.A, X0)
    Xb, Xbl, lb, _, rb_, eb = oracle.herm_dd_step(A2, X2)
    scale = np.max(np.abs(Xa - X0))     # size of the correction (about 1e-4)
    assert scale > 1e-6
    # double-double agreement: differences far below the correction itself
    assert np.max(np.abs((Xb + Xbl) - P[:, None] * (Xa + Xal))) <= 1e-25
    assert np.max(np.abs(lb - la)) <= 1e-25 * np.max(np.abs(la))
    assert np.max(np.abs(rb_ - ra)) <= 1e-25 and abs(eb - ea) <= 1e-12 * ea


def test_phase_equivariance_method_step():
    p = workloads.hermitian_problem(2, 48)
    X0 = _rough_start(p, 1e-6, 5)
    P = _phases(p.n, 6)
    A2 = (P[:, None] * p.A) * np.conj(P)[None, :]
    X2 = P[:, None] * X0
    a = oracle.herm_method_step(p.A, X0, p.D0, 1e-15)
    b = oracle.herm_method_step(A2, X2, p.D0, 1e-15)
    assert (a.beta, a.kx) == (b.beta, b.kx)
    # the truncation commutes with the phases exactly (the column's component maximum and
    # every digit move with the parts)
    assert np.array_equal(b.X1, P[:, None] * a.X1)
    assert np.max(np.abs((b.X_hi + b.X_lo) - P[:, None] * (a.X_hi + a.X_lo))) <= 1e-25


def test_fixed_point_matches_lapack_well_conditioned():
    n = 32
    rng = np.random.default_rng(7)
    lam = 1.0 + np.arange(n) / n            # gaps 1/n, condition about 2
    A = workloads.hermitian_matrix(lam, rng.standard_normal((n, 4)), rng.standard_normal((n, 4)))
    w, V = np.linalg.eigh(A)
    X0 = np.asfortranarray(V + 1e-5 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))))
    Xh, Xl, lamd, hist = oracle.refine_dd_herm(A, X0)
    assert hist[-1] < 1e-25
    assert np.max(np.abs(Xh - oracle.phase_align(Xh, V))) <= 2e-14
    assert np.max(np.abs(np.sort(lamd) - w)) <= 1e-14
    assert np.max(np.abs(np.sort(lamd) - np.sort(lam))) <= 1e-14


def test_two_by_two_closed_form():
    # A = [[3, 1+i], [1-i, 1]]: eigenvalues 2 +- sqrt(3); for 2 + sqrt(3) the eigenvector
    # is proportional to (1 + i, sqrt(3) - 1), for 2 - sqrt(3) to (1 + i, -sqrt(3) - 1).
    A = np.asfortranarray(np.array([[3.0, 1 + 1j], [1 - 1j, 1.0]]))
    s3 = np.sqrt(3.0)
    V = np.array([[1 + 1j, 1 + 1j], [-s3 - 1, s3 - 1]])
    V = V / np.linalg.norm(V, axis=0)       # columns: lambda = 2 - sqrt 3, 2 + sqrt 3
    t = 0.05                                # a rotated, phase-shifted start
    R = np.array([[np.cos(t), -np.sin(t)], [np.sin(t), np.cos(t)]])
    X0 = np.asfortranarray((V @ R) * np.exp(0.3j))
    Xh, Xl, lam, hist = oracle.refine_dd_herm(A, X0)
    assert np.max(np.abs(lam - np.array([2 - s3, 2 + s3]))) <= 4e-16
    assert np.max(np.abs(Xh - oracle.phase_align(Xh, V))) <= 4e-16
    # quadratic convergence from the rotated start
    assert hist[1] <= 10 * hist[0] ** 2 and hist[2] <= 10 * hist[1] ** 2


def test_truncation_grid_and_beta_on_component_maxima():
    p = workloads.hermitian_problem(1, 40)
    X0 = _rough_start(p, 1e-3, 8)
    delta = 1e-12
    a = oracle.herm_method_step(p.A, X0, p.D0, delta)
    for j in range(p.n):
        m = max(np.max(np.abs(X0[:, j].real)), np.max(np.abs(X0[:, j].imag)))
        e = int(np.frexp(m)[1])
        ulp = 2.0 ** (e - 7 * a.kx)
        for part, part1 in ((X0[:, j].real, a.X1[:, j].real), (X0[:, j].imag, a.X1[:, j].imag)):
            q = part1 / ulp
            assert np.array_equal(q, np.trunc(q))             # on the grid
            assert np.all(np.abs(part - part1) < ulp)          # truncated toward zero
            assert np.all(np.abs(part1) <= np.abs(part))
    # beta and kx: the real rule on any real matrix with the same column maxima
    wmax = np.maximum(np.abs(X0.real).max(axis=0), np.abs(X0.imag).max(axis=0))
    Y = np.zeros((p.n, p.n), order="F")
    Y[0, :] = wmax
    rr = oracle.beta_rule(p.D0, Y, delta)
    assert (a.beta, a.kx) == (rr["beta"], rr["kx"])
    hb = oracle.herm_beta_rule(p.D0, 1j * X0.real + X0.imag, delta)   # parts swapped
    assert (hb["beta"], hb["kx"]) == (a.beta, a.kx)
