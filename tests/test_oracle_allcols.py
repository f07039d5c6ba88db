"""Pins of the all-column forward-error check (oracle/dd_numpy.py, oracle/allcols.c): the
error-free FP64 slice products against exact integers and the C oracle's double-double
product, and the one-step estimate against forward errors known exactly."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads
from oracle import dd_numpy as dn


def test_slice_products_are_exact():
    """With alpha from the reduction length (eq. alp_beta), every FP64 product of two
    slices equals the exact rational product: any summation order gives the same bits."""
    rng = np.random.default_rng(1)
    m, K, n = 6, 512, 5
    L = rng.standard_normal((m, K)) * 2.0 ** rng.integers(-30, 30, (m, 1))
    R = rng.standard_normal((K, n)) * 2.0 ** rng.integers(-30, 30, (1, n))
    a = dn.slice_alpha(K)
    Ls, Rs = dn.row_slices(L, 3, a), dn.col_slices(R, 3, a)
    for r in range(3):
        for s in range(3):
            P = Ls[r] @ Rs[s]
            Pt = np.ascontiguousarray(Rs[s].T) @ np.ascontiguousarray(Ls[r].T)   # other order
            for i in range(m):
                for j in range(n):
                    exact = sum(Fraction(float(x)) * Fraction(float(y))
                                for x, y in zip(Ls[r][i], Rs[s][:, j]))
                    assert Fraction(float(P[i, j])) == exact
                    assert Pt[j, i] == P[i, j]


def test_dd_product_matches_the_c_oracle():
    rng = np.random.default_rng(2)
    m, K, n = 90, 300, 70
    L = np.asfortranarray(rng.standard_normal((m, K)) * 2.0 ** rng.integers(-20, 20, (m, K)))
    R = np.asfortranarray(rng.standard_normal((K, n)) * 2.0 ** rng.integers(-20, 20, (K, n)))
    h, l = dn.dd_product(L, R)
    ch, cl = oracle.dd_gemm(L, R)
    scale = np.abs(L) @ np.abs(R)
    diff = np.abs((h - ch) + (l - cl))
    assert float(np.max(diff / scale)) < 2.0 ** -100
    # a transposed operand is caught
    h2, _ = dn.dd_product(L, np.asfortranarray(R[::-1]))
    assert float(np.max(np.abs(h2 - ch) / scale)) > 1e-3


def _xtrue(cfg, n):
    p = workloads.make_problem(cfg, n, x0="eigh")
    Xh, Xl, lh, ll, _ = oracle.refine_dd(p.A, p.X0)
    return p, Xh, Xl, lh, ll


@pytest.mark.parametrize("cfg,n", [(3, 300), (2, 257)])
def test_estimate_of_the_rounded_true_eigenvectors(cfg, n):
    """X = the FP64 high words of X_true: the exact forward error is the low words, about
    1e-17, at condition 1e12. The one-step estimate finds it column by column, which needs
    double-double products down to the smallest gaps."""
    p, Xh, Xl, lh, ll = _xtrue(cfg, n)
    res = dn.allcols_forward_error(p.A, Xh, lh)
    true = np.max(np.abs(Xl), axis=0)
    assert np.all(np.abs(res["est"] - true) <= 1e-3 * true + 1e-20), \
        float(np.max(np.abs(res["est"] - true)))
    assert float(np.max(res["second"])) < 1e-20
    # the Rayleigh quotients of the high words against the eigenvalues of X_true, to the
    # accuracy each column's products were sized for (resolve 1e-17 of its gap)
    g = dn._gaps(lh)
    assert np.all(np.abs((res["lam_h"] - lh) + (res["lam_l"] - ll))
                  <= 1e-17 * g + 1e-28 * np.max(np.abs(lh)))


def test_estimate_of_a_perturbed_iterate():
    """Perturbations of known size in known entries: the estimate returns them."""
    p, Xh, Xl, lh, ll = _xtrue(1, 200)
    rng = np.random.default_rng(3)
    X = Xh.copy(order="F")
    cols = rng.choice(200, 12, replace=False)
    rows = rng.integers(0, 200, 12)
    size = 10.0 ** rng.uniform(-14, -11, 12)
    for c, r, z in zip(cols, rows, size):
        X[r, c] += z
    res = dn.allcols_forward_error(p.A, X, lh)
    true = np.max(np.abs((Xh - X) + Xl), axis=0)
    assert np.all(np.abs(res["est"] - true) <= 1e-3 * true + 1e-18)
    assert np.all(res["est"][cols] > 0.99 * size)
