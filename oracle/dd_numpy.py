"""The error-free slice products of the Ozaki scheme (Sec. 2.3) on the host's FP64 BLAS,
and a check of the forward error of every column of an eigenvector matrix — test
infrastructure.

Only the tests, ``__graft_entry__.smoke()`` and ``bench.py`` (its CPU legs) may import
this module. The GPU library neither links nor calls it; the two share no code.

Why it exists: the C oracle's double-double products (``oracle.dd_gemm``) take minutes per
n x n x n product at n = 8192. The Ozaki scheme itself gives double-double products from
FP64 matrix products: split each factor by rows / columns into FP64 slices with the
extraction of eq. (a)/(x) (the oracle's ``sigma_split``), sized so that every slice product
is exact in FP64 for the reduction length (eq. alp_beta, alpha + beta >= 53 + log2 n); then
any FP64 GEMM returns those products exactly, whatever its summation order, and their sum
is accumulated in double-double (the element-wise and column passes are plain C in
``allcols.c``, with the double-double arithmetic of ``dd.h``).

``allcols_forward_error`` takes one double-double step of Algorithm 1 (Sec. 2.4) from a
given X: the first-order correction X E~ is X_true - X up to second-order terms, so
max_i |(X E~)_ij| estimates the forward error of column j, for every column at once.
"""
from __future__ import annotations

import numpy as np

# ---------------------------------------------------------------- error-free slice products
def slice_alpha(k):
    """alpha = beta of eq. (alp_beta) for reduction length k: alpha + beta >= 53 + log2 k,
    so each slice keeps 53 - alpha bits and every slice product is exact in FP64."""
    return int(np.ceil((53.0 + np.log2(max(k, 2))) / 2.0))


def row_slices(M, ns, alpha):
    """ns FP64 slices of M by rows (eq. a, sigma_i per row); remainder dropped."""
    from . import sigma_split
    sl, _ = sigma_split(M, alpha, ns, by_rows=True)
    return sl


def col_slices(M, ns, alpha):
    """ns FP64 slices of M by columns (eq. x, tau_j per column); remainder dropped."""
    from . import sigma_split
    sl, _ = sigma_split(M, alpha, ns, by_rows=False)
    return sl


def _ptr(a):
    import ctypes
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def ozaki_product(Ls, Rs, dmax):
    """sum over slice pairs (r, s), r + s <= dmax (1-based), of Ls[r] @ Rs[s]: every pair
    product is exact in FP64 (slices from row_slices / col_slices with slice_alpha of the
    reduction length); the sum is accumulated in double-double, smallest pairs first.
    Returns (hi, lo), Fortran order."""
    from . import _load
    lib = _load()
    acc_h = acc_l = None
    for d in range(dmax, 1, -1):
        for r in range(1, d):
            s = d - r
            if r > len(Ls) or s > len(Rs):
                continue
            P = np.asfortranarray(Ls[r - 1] @ Rs[s - 1])
            if acc_h is None:
                acc_h, acc_l = P, np.zeros_like(P, order="F")
            else:
                lib.or_dd_acc(P.size, _ptr(acc_h), _ptr(acc_l), _ptr(P))
            del P
    lib.or_dd_norm(acc_h.size, _ptr(acc_h), _ptr(acc_l))
    return acc_h, acc_l


def dd_product(L, R, dmax=7, ns=6):
    """L @ R (FP64 factors) to double-double accuracy: ns slices of 53 - alpha bits each
    (alpha from the reduction length), pairs r + s <= dmax."""
    a = slice_alpha(L.shape[1])
    return ozaki_product(row_slices(L, ns, a), col_slices(R, ns, a), dmax)


# ---------------------------------------------------------------- all-column forward error
def _pairs_for_gap(g, lmax, n, resolve=1e-17):
    """Last slice-pair diagonal of the V product for a column with eigenvalue gap g: V's
    dropped pairs (about 2^(-b (d - 1)) sqrt(n) max|lambda| with b-bit slices) must stay within
    resolve * g, so that they move that column's correction by less than `resolve`."""
    b = 53 - slice_alpha(n)
    need = np.log2(np.sqrt(n) * 8.0 * lmax / (resolve * np.maximum(g, 1e-300)))
    return int(np.clip(np.ceil(need / b) + 1, 4, 8))


def _gaps(lam):
    o = np.argsort(lam, kind="stable")
    s = lam[o]
    d = np.diff(s)
    g = np.empty_like(s)
    g[0], g[-1] = d[0], d[-1]
    g[1:-1] = np.minimum(d[:-1], d[1:])
    out = np.empty_like(g)
    out[o] = g
    return out


def allcols_forward_error(A, X, lam_est, resolve=1e-17, ns=6, log=None):
    """One double-double step of Algorithm 1 from X (n x n FP64, columns = eigenvectors):
        V = A X, r_j = 1 - x_j^T x_j, lambda_j = x_j^T v_j / (1 - r_j),
        W = X^T (V - X diag(lambda)), e_ij = w_ij / (lambda_j - lambda_i), e_jj = r_j / 2.
    X + X E~ is X_true up to terms of second order in the error of X, so column j's
    forward error (max-abs, against the eigenvector with X's sign) is estimated by
    est_j = max_i |(X E~)_ij|. lam_est (n): eigenvalue estimates that fix each column's
    product accuracy (their gaps; any estimates good to a small fraction of the gaps).
    Returns a dict: est (n), eps_j = max_{i != j} |e_ij|, lam_h / lam_l (double-double
    Rayleigh quotients), second_j = eps_j^2 max|lambda| / gap_j (the size of the neglected
    second-order term, by the eq. (assume2) model with xi = 1)."""
    import time
    from . import _load
    lib = _load()
    A = np.asfortranarray(A, dtype=np.float64)
    X = np.asfortranarray(X, dtype=np.float64)
    n = A.shape[0]
    lam_est = np.asarray(lam_est, dtype=np.float64)
    lmax = float(np.max(np.abs(lam_est)))
    gaps = _gaps(lam_est)
    alpha = slice_alpha(n)
    t0 = time.perf_counter()
    Asl = row_slices(A, ns, alpha)
    # V = A X: columns in groups by the slice pairs their gap needs
    dcol = np.array([_pairs_for_gap(g, lmax, n, resolve) for g in gaps])
    Vh = np.empty((n, n), order="F")
    Vl = np.empty((n, n), order="F")
    for d in sorted(set(dcol.tolist())):
        cols = np.nonzero(dcol == d)[0]
        Xs = col_slices(np.asfortranarray(X[:, cols]), ns, alpha)
        h, l = ozaki_product(Asl, Xs, d)
        Vh[:, cols], Vl[:, cols] = h, l
        del Xs, h, l
        if log:
            log(f"V: {len(cols)} columns with slice pairs up to {d} "
                f"({time.perf_counter() - t0:.1f} s)")
    del Asl
    # column pass: r_j, lambda_j, and V <- V - X diag(lambda) (the residual R), in place
    lam_h, lam_l, r_h, r_l = (np.empty(n) for _ in range(4))
    lib.or_colpass(n, n, _ptr(X), _ptr(Vh), _ptr(Vl), _ptr(lam_h), _ptr(lam_l), _ptr(r_h),
                   _ptr(r_l))
    # W = X^T R: the high words by slices (pairs r + s <= 5 give about 2^-80 of |X|^T |R|,
    # far below what the smallest gaps need), the low words in FP64
    XT = np.ascontiguousarray(X.T)
    Wh, Wl = ozaki_product(row_slices(XT, 4, alpha), col_slices(Vh, 4, alpha), 5)
    Wl += XT @ Vl
    del Vh, Vl
    if log:
        log(f"W done ({time.perf_counter() - t0:.1f} s)")
    E = np.empty((n, n), order="F")
    eps = np.empty(n)
    lib.or_form_e(n, _ptr(Wh), _ptr(Wl), _ptr(lam_h), _ptr(lam_l), _ptr(r_h), _ptr(r_l),
                  _ptr(E), _ptr(eps))
    del Wh, Wl
    est = np.max(np.abs(X @ E), axis=0)
    if log:
        log(f"all-column estimate done ({time.perf_counter() - t0:.1f} s)")
    second = eps ** 2 * lmax / gaps
    return {"est": est, "eps": eps, "lam_h": lam_h, "lam_l": lam_l, "second": second,
            "seconds": time.perf_counter() - t0}
