"""CPU oracle (double-double) for eigenvector refinement — test infrastructure.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The GPU library neither links nor calls
it, and the two share no code.

Every function below wraps the plain C implementation in ``oracle.c``; see
that file for the passage of the paper each one follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

CFLAGS = ["-O3", "-mavx2", "-mfma", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
          "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    srcs = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "oracle_herm.c"),
            os.path.join(_HERE, "allcols.c")]
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, *srcs, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)
_I8 = ctypes.POINTER(ctypes.c_int8)
_I64 = ctypes.POINTER(ctypes.c_int64)
_c_int, _c_double = ctypes.c_int, ctypes.c_double


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        lib.or_num_threads.restype = _c_int
        lib.or_dd_gemm.argtypes = [_c_int, _c_int, _c_int, _c_int, _D, _D, _c_int, _D, _D, _c_int,
                                   _D, _D, _c_int]
        lib.or_refine_dd_step.argtypes = [_c_int, _D, _D, _D, _D, _D, _D, _D, _D]
        lib.or_split_s7.argtypes = [_c_int, _c_int, _c_int, _D, _c_int, _c_int, _I, _I8, _D]
        lib.or_slice_gemm_i64.argtypes = [_c_int, _c_int, _c_int, _I8, _c_int, _I8, _c_int, _I64]
        lib.or_sigma_split.argtypes = [_c_int, _c_int, _c_int, _D, _c_int, _c_int, _c_int, _D]
        lib.or_beta_rule.argtypes = [_c_int, _D, _D, _c_int, _c_double, _c_double, _c_int, _I, _I,
                                     _D, _D, _D]
        lib.or_method_step.argtypes = [_c_int, _D, _D, _D, _c_double, _c_double, _c_int, _c_int,
                                       _D, _D, _D, _D, _D, _D, _D, _I, _I]
        lib.or_method_step_grouped.argtypes = [_c_int, _D, _D, _D, _c_double, _c_double, _c_int,
                                               _c_int, _D, _D, _D, _D, _D, _D, _D, _I, _I,
                                               _c_double, _I]
        lib.or_refine_dd_step_grouped.argtypes = [_c_int, _D, _D, _D, _D, _D, _D, _D, _D,
                                                  _c_double, _I]
        lib.or_secular_rank1.argtypes = [_c_int, _D, _D, _c_double, _D, _D, _D, _D, _D, _c_int,
                                         _c_int]
        lib.or_herm_dd_step.argtypes = [_c_int, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D]
        lib.or_herm_beta_rule.argtypes = [_c_int, _D, _D, _D, _c_double, _c_double, _c_int, _I,
                                          _I]
        lib.or_herm_method_step.argtypes = [_c_int, _D, _D, _D, _D, _D, _c_double, _c_double,
                                            _c_int, _c_int, _D, _D, _D, _D, _D, _D, _D, _D, _D,
                                            _D, _I, _I]
        lib.or_dd_acc.argtypes = [ctypes.c_size_t, _D, _D, _D]
        lib.or_dd_norm.argtypes = [ctypes.c_size_t, _D, _D]
        lib.or_colpass.argtypes = [_c_int, _c_int, _D, _D, _D, _D, _D, _D, _D]
        lib.or_form_e.argtypes = [_c_int, _D, _D, _D, _D, _D, _D, _D, _D]
        lib.or_two_sum.argtypes = [_c_double, _c_double, _D, _D]
        lib.or_two_prod.argtypes = [_c_double, _c_double, _D, _D]
        lib.or_dd_binop.argtypes = [_c_int, _c_double, _c_double, _c_double, _c_double, _D, _D]
        _lib = lib
    return _lib


def two_sum(a, b):
    s = ctypes.c_double(); e = ctypes.c_double()
    _load().or_two_sum(float(a), float(b), ctypes.byref(s), ctypes.byref(e))
    return s.value, e.value


def two_prod(a, b):
    s = ctypes.c_double(); e = ctypes.c_double()
    _load().or_two_prod(float(a), float(b), ctypes.byref(s), ctypes.byref(e))
    return s.value, e.value


_OPS = {"add": 0, "mul": 1, "div": 2, "sqrt": 3, "pair": 4}


def dd_op(op, a, b=(0.0, 0.0)):
    """Double-double add/mul/div/sqrt/pair-add on (hi, lo) tuples."""
    rh = ctypes.c_double(); rl = ctypes.c_double()
    _load().or_dd_binop(_OPS[op], float(a[0]), float(a[1]), float(b[0]), float(b[1]),
                        ctypes.byref(rh), ctypes.byref(rl))
    return rh.value, rl.value


def _f64(a, order="F"):
    return np.require(a, dtype=np.float64, requirements=[order, "A", "W"])


def _p(a):
    if a is None:
        return None
    if a.dtype == np.float64:
        return a.ctypes.data_as(_D)
    if a.dtype == np.int8:
        return a.ctypes.data_as(_I8)
    if a.dtype == np.int64:
        return a.ctypes.data_as(_I64)
    if a.dtype == np.int32:
        return a.ctypes.data_as(_I)
    raise TypeError(a.dtype)


def num_threads() -> int:
    return _load().or_num_threads()


def dd_gemm(A_hi, B_hi, A_lo=None, B_lo=None, transA=False):
    """op(A) @ B in double-double; returns (C_hi, C_lo) (Fortran order)."""
    A_hi = _f64(A_hi); B_hi = _f64(B_hi)
    A_lo = None if A_lo is None else _f64(A_lo)
    B_lo = None if B_lo is None else _f64(B_lo)
    m = A_hi.shape[1] if transA else A_hi.shape[0]
    k = A_hi.shape[0] if transA else A_hi.shape[1]
    n = B_hi.shape[1]
    Ch = np.empty((m, n), order="F"); Cl = np.empty((m, n), order="F")
    _load().or_dd_gemm(int(transA), m, n, k, _p(A_hi), _p(A_lo), A_hi.shape[0], _p(B_hi), _p(B_lo),
                       B_hi.shape[0], _p(Ch), _p(Cl), m)
    return Ch, Cl


class DDStep:
    def __init__(self, lam_h, lam_l, r, emax, E=None):
        self.lam_h, self.lam_l, self.r, self.emax, self.E = lam_h, lam_l, r, emax, E


def refine_dd_step(A, X_hi, X_lo, want_E=False, tau=0.0):
    """One iteration of Algorithm 1 in double-double. X_hi/X_lo updated in place.
    tau > 0: columns i, j whose first-order correction |e_ij| exceeds tau are grouped and
    corrected by the Rayleigh-Ritz problem on their span (or_refine_dd_step_grouped);
    the number of groups is returned in .groups."""
    n = A.shape[0]
    A = _f64(A)
    lam_h = np.empty(n); lam_l = np.empty(n); r = np.empty(n); em = np.zeros(1)
    E = np.empty((n, n), order="F") if want_E else None
    g = ctypes.c_int(0)
    st = _load().or_refine_dd_step_grouped(n, _p(A), _p(X_hi), _p(X_lo), _p(lam_h), _p(lam_l),
                                           _p(r), _p(E), _p(em), float(tau), ctypes.byref(g))
    if st != 0:
        raise RuntimeError(f"or_refine_dd_step status {st}")
    out = DDStep(lam_h, lam_l, r, float(em[0]), E)
    out.groups = g.value
    return out


def refine_dd(A, X0, max_iter=12, tol=1e-28, verbose=False):
    """Iterate Algorithm 1 in double-double from X0 to its fixed point.

    Stops when max|E~| <= tol, or when max|E~| no longer falls by 10x (the
    double-double floor). Returns (X_hi, X_lo, lam_h, lam_l, history)."""
    X_hi = _f64(np.array(X0, dtype=np.float64, order="F"))
    X_lo = np.zeros_like(X_hi, order="F")
    hist = []
    st = None
    for _ in range(max_iter):
        st = refine_dd_step(A, X_hi, X_lo)
        hist.append(st.emax)
        if verbose:
            print(f"  dd iter {len(hist)}: max|E| = {st.emax:.3e}", flush=True)
        if st.emax <= tol:
            break
        if len(hist) >= 3 and hist[-1] > 0.1 * hist[-2] and hist[-2] < 1e-10:
            break
    # Rayleigh quotients of the final iterate
    fin = _rayleigh_dd(A, X_hi, X_lo)
    return X_hi, X_lo, fin[0], fin[1], hist


def _rayleigh_dd(A, X_hi, X_lo):
    Xh = X_hi.copy(order="F"); Xl = X_lo.copy(order="F")
    st = refine_dd_step(A, Xh, Xl)
    return st.lam_h, st.lam_l


def split_s7(M, k, by_rows=False):
    """7-bit digit planes. Returns (exps int32, planes int8 (k, ...), truncated value).

    by_rows=False: planes[r] has shape (ncols, m): planes[r][j, i] = digit of M[i, j]
    (each column's K-run contiguous). by_rows=True: planes[r][i, j]."""
    M = _f64(M)
    m, nc = M.shape
    nvec = m if by_rows else nc
    ex = np.empty(nvec, dtype=np.int32)
    pl = np.empty(k * m * nc, dtype=np.int8)
    tr = np.empty((m, nc), order="F")
    st = _load().or_split_s7(int(by_rows), m, nc, _p(M), m, k, _p(ex), _p(pl), _p(tr))
    if st != 0:
        raise RuntimeError(f"or_split_s7 status {st}")
    pl = pl.reshape(k, m, nc) if by_rows else pl.reshape(k, nc, m)
    return ex, pl, tr


def slice_gemm_i64(Ap, Bp):
    """Exact C[i, j] = sum_p Ap[i, p] * Bp[j, p] (both K-contiguous rows)."""
    Ap = np.ascontiguousarray(Ap, dtype=np.int8)
    Bp = np.ascontiguousarray(Bp, dtype=np.int8)
    m, K = Ap.shape
    n = Bp.shape[0]
    C = np.empty((m, n), dtype=np.int64, order="F")
    _load().or_slice_gemm_i64(m, n, K, _p(Ap), K, _p(Bp), K, _p(C))
    return C


def coprime_moduli(count):
    """The first `count` odd moduli <= 255 taken greedily from 255 down, each coprime to
    all taken before it (the modulus set of a Chinese-remainder form of the exact
    product of Sec. 2.3)."""
    from math import gcd
    out = []
    for m in range(255, 2, -2):
        if all(gcd(m, x) == 1 for x in out):
            out.append(m)
        if len(out) == count:
            break
    return out


def _sym(r, m):
    """Residues r in [0, m) to the symmetric range [-(m - 1) / 2, (m - 1) / 2] (m odd)."""
    return np.where(r > m // 2, r - m, r)


def digit_residues(planes, moduli):
    """Residues of the integers that digit planes encode: planes (k, ...) int8 holds digits
    d_0 .. d_{k-1} (most significant first) of z = sum_t d_t 128^(k-1-t); returns (N, ...)
    int8 with z mod m_q in the symmetric range. Horner's rule in int64 (every partial value
    stays below 2^16 in magnitude)."""
    P = np.asarray(planes, dtype=np.int64)
    out = []
    for m in moduli:
        z = np.zeros(P.shape[1:], dtype=np.int64)
        for t in range(P.shape[0]):
            z = np.mod(z * 128 + P[t], m)
        out.append(_sym(z, m))
    return np.asarray(out, dtype=np.int8)


def residue_product(Lres, Rres, moduli):
    """C[q][i, j] = (sum_k Lres[q][i, k] Rres[q][j, k]) mod m_q, symmetric range, int8.
    The FP64 matrix product is exact: every term is below 127^2 and the sums stay far
    below 2^53 for K < 2^38."""
    out = []
    for q, m in enumerate(moduli):
        c = np.asarray(Lres[q], dtype=np.float64) @ np.asarray(Rres[q], dtype=np.float64).T
        assert Lres.shape[-1] < (1 << 38)
        out.append(_sym(np.mod(c.astype(np.int64), m), m))
    return np.asarray(out, dtype=np.int8)


def sigma_split(M, alpha, ns, by_rows=True):
    """FP64 splitting of eq. (a)/(x). Returns (slices (ns, m, n), remainder)."""
    M = _f64(M)
    m, nc = M.shape
    out = np.empty((ns + 1) * m * nc)
    _load().or_sigma_split(int(by_rows), m, nc, _p(M), m, int(alpha), int(ns), _p(out))
    sl = [out[r * m * nc:(r + 1) * m * nc].reshape((m, nc), order="F") for r in range(ns + 1)]
    return sl[:ns], sl[ns]


def beta_rule(lam, X, delta, xi=0.0, kx_max=9):
    """beta (Sec. 4.1) and the plane count kx. Returns dict."""
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    X = _f64(X)
    n = X.shape[0]
    b = ctypes.c_int(); k = ctypes.c_int()
    g = np.zeros(1); L = np.zeros(1); S = np.zeros(1)
    st = _load().or_beta_rule(n, _p(lam), _p(X), n, float(delta), float(xi), int(kx_max),
                              ctypes.byref(b), ctypes.byref(k), _p(g), _p(L), _p(S))
    return {"status": st, "beta": b.value, "kx": k.value, "gap": float(g[0]), "lmax": float(L[0]),
            "S": float(S[0])}


class MethodStep:
    pass


def method_step(A, X, lam_prev, delta, xi=0.0, kx_max=9, kx_force=0, tau=0.0):
    """One iteration of the proposed method with exact (double-double) products
    (tau > 0: with the grouped correction, see refine_dd_step)."""
    A = _f64(A); X = _f64(X)
    lam_prev = np.ascontiguousarray(lam_prev, dtype=np.float64)
    n = A.shape[0]
    out = MethodStep()
    out.X1 = np.empty((n, n), order="F")
    out.X_hi = np.empty((n, n), order="F"); out.X_lo = np.empty((n, n), order="F")
    out.lam_h = np.empty(n); out.lam_l = np.empty(n); out.r = np.empty(n)
    em = np.zeros(1); b = ctypes.c_int(); k = ctypes.c_int(); g = ctypes.c_int(0)
    st = _load().or_method_step_grouped(n, _p(A), _p(X), _p(lam_prev), float(delta), float(xi),
                                        int(kx_max), int(kx_force), _p(out.X1), _p(out.X_hi),
                                        _p(out.X_lo), _p(out.lam_h), _p(out.lam_l), _p(out.r),
                                        _p(em), ctypes.byref(b), ctypes.byref(k), float(tau),
                                        ctypes.byref(g))
    if st != 0:
        raise RuntimeError(f"or_method_step status {st}")
    out.emax, out.beta, out.kx, out.groups = float(em[0]), b.value, k.value, g.value
    return out


def secular_rank1(d_hi, d_lo, rho, u, idx=None):
    """Eigenpairs of diag(d) + rho u u^T (d ascending, double-double).

    idx: optional (lo, hi) column range to compute. Returns (lam_h, lam_l, X_hi, X_lo)."""
    d_hi = np.ascontiguousarray(d_hi, dtype=np.float64)
    d_lo = np.ascontiguousarray(d_lo, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    n = d_hi.size
    lam_h = np.zeros(n); lam_l = np.zeros(n)
    Xh = np.zeros((n, n), order="F"); Xl = np.zeros((n, n), order="F")
    lo, hi = (0, n) if idx is None else idx
    st = _load().or_secular_rank1(n, _p(d_hi), _p(d_lo), float(rho), _p(u), _p(lam_h), _p(lam_l),
                                  _p(Xh), _p(Xl), int(lo), int(hi))
    if st != 0:
        raise RuntimeError(f"or_secular_rank1 status {st}")
    return lam_h, lam_l, Xh, Xl


def exact_diag_rank1(A, rho, u):
    """Recover diag(d) exactly from A = fl(diag) + rho u u^T: d_i = A_ii - rho u_i^2 as a
    double-double (TwoSum), sorted ascending with the matching permutation."""
    n = A.shape[0]
    a = np.diag(A).copy()
    b = -(rho * u) * u
    s = a + b
    z = s - a
    e = (a - (s - z)) + (b - z)
    order = np.lexsort((e, s))
    return s[order], e[order], order


def sign_align(X, Xref):
    """Flip the columns of Xref to match the signs of X column by column."""
    s = np.sign(np.sum(X * Xref, axis=0))
    s[s == 0] = 1.0
    return Xref * s


# ---------------------------------------------------------------- complex Hermitian case
# Complex matrices are complex128 numpy arrays; the C side takes real and imaginary
# parts (oracle_herm.c).

def _parts(Z):
    Z = np.asarray(Z, dtype=np.complex128)
    return _f64(Z.real), _f64(Z.imag)


def _cplx(re, im):
    Z = np.empty(re.shape, dtype=np.complex128, order="F")
    Z.real, Z.imag = re, im
    return Z


def herm_dd_step(A, X_hi, X_lo=None):
    """One iteration of Algorithm 1 for Hermitian A in complex double-double.
    Returns (X_hi, X_lo, lam_h, lam_l, r, emax) with X as complex128 pairs."""
    Ar, Ai = _parts(A)
    n = Ar.shape[0]
    Xrh, Xih = _parts(X_hi)
    Xrh, Xih = Xrh.copy(order="F"), Xih.copy(order="F")
    if X_lo is None:
        Xrl, Xil = np.zeros_like(Xrh, order="F"), np.zeros_like(Xih, order="F")
    else:
        Xrl, Xil = _parts(X_lo)
        Xrl, Xil = Xrl.copy(order="F"), Xil.copy(order="F")
    lh, ll, r, em = np.empty(n), np.empty(n), np.empty(n), np.zeros(1)
    st = _load().or_herm_dd_step(n, _p(Ar), _p(Ai), _p(Xrh), _p(Xrl), _p(Xih), _p(Xil), _p(lh),
                                 _p(ll), _p(r), _p(em))
    if st != 0:
        raise RuntimeError(f"or_herm_dd_step status {st}")
    return _cplx(Xrh, Xih), _cplx(Xrl, Xil), lh, ll, r, float(em[0])


def refine_dd_herm(A, X0, max_iter=12, tol=1e-28):
    """Iterate the complex double-double step from X0 to its fixed point (stops as
    refine_dd does). Returns (X_hi, X_lo, lam_h, history)."""
    Xh, Xl = np.asarray(X0, dtype=np.complex128), None
    hist, lh = [], None
    for _ in range(max_iter):
        Xh, Xl, lh, ll, r, em = herm_dd_step(A, Xh, Xl)
        hist.append(em)
        if em <= tol:
            break
        if len(hist) >= 3 and hist[-1] > 0.1 * hist[-2] and hist[-2] < 1e-10:
            break
    # Rayleigh quotients of the final iterate (one more step's lambda)
    lam = herm_dd_step(A, Xh, Xl)[2]
    return Xh, Xl, lam, hist


def herm_beta_rule(lam, X, delta, xi=0.0, kx_max=9):
    Xr, Xi = _parts(X)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    b = ctypes.c_int(); k = ctypes.c_int()
    st = _load().or_herm_beta_rule(Xr.shape[0], _p(lam), _p(Xr), _p(Xi), float(delta), float(xi),
                                   int(kx_max), ctypes.byref(b), ctypes.byref(k))
    return {"status": st, "beta": b.value, "kx": k.value}


def herm_method_step(A, X, lam_prev, delta, xi=0.0, kx_max=9, kx_force=0):
    """One iteration of the proposed method for Hermitian A with exact (double-double)
    products."""
    Ar, Ai = _parts(A)
    Xr, Xi = _parts(X)
    n = Ar.shape[0]
    lam_prev = np.ascontiguousarray(lam_prev, dtype=np.float64)
    X1r, X1i = np.empty((n, n), order="F"), np.empty((n, n), order="F")
    outs = [np.empty((n, n), order="F") for _ in range(4)]
    lh, ll, r, em = np.empty(n), np.empty(n), np.empty(n), np.zeros(1)
    b = ctypes.c_int(); k = ctypes.c_int()
    st = _load().or_herm_method_step(n, _p(Ar), _p(Ai), _p(Xr), _p(Xi), _p(lam_prev),
                                     float(delta), float(xi), int(kx_max), int(kx_force),
                                     _p(X1r), _p(X1i), *[_p(o) for o in outs], _p(lh), _p(ll),
                                     _p(r), _p(em), ctypes.byref(b), ctypes.byref(k))
    if st != 0:
        raise RuntimeError(f"or_herm_method_step status {st}")
    out = MethodStep()
    out.X1 = _cplx(X1r, X1i)
    out.X_hi, out.X_lo = _cplx(outs[0], outs[2]), _cplx(outs[1], outs[3])
    out.lam_h, out.lam_l, out.r, out.emax = lh, ll, r, float(em[0])
    out.beta, out.kx = b.value, k.value
    return out


def phase_align(X, Xref):
    """Multiply each column of Xref by the unit complex number that best aligns it with
    the same column of X (the phase of xref_j^H x_j)."""
    s = np.sum(np.conj(Xref) * X, axis=0)
    a = np.abs(s)
    ph = np.where(a > 0, s / np.where(a > 0, a, 1.0), 1.0)
    return Xref * ph
