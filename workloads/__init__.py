"""Seeded synthetic inputs for the eigenvector-refinement hot path.

This module only generates inputs. It holds none of the refinement method's
arithmetic and is shared by the oracle tests and the GPU path alike.

The paper's random test matrices (Sec. 4, a geometric spectrum generated with
MATLAB's randsvd) are replaced by A = Q diag(lambda) Q^T where Q is a product
of four Householder reflectors drawn from seeded N(0, 1) vectors, and
lambda_i = 10^(-c (i-1)/(n-1)). The reflector application runs in a small C
library (``gen.c``) with a fixed loop order so the same seed gives the same
bits on every x86-64 host.

All matrices are numpy arrays in Fortran (column-major) order, the layout the
C ABI of the GPU library uses: eigenvector j is the contiguous column j.
"""
from __future__ import annotations

import ctypes
import hashlib
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libworkloads.so")
_lib = None

SEED_BASE = (2602, 19090)


def build(force: bool = True) -> str:
    """Compile gen.c into libworkloads.so (in-tree)."""
    src = os.path.join(_HERE, "gen.c")
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-o", tmp, src])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER(ctypes.c_double)
        lib.wl_householder_sym.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P]
        lib.wl_householder_q.argtypes = [ctypes.c_int, ctypes.c_int, P, P]
        lib.wl_diag_rank1.argtypes = [ctypes.c_int, P, ctypes.c_double, P, P]
        lib.wl_householder_herm.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def rng_for(config_id: int, index: int = 0) -> np.random.Generator:
    return np.random.default_rng([SEED_BASE[0], SEED_BASE[1], config_id, index])


def geometric_spectrum(n: int, c: float) -> np.ndarray:
    """lambda_i = 10^(-c (i-1)/(n-1)), i = 1..n, descending from 1 to 10^-c.

    Evaluated per element with the C library's pow so the bits do not depend
    on numpy's SIMD dispatch."""
    if n == 1:
        return np.ones(1)
    return np.array([math.pow(10.0, -c * i / (n - 1)) for i in range(n)], dtype=np.float64)


def householder_vectors(rng: np.random.Generator, n: int, m: int = 4) -> np.ndarray:
    return np.asfortranarray(rng.standard_normal((n, m)))


def householder_matrix(lam: np.ndarray, V: np.ndarray) -> np.ndarray:
    n, m = V.shape
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    V = np.asfortranarray(V, dtype=np.float64)
    A = np.empty((n, n), dtype=np.float64, order="F")
    if _load().wl_householder_sym(n, m, _ptr(V), _ptr(lam), _ptr(A)) != 0:
        raise RuntimeError("wl_householder_sym failed")
    return A


def householder_q(V: np.ndarray) -> np.ndarray:
    n, m = V.shape
    V = np.asfortranarray(V, dtype=np.float64)
    Q = np.empty((n, n), dtype=np.float64, order="F")
    if _load().wl_householder_q(n, m, _ptr(V), _ptr(Q)) != 0:
        raise RuntimeError("wl_householder_q failed")
    return Q


def matrix_digest(A: np.ndarray) -> str:
    return hashlib.sha256(np.asfortranarray(A).tobytes(order="F")).hexdigest()


class Problem:
    """A symmetric test matrix with its construction and a starting point."""

    def __init__(self, name, A, lam, Q, X0, D0, meta):
        self.name, self.A, self.lam, self.Q, self.X0, self.D0, self.meta = name, A, lam, Q, X0, D0, meta

    @property
    def n(self):
        return self.A.shape[0]


def spectrum_for_config(config_id: int, n: int, rng: np.random.Generator, cond_exp: float | None = None):
    """Eigenvalues for the five workload families.

    1: geometric 1 -> 1e-8 (SPD).
    2: geometric 1 -> 1e-12, then n/2 indices (seeded) flipped in sign.
    3: geometric 1 -> 1e-12 with 16 clustered pairs: at the index nearest
       10^(-4 (m + 1/2)/16), m = 0..15, the next eigenvalue is set to
       lambda_p (1 - 1e-9).
    4, 5: geometric with exponent cond_exp (given by the caller)."""
    if config_id == 1:
        return geometric_spectrum(n, 8.0)
    if config_id == 2:
        lam = geometric_spectrum(n, 12.0)
        idx = rng.choice(n, size=n // 2, replace=False)
        lam[idx] = -lam[idx]
        return lam
    if config_id == 3:
        lam = geometric_spectrum(n, 12.0)
        logs = np.array([-12.0 * i / (n - 1) for i in range(n)])
        for m in range(16):
            target = -4.0 * (m + 0.5) / 16.0
            p = int(np.argmin(np.abs(logs - target)))
            if p + 1 < n:
                lam[p + 1] = lam[p] * (1.0 - 1e-9)
        return lam
    if cond_exp is None:
        raise ValueError("cond_exp required for configs 4/5")
    return geometric_spectrum(n, float(cond_exp))


def banded_problem(n: int, bw: int, index: int = 0, x0: str = "eigh") -> Problem:
    """A sparse stand-in (Sec. 4.3 measures sparse matrices from ELSES and SuiteSparse, which
    are not available): a symmetric band matrix of half-bandwidth bw (at most 2 bw + 1
    nonzeros per row) with N(0, 1) entries plus a diagonal ramp 0..n-1, seeded by
    (2602, 19090, 6, index). Start from an FP64 eigensolve (ascending)."""
    rng = np.random.default_rng([SEED_BASE[0], SEED_BASE[1], 6, index])
    A = np.zeros((n, n))
    for d in range(1, bw + 1):
        v = rng.standard_normal(n - d)
        A[np.arange(n - d), np.arange(d, n)] = v
    A = A + A.T
    A[np.arange(n), np.arange(n)] = rng.standard_normal(n) + np.arange(n, dtype=np.float64)
    A = np.asfortranarray(A)
    X0 = D0 = None
    if x0 == "eigh":
        w, X = np.linalg.eigh(A)
        X0, D0 = np.asfortranarray(X), w.copy()
    meta = {"config": 6, "n": n, "index": index, "bw": bw, "digest": matrix_digest(A)}
    return Problem(f"band{bw}_n{n}_i{index}", A, None, None, X0, D0, meta)


def config4_sizes(count: int, batch: int = 0):
    """Orders and condition exponents of the many-small-matrices workload (config 4):
    n = round(exp(U(ln 32, ln 1024))), cond = 10^c with c ~ U(4, 12), seeded per batch.
    Matrix i of the batch is make_problem(4, n[i], index=i, cond_exp=c[i])."""
    rng = rng_for(4, 1_000_000 + batch)
    ns = np.rint(np.exp(rng.uniform(np.log(32.0), np.log(1024.0), count))).astype(int)
    cs = rng.uniform(4.0, 12.0, count)
    return ns, cs


def make_problem(config_id: int, n: int, index: int = 0, x0: str = "eigh",
                 cond_exp: float | None = None) -> Problem:
    """Build (A, X0, D0) for a workload family.

    x0: "eigh" (FP64 LAPACK eigensolve, the paper's start), "q" (the
    construction's Q rounded to FP64, columns in descending-lambda order),
    "jacobi32" (FP32 cyclic Jacobi), or "none"."""
    rng = rng_for(config_id, index)
    V = householder_vectors(rng, n, 4)
    lam = spectrum_for_config(config_id, n, rng, cond_exp)
    A = householder_matrix(lam, V)
    Q = None
    X0 = D0 = None
    if x0 == "eigh":
        w, X = np.linalg.eigh(A)
        X0, D0 = np.asfortranarray(X), w.copy()
    elif x0 == "q":
        Q = householder_q(V)
        order = np.argsort(lam, kind="stable")
        X0, D0 = np.asfortranarray(Q[:, order]), lam[order].copy()
    elif x0 == "jacobi32":
        w, X = jacobi_eig_fp32(A)
        X0, D0 = np.asfortranarray(X.astype(np.float64)), w.astype(np.float64)
    elif x0 != "none":
        raise ValueError(x0)
    meta = {"config": config_id, "n": n, "index": index, "x0": x0, "digest": matrix_digest(A)}
    return Problem(f"cfg{config_id}_n{n}_i{index}", A, lam, Q, X0, D0, meta)


def hermitian_matrix(lam: np.ndarray, Vr: np.ndarray, Vi: np.ndarray) -> np.ndarray:
    """A = Q diag(lam) Q^H with Q the product of the complex reflectors Vr + i Vi (columns);
    exactly Hermitian, complex128, column-major."""
    n, m = Vr.shape
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    Vr = np.asfortranarray(Vr, dtype=np.float64)
    Vi = np.asfortranarray(Vi, dtype=np.float64)
    Ar = np.empty((n, n), dtype=np.float64, order="F")
    Ai = np.empty((n, n), dtype=np.float64, order="F")
    if _load().wl_householder_herm(n, m, _ptr(Vr), _ptr(Vi), _ptr(lam), _ptr(Ar), _ptr(Ai)) != 0:
        raise RuntimeError("wl_householder_herm failed")
    A = np.empty((n, n), dtype=np.complex128, order="F")
    A.real, A.imag = Ar, Ai
    return A


def hermitian_problem(config_id: int, n: int, index: int = 0, x0: str = "eigh") -> Problem:
    """Complex Hermitian counterpart of make_problem: the spectrum of config 1, 2 or 3 and
    four complex Householder reflectors with seeded N(0, 1) real and imaginary parts.
    x0: "eigh" (LAPACK's complex Hermitian eigensolver in FP64) or "none"."""
    rng = np.random.default_rng([SEED_BASE[0], SEED_BASE[1], 1000 + config_id, index])
    Vr = np.asfortranarray(rng.standard_normal((n, 4)))
    Vi = np.asfortranarray(rng.standard_normal((n, 4)))
    lam = spectrum_for_config(config_id, n, rng)
    A = hermitian_matrix(lam, Vr, Vi)
    X0 = D0 = None
    if x0 == "eigh":
        w, X = np.linalg.eigh(A)
        X0, D0 = np.asfortranarray(X), w.copy()
    elif x0 != "none":
        raise ValueError(x0)
    meta = {"config": config_id, "n": n, "index": index, "x0": x0, "hermitian": True,
            "digest": matrix_digest(A)}
    return Problem(f"herm_cfg{config_id}_n{n}_i{index}", A, lam, None, X0, D0, meta)


def jacobi_eig_fp32(A: np.ndarray, tol: float = 1e-7, max_sweeps: int = 60):
    """Cyclic Jacobi eigensolver in FP32 arithmetic (a low-precision start).

    Sweeps until off(A) <= tol * ||A||_F. Returns eigenvalues ascending and the
    matching eigenvectors (FP32)."""
    M = np.array(A, dtype=np.float32)
    n = M.shape[0]
    X = np.eye(n, dtype=np.float32)
    fro = float(np.linalg.norm(M.astype(np.float64)))
    for _ in range(max_sweeps):
        off = float(np.sqrt(np.sum(np.triu(M.astype(np.float64), 1) ** 2) * 2.0))
        if off <= tol * fro:
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                apq = M[p, q]
                if apq == 0:
                    continue
                app, aqq = M[p, p], M[q, q]
                theta = np.float32(aqq - app) / np.float32(2.0 * apq)
                sgn = np.float32(1.0) if theta >= 0 else np.float32(-1.0)
                at = np.float32(abs(theta))
                if at > np.float32(1e15):          # t = 1/(2 theta) to working precision
                    t = sgn / (np.float32(2.0) * at)
                else:
                    t = sgn / (at + np.sqrt(at * at + np.float32(1.0)))
                c = np.float32(1.0) / np.sqrt(np.float32(t * t + np.float32(1.0)))
                s = np.float32(t * c)
                Mp, Mq = M[:, p].copy(), M[:, q].copy()
                M[:, p] = c * Mp - s * Mq
                M[:, q] = s * Mp + c * Mq
                Mp, Mq = M[p, :].copy(), M[q, :].copy()
                M[p, :] = c * Mp - s * Mq
                M[q, :] = s * Mp + c * Mq
                Xp, Xq = X[:, p].copy(), X[:, q].copy()
                X[:, p] = c * Xp - s * Xq
                X[:, q] = s * Xp + c * Xq
    w = np.diag(M).copy()
    order = np.argsort(w, kind="stable")
    return w[order], X[:, order]


def diag_rank1_problem(n: int, seed: int = 0, c: float = 6.0, rho: float = 0.375):
    """A = diag(d) + rho u u^T stored exactly in FP64.

    u_i are integers in [-15, 15] \\ {0} scaled by 1/16 (4 significant bits) and
    rho has 2 significant bits, so every off-diagonal entry rho u_i u_j is
    exact. The diagonal is rounded once; the caller recovers the exact diagonal
    part as A_ii - rho u_i^2. Returns (A, d_nominal, rho, u)."""
    rng = np.random.default_rng([SEED_BASE[0], SEED_BASE[1], 99, seed])
    d = geometric_spectrum(n, c)
    k = rng.integers(1, 16, size=n) * rng.choice([-1, 1], size=n)
    u = k.astype(np.float64) / 16.0
    A = np.empty((n, n), dtype=np.float64, order="F")
    d_c = np.ascontiguousarray(d)
    u_c = np.ascontiguousarray(u)
    if _load().wl_diag_rank1(n, _ptr(d_c), float(rho), _ptr(u_c), _ptr(A)) != 0:
        raise RuntimeError("wl_diag_rank1 failed")
    return A, d, rho, u
