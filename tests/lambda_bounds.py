"""Per-column bounds on the eigenvalue estimates the GPU returns, derived from the
product cutoffs (not a tolerance chosen to pass).

One step (same X^(1) on both sides). The GPU's lambda_j is the Rayleigh quotient
x^T v / (x^T x) of column j of X^(1) with v the truncated product A x. Either form of
V keeps every entry of column j within 1.1 sqrt(n) theta delta g_j in the worst case:
the cutoffs are set so that the statistical estimate (sqrt(n) growth of n terms) is
theta delta g_j, and n terms can add up to sqrt(n) times that; the residue form adds the
reconstruction error, which the solver keeps below theta delta g_j / 4. Then
|x^T dv| / (x^T x) <= ||x||_1 max|dv| / ||x||^2 <= sqrt(n) max|dv| / ||x||, so

    |lambda_gpu - lambda_oracle| <= 1.1 n theta delta g_j / ||x_j|| + 0.25 sqrt(n) theta
                                    delta g_j / ||x_j|| + u |lambda_j| + 2 n 2^-104 max|lambda|

(u |lambda_j|: the FP64 rounding of the double-word value; the last term: double-word
dot products on both sides). g_j is the gap of the iteration's entry estimates.

A solve. lambda is the Rayleigh quotient of the last iteration's X^(1) = y. For
y = x + e with x the unit eigenvector, rho(y) - lambda_true = e^T (A - lambda I) e / y^T y,
so |rho(y) - lambda_true| <= 2 max|lambda| ||e||^2 / (1 - ||e||)^2 (exact), and ||e|| is
at most the error of the last iteration's input plus the X^(1) cut, sqrt(n) 2^(e_j - 7 kx).
"""
import numpy as np

U = 2.0 ** -53


def entry_gaps(lam):
    """Distance from each eigenvalue estimate to its nearest other one."""
    lam = np.asarray(lam, dtype=np.float64)
    n = len(lam)
    if n == 1:
        return np.array([np.inf])
    o = np.argsort(lam, kind="stable")
    s = lam[o]
    d = np.diff(s)
    g = np.empty(n)
    g[0], g[-1] = d[0], d[-1]
    if n > 2:
        g[1:-1] = np.minimum(d[:-1], d[1:])
    out = np.empty(n)
    out[o] = g
    return out


def _coef(n, cplx):
    # real: n terms per entry of V, worst case 1.1 sqrt(n) theta delta g per entry (plus a
    # quarter for the residue form's reconstruction), sqrt(n) more in the quotient; complex
    # (slice products of 2n real terms, both parts): sqrt(2) 1.1 sqrt(2n) per entry
    return 2.2 * n if cplx else 1.1 * n + 0.25 * np.sqrt(n)


def one_step_tol(X1, lam, gaps, delta, lmax, theta=0.25, cplx=False):
    """Per-column bound on |lambda_gpu - lambda_oracle| after one step: X1 the step's X^(1)
    (n x m, columns), lam (m) the oracle's Rayleigh quotients, gaps (m) the gaps of the
    iteration's entry estimates (entry_gaps of all n, at these columns), delta the internal
    delta, lmax = max |lambda|."""
    n = X1.shape[0]
    nx = np.linalg.norm(X1, axis=0)
    g = np.where(np.isfinite(gaps), gaps, 0.0)
    dots = (4.0 if cplx else 2.0) * n * 2.0 ** -104 * lmax
    return _coef(n, cplx) * theta * delta * g / nx + U * np.abs(lam) + dots


def solve_tol(Xin, Xtrue_aligned, kx, lam_true, gaps, delta, lmax, theta=0.25, cplx=False):
    """Per-column bound on |D_j - lambda_true_j| after a solve whose last iteration started
    from Xin (n x m columns) with kx digit planes of X^(1); Xtrue_aligned: the true
    eigenvectors of those columns, aligned to Xin (sign, or unit complex factor); gaps (m):
    the gaps of that iteration's entry estimates; lmax = max |lambda|."""
    n = Xin.shape[0]
    e_in = np.linalg.norm(Xin - Xtrue_aligned, axis=0)
    if cplx:
        mx = np.max(np.maximum(np.abs(Xin.real), np.abs(Xin.imag)), axis=0)
    else:
        mx = np.max(np.abs(Xin), axis=0)
    ex = np.where(mx > 0, np.floor(np.log2(np.where(mx > 0, mx, 1.0))) + 1, 0)
    e = e_in + np.sqrt((2 if cplx else 1) * n) * np.ldexp(1.0, (ex - 7 * kx).astype(int))
    assert np.all(e < 0.5), "the last iteration's input is too far off for this bound"
    rq = 2.0 * lmax * e ** 2 / (1.0 - e) ** 2
    g = np.where(np.isfinite(gaps), gaps, 0.0)
    dots = (4.0 if cplx else 2.0) * n * 2.0 ** -104 * lmax
    step = _coef(n, cplx) * theta * delta * g / (1.0 - e) + U * np.abs(lam_true) + dots
    return rq + step
