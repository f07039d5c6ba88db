"""Pins of the oracle's grouped correction (Rayleigh-Ritz on strongly coupled columns).

This step extends Algorithm 1 (Sec. 2.4), which assumes well-separated eigenvalues
(Sec. 3.2). The first-order Ogita-Aishima correction stalls on a column pair mixed by
a large angle. When the pair's span holds the two eigenvectors exactly, the
Rayleigh-Ritz problem on that span has a closed-form answer: the eigenvectors
themselves. For a general span the Ritz pairs are those of the projected matrix, which
a library eigensolver gives independently. With grouping off, or with no group formed,
the step is bit-for-bit the plain step.
"""
import numpy as np
import pytest

import oracle
import workloads


def _rotated_identity(n, pairs, theta):
    X = np.eye(n)
    for (a, b), t in zip(pairs, theta):
        c, s = np.cos(t), np.sin(t)
        X[a, a], X[b, a], X[a, b], X[b, b] = c, s, -s, c
    return np.asfortranarray(X)


def _max_err_to_identity(Xh):
    S = np.sign(np.diag(Xh))
    S[S == 0] = 1
    return float(np.max(np.abs(Xh * S - np.eye(Xh.shape[0]))))


@pytest.mark.parametrize("theta", [0.05, 0.3, 0.7])
def test_rotated_tight_pair_resolved_in_one_step(theta):
    """A = diag(d) with d_0, d_1 1e-10 apart; X0 = I with columns 0, 1 rotated by theta.
    span(X0[:, :2]) = span(e_0, e_1) exactly, so one grouped step returns I (up to signs),
    while the plain first-order step leaves an error of order theta^2."""
    n = 12
    d = np.concatenate([[1.0, 1.0 + 1e-10], np.arange(2.0, n)])
    A = np.asfortranarray(np.diag(d))
    X0 = _rotated_identity(n, [(0, 1)], [theta])
    Xh, Xl = X0.copy(order="F"), np.zeros((n, n), order="F")
    st = oracle.refine_dd_step(A, Xh, Xl, tau=1e-3)
    assert st.groups == 1
    assert _max_err_to_identity(Xh) <= 1e-15
    Ph, Pl = X0.copy(order="F"), np.zeros((n, n), order="F")
    oracle.refine_dd_step(A, Ph, Pl)
    assert _max_err_to_identity(Ph) > 0.1 * theta ** 2


def test_chain_forms_one_group():
    """Columns 0-1, 1-2 and 2-3 rotated in turn: the couplings chain the four columns into
    one group, and one grouped step returns I."""
    n = 14
    d = np.concatenate([[1.0, 1.0 + 1e-10, 1.0 + 2e-10, 1.0 + 3e-10], np.arange(3.0, 3.0 + n - 4)])
    A = np.asfortranarray(np.diag(d))
    X0 = np.eye(n)
    for a, t in ((0, 0.3), (1, 0.2), (2, 0.25)):
        R = np.eye(n)
        c, s_ = np.cos(t), np.sin(t)
        R[a, a], R[a + 1, a], R[a, a + 1], R[a + 1, a + 1] = c, s_, -s_, c
        X0 = X0 @ R
    X0 = np.asfortranarray(X0)
    Xh, Xl = X0.copy(order="F"), np.zeros((n, n), order="F")
    st = oracle.refine_dd_step(A, Xh, Xl, tau=1e-3)
    assert st.groups == 1
    assert _max_err_to_identity(Xh) <= 1e-15


def test_two_separate_groups():
    n = 16
    d = np.concatenate([[1.0, 1.0 + 1e-9, 5.0, 5.0 + 2e-9], np.arange(10.0, 10.0 + n - 4)])
    A = np.asfortranarray(np.diag(d))
    X0 = _rotated_identity(n, [(0, 1), (2, 3)], [0.4, 0.2])
    Xh, Xl = X0.copy(order="F"), np.zeros((n, n), order="F")
    st = oracle.refine_dd_step(A, Xh, Xl, tau=1e-3)
    assert st.groups == 2
    assert _max_err_to_identity(Xh) <= 1e-15


def test_three_column_group_matches_library_eigensolver():
    """A dense A; X0 = its eigenvectors (the oracle's fixed point) with columns 3, 4, 5
    mixed by a random orthogonal 3 x 3 matrix R. One grouped step must return those
    columns to eigenvectors: each column gets the one it overlaps most (R's largest
    entries, taken greedily), the other columns stay put, and the new Rayleigh
    quotients equal the eigenvalues of X_C^T A X_C computed by numpy."""
    n = 40
    p = workloads.make_problem(2, n, x0="eigh")
    Xt, Xtl, lh, ll, _ = oracle.refine_dd(p.A, p.X0)
    rng = np.random.default_rng(3)
    R, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    X0 = Xt.copy(order="F")
    X0[:, 3:6] = Xt[:, 3:6] @ R
    Xh, Xl = X0.copy(order="F"), np.zeros((n, n), order="F")
    st = oracle.refine_dd_step(p.A, Xh, Xl, tau=1e-2)
    assert st.groups == 1
    # expected partner of each mixed column: column a of X0 is sum_v R[v, a] x_v
    partner, used_v, used_c = {}, set(), set()
    for _ in range(3):
        best = max(((abs(R[v, a]), a, v) for a in range(3) for v in range(3)
                    if a not in used_c and v not in used_v), key=lambda t: (t[0], -t[1], -t[2]))
        partner[best[1]] = best[2]
        used_c.add(best[1]); used_v.add(best[2])
    Xexp = Xt.copy(order="F")
    for a, v in partner.items():
        Xexp[:, 3 + a] = Xt[:, 3 + v]
    err = float(np.max(np.abs(Xh - oracle.sign_align(Xh, Xexp))))
    assert err <= 1e-14
    P = X0[:, 3:6].T @ p.A @ X0[:, 3:6]
    ritz = np.linalg.eigvalsh(0.5 * (P + P.T))
    st2 = oracle.refine_dd_step(p.A, Xh, Xl)          # Rayleigh quotients of the new columns
    got = np.sort(st2.lam_h[3:6])
    assert np.allclose(got, np.sort(ritz), rtol=0, atol=1e-14 * np.max(np.abs(p.lam)))


@pytest.mark.parametrize("tau", [0.0, 1e300])
def test_no_group_is_the_plain_step(tau):
    n = 30
    p = workloads.make_problem(1, n, x0="eigh")
    Ah = p.A
    X1h, X1l = p.X0.copy(order="F"), np.zeros((n, n), order="F")
    X2h, X2l = p.X0.copy(order="F"), np.zeros((n, n), order="F")
    a = oracle.refine_dd_step(Ah, X1h, X1l)
    b = oracle.refine_dd_step(Ah, X2h, X2l, tau=tau)
    assert b.groups == 0
    assert np.array_equal(X1h, X2h) and np.array_equal(X1l, X2l)
    assert np.array_equal(a.lam_h, b.lam_h) and a.emax == b.emax
