"""The library's host-side planning, on the CPU (no GPU needed):
- beta of Sec. 4.1 and X^(1)'s plane count: the hand-derived cases and the oracle's rule;
- the working column order;
- the Rayleigh-Ritz solve of the grouped correction, against numpy's eigensolver."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads

HERE = os.path.dirname(os.path.abspath(__file__))


def _rb():
    from paper_2602_19090_amd import binding
    return binding


def _colstats(X):
    """e_j = floor(log2 max|x|) + 1 (frexp exponent), c_j = ceil(log2 max|x|), max."""
    mx = np.max(np.abs(X), axis=0)
    e = np.array([math.frexp(v)[1] if v != 0 else 0 for v in mx], dtype=np.int32)
    c = np.array([(math.frexp(v)[1] - 1 if math.frexp(v)[0] == 0.5 else math.frexp(v)[1])
                  if v != 0 else 0 for v in mx], dtype=np.int32)
    return e, c, mx


def test_beta_hand_derived_cases():
    rb = _rb()
    cases = json.load(open(os.path.join(HERE, "golden", "beta_cases.json")))["cases"]
    for cs in cases:
        n = cs["n"]
        X = np.array(cs["X"], dtype=np.float64).reshape(n, n, order="F")
        e, c, mx = _colstats(X)
        # refeig_host_beta takes the target; the rule uses target / delta_safety
        o = rb.default_opts(delta_safety=1.0)
        st, beta, kx = rb.host_beta(cs["lam"], e, c, mx, cs["delta"], o)
        assert st == 0 and (beta, kx) == (cs["beta"], cs["kx"]), (cs["why"], beta, kx)


@pytest.mark.parametrize("cfg,n,target", [(1, 80, 1e-8), (2, 200, 1e-14), (3, 300, 1e-11),
                                          (2, 513, 1e-12)])
def test_beta_matches_oracle(cfg, n, target):
    rb = _rb()
    p = workloads.make_problem(cfg, n, x0="eigh")
    e, c, mx = _colstats(p.X0)
    st, beta, kx = rb.host_beta(p.D0, e, c, mx, target)
    ref = oracle.beta_rule(p.D0, p.X0, target / 8.0)
    assert st == 0 and (beta, kx) == (ref["beta"], ref["kx"])


def test_beta_rejects_coincident_estimates():
    rb = _rb()
    st, _, _ = rb.host_beta([1.0, 1.0, 2.0], [1, 1, 1], [0, 0, 0], [0.5, 0.5, 0.5], 1e-10)
    assert st == rb.REFEIG_E_GAP


def test_working_column_order():
    rb = _rb()
    lam = np.array([0.0, 10.0, 1.0, 1.5, 4.0, 4.5])
    # gaps: 1, 5.5, 0.5, 0.5, 0.5, 0.5 -> widest first; equal gaps by eigenvalue
    st, order = rb.host_column_order(lam)
    assert st == 0
    assert order.tolist() == [1, 0, 2, 3, 4, 5]
    perm = np.random.default_rng(2).permutation(len(lam))
    st, order2 = rb.host_column_order(lam[perm])
    assert [int(perm[k]) for k in order2] == order.tolist()   # order follows the values


@pytest.mark.parametrize("k,seed", [(2, 0), (3, 1), (5, 2), (12, 3), (32, 4)])
def test_group_ritz_against_numpy(k, seed):
    """A group's Gram matrix G (near I, as for nearly orthonormal columns) and T = W + G
    diag(lam): the returned Ritz pairs satisfy T y = mu G y and Y^T G Y = I, their values are
    numpy's generalized eigenvalues, and the assignment and sign rules hold."""
    rb = _rb()
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((k, k)))
    R = Q @ np.diag(np.linspace(1.0, 2.0, k) * 1e-3) @ Q.T     # a strongly coupled group
    lam = 1.0 + np.sort(rng.uniform(0, 1e-3, k))
    G = np.eye(k) + 1e-14 * (lambda B: B + B.T)(rng.standard_normal((k, k)))
    T = np.diag(lam) + R
    W = T - G @ np.diag(lam)
    st, Y, mh, ml = rb.host_group_ritz(G, np.zeros((k, k)), W, lam, np.zeros(k))
    assert st == 0
    Ts = 0.5 * (T + T.T)
    assert np.max(np.abs(Ts @ Y - G @ Y @ np.diag(mh))) <= 1e-13
    assert np.max(np.abs(Y.T @ G @ Y - np.eye(k))) <= 1e-13
    L = np.linalg.cholesky(G)
    Li = np.linalg.inv(L)
    ref = np.linalg.eigvalsh(Li @ Ts @ Li.T)
    assert np.allclose(np.sort(mh), ref, rtol=0, atol=1e-13)
    assert np.all(np.diag(Y) > 0)
    # greedy assignment: each column keeps the vector with the largest remaining entry
    used_r, used_c = set(), set()
    A = np.abs(Y)
    for _ in range(k):
        best = max(((A[r, c_], r, c_) for r in range(k) for c_ in range(k)
                    if r not in used_r and c_ not in used_c), key=lambda t: (t[0], -t[1], -t[2]))
        assert best[1] == best[2]
        used_r.add(best[1]); used_c.add(best[2])


def test_group_ritz_rejects_indefinite_gram():
    rb = _rb()
    G = np.array([[1.0, 2.0], [2.0, 1.0]])
    st, *_ = rb.host_group_ritz(G, np.zeros((2, 2)), np.zeros((2, 2)), [1.0, 1.0], [0.0, 0.0])
    assert st == rb.REFEIG_E_GAP


def test_sparse_rule_beta_matches_oracle():
    """Under the sparse rule (Sec. 4.3) beta takes xi = min(k^2, n)."""
    rb = _rb()
    p = workloads.banded_problem(300, 3)
    e, c, mx = _colstats(p.X0)
    k = 7
    st, beta, kx = rb.host_beta(p.D0, e, c, mx, 1e-12, rb.default_opts(sparse_k=k))
    ref = oracle.beta_rule(p.D0, p.X0, 1e-12 / 8.0, xi=float(min(k * k, 300)))
    dense = oracle.beta_rule(p.D0, p.X0, 1e-12 / 8.0)
    assert st == 0 and (beta, kx) == (ref["beta"], ref["kx"])
    assert ref["beta"] < dense["beta"]
