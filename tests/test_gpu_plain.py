"""Parity of the FP64 plain form (FP64 Ozaki slices on DGEMM, mode REFEIG_FP64_PLAIN)
with the CPU oracle.

The plain form takes X^(1) as the paper's rounding split, fl((tau_j + x) - tau_j) with
tau_j = 0.75 * 2^(ceil(log2 w_j) + beta) (eq. tau/x, Sec. 3.3); the oracle builds the same
X^(1) with its own FP64 splitting and runs Algorithm 1 on it in double-double.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def _rb():
    from paper_2602_19090_amd import binding
    return binding


def _dev(p):
    import torch
    rb = _rb()
    return rb.colmajor(p.A), rb.colmajor(p.X0), torch.from_numpy(np.array(p.D0)).cuda()


@pytest.mark.parametrize("cfg,n,target", [(1, 100, 1e-12), (2, 300, 1e-14)])
def test_plain_one_step_vs_oracle(cfg, n, target):
    rb = _rb()
    p = workloads.make_problem(cfg, n, x0="eigh")
    A, X, D = _dev(p)
    opts = rb.default_opts(mode=rb.REFEIG_FP64_PLAIN, fixed_iters=1)
    st, rep = rb.refine_eigvecs(A, X, D, target, opts)
    assert st == rb.REFEIG_OK, rb.strerror(st)
    br = oracle.beta_rule(p.D0, p.X0, target / opts.delta_safety)
    assert rep.beta[0] == br["beta"]
    (X1,), _ = oracle.sigma_split(p.X0, br["beta"], 1, by_rows=False)
    Xh = np.asfortranarray(X1.copy()); Xl = np.zeros_like(Xh, order="F")
    step = oracle.refine_dd_step(p.A, Xh, Xl)
    diff = float(np.max(np.abs(rb.from_colmajor(X) - Xh)))
    print(f"plain step n={n}: dv={rep.dv[0]} dgemm={rep.pairs[0]} |X_gpu - X_oracle|={diff:.3e}")
    assert diff <= target / opts.delta_safety
    assert float(np.max(np.abs(D.cpu().numpy() - step.lam_h))) <= 1e-15


@pytest.mark.parametrize("cfg,n,target", [(1, 100, 1e-14), (2, 512, 1e-14), (3, 700, 1e-12)])
def test_plain_refine_to_target(cfg, n, target):
    rb = _rb()
    p = workloads.make_problem(cfg, n, x0="eigh")
    Xt, _, lt, _, _ = oracle.refine_dd(p.A, p.X0)
    A, X, D = _dev(p)
    st, rep = rb.refine_eigvecs(A, X, D, target, rb.default_opts(mode=rb.REFEIG_FP64_PLAIN))
    Xg = rb.from_colmajor(X)
    err = float(np.max(np.abs(Xg - oracle.sign_align(Xg, Xt))))
    print(f"plain n={n}: status {st} iters {rep.iters} eps {list(rep.eps[:rep.iters])} fwd {err:.3e}")
    assert st == rb.REFEIG_OK, rb.strerror(st)
    assert err <= target
