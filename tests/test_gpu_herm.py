"""GPU parity of the complex Hermitian path (refine_eigvecs_herm) against the Hermitian
oracle: one step against the oracle's method step (same beta, k_X; X within delta), solves
to the target against X_true (the complex double-double fixed point, compared up to a unit
complex factor per column), and checks that need no oracle (equivariance under +-1 / +-i
phases, a real symmetric input against the real path's X_true)."""
import numpy as np
import pytest

import lambda_bounds
import oracle
import workloads

pytestmark = pytest.mark.gpu

_XT = {}


def _rb():
    from paper_2602_19090_amd import binding as rb
    return rb


def _xtrue_herm(p):
    key = p.meta["digest"]
    if key not in _XT:
        Xh, Xl, lam, hist = oracle.refine_dd_herm(p.A, p.X0)
        _XT[key] = (Xh, lam)
    return _XT[key]


def _dev(p, X0=None):
    import torch
    rb = _rb()
    A = rb.colmajor_complex(p.A)
    X = rb.colmajor_complex(p.X0 if X0 is None else X0)
    D = torch.from_numpy(np.array(p.D0, dtype=np.float64)).cuda()
    return A, X, D


def _fwd(X, Xt):
    return float(np.max(np.abs(X - oracle.phase_align(X, Xt))))


@pytest.mark.parametrize("cfg,n,target", [(1, 100, 1e-14), (2, 300, 1e-12), (3, 1100, 1e-14)])
def test_herm_one_step_vs_oracle(cfg, n, target):
    print(f"herm step cfg={cfg} n={n} target={target}", flush=True)
    rb = _rb()
    p = workloads.hermitian_problem(cfg, n)
    A, X, D = _dev(p)
    opts = rb.default_opts(fixed_iters=1)
    st, rep = rb.refine_eigvecs_herm(A, X, D, target, opts)
    assert st == rb.REFEIG_OK, rb.strerror(st)
    ref = oracle.herm_method_step(p.A, p.X0, p.D0, target / opts.delta_safety)
    assert rep.beta[0] == ref.beta and rep.kx[0] == ref.kx
    Xg = rb.from_colmajor(X)
    diff = float(np.max(np.abs(Xg - ref.X_hi)))
    print(f"  beta={ref.beta} kx={ref.kx} dv={rep.dv[0]} dw={rep.dw[0]} du={rep.du[0]} "
          f"|X_gpu - X_oracle|max={diff:.3e}", flush=True)
    assert diff <= target / opts.delta_safety
    lam = D.cpu().numpy()
    tol = lambda_bounds.one_step_tol(ref.X1, ref.lam_h, lambda_bounds.entry_gaps(p.D0),
                                     target / opts.delta_safety,
                                     float(np.max(np.abs(ref.lam_h))), opts.theta, cplx=True)
    ratio = np.abs(lam - ref.lam_h) / tol
    print(f"  eigenvalues: max |err| / bound = {float(np.max(ratio)):.3e}", flush=True)
    assert np.all(ratio <= 1.0)


@pytest.mark.parametrize("cfg,n,target", [(1, 100, 1e-14), (2, 300, 1e-12), (3, 700, 1e-14),
                                          (2, 255, 1e-13), (2, 257, 1e-13)])
def test_herm_refine_to_target(cfg, n, target):
    print(f"herm refine cfg={cfg} n={n} target={target}", flush=True)
    rb = _rb()
    p = workloads.hermitian_problem(cfg, n)
    Xt, lt = _xtrue_herm(p)
    A, X, D = _dev(p)
    st, rep = rb.refine_eigvecs_herm(A, X, D, target)
    r = rep.as_dict()
    err = _fwd(rb.from_colmajor(X), Xt)
    print(f"  status={st} iters={r['iters']} eps={['%.1e' % e for e in r['eps']]} "
          f"fwd={err:.3e}", flush=True)
    assert st == rb.REFEIG_OK, rb.strerror(st)
    assert err <= target
    # eigenvalues within their derived bound (lambda_bounds); the last iteration's input is
    # the solve of one iteration fewer
    K = rep.iters
    _, Xin, Din = _dev(p)
    if K > 1:
        st1, _ = rb.refine_eigvecs_herm(A, Xin, Din, target, rb.default_opts(fixed_iters=K - 1))
        assert st1 == rb.REFEIG_OK
    Xi = rb.from_colmajor(Xin)
    tol = lambda_bounds.solve_tol(Xi, oracle.phase_align(Xi, Xt), rep.kx[K - 1], lt,
                                  lambda_bounds.entry_gaps(Din.cpu().numpy()), target / 8.0,
                                  float(np.max(np.abs(lt))), cplx=True)
    ratio = np.abs(D.cpu().numpy() - lt) / tol
    print(f"  eigenvalues: max |err| / bound = {float(np.max(ratio)):.3e}", flush=True)
    assert np.all(ratio <= 1.0)


def test_herm_loose_target_is_a_stable_fixed_point():
    """Config 3 at n = 1024 (smallest gap about 3e-14 of max|lambda|) at a loose target: the
    solve with the stop rule and one of 8 fixed iterations both stay within the target, so the
    products' own noise does not return amplified by max|lambda| / g_j."""
    print("herm loose target cfg=3 n=1024 target=1e-8", flush=True)
    rb = _rb()
    p = workloads.hermitian_problem(3, 1024)
    Xt, _ = _xtrue_herm(p)
    for fixed in (0, 8):
        A, X, D = _dev(p)
        st, rep = rb.refine_eigvecs_herm(A, X, D, 1e-8, rb.default_opts(fixed_iters=fixed))
        err = _fwd(rb.from_colmajor(X), Xt)
        print(f"  fixed_iters={fixed} status={st} iters={rep.iters} "
              f"eps={['%.1e' % e for e in rep.eps[:rep.iters]]} fwd={err:.3e}", flush=True)
        assert st == rb.REFEIG_OK, rb.strerror(st)
        assert err <= 1e-8


def test_herm_phase_equivariance():
    """A' = P A P^H, X' = P X with phases in {1, i, -1, -i} (exact): every integer product
    is the same up to the exchange of parts, so two iterations give X' = P X to rounding."""
    rb = _rb()
    p = workloads.hermitian_problem(3, 300)
    rng = np.random.default_rng(11)
    P = np.array([1.0, 1j, -1.0, -1j])[rng.integers(0, 4, p.n)]
    A, X, D = _dev(p)
    st, rep = rb.refine_eigvecs_herm(A, X, D, 1e-14, rb.default_opts(fixed_iters=2))
    assert st == rb.REFEIG_OK
    p2 = workloads.Problem("phased", (P[:, None] * p.A) * np.conj(P)[None, :], p.lam, None,
                           P[:, None] * p.X0, p.D0, {})
    A2, X2, D2 = _dev(p2)
    st2, rep2 = rb.refine_eigvecs_herm(A2, X2, D2, 1e-14, rb.default_opts(fixed_iters=2))
    assert st2 == rb.REFEIG_OK
    assert list(rep.kx[:2]) == list(rep2.kx[:2]) and list(rep.dv[:2]) == list(rep2.dv[:2])
    diff = float(np.max(np.abs(rb.from_colmajor(X2) - P[:, None] * rb.from_colmajor(X))))
    print(f"  |X' - P X|max = {diff:.2e}", flush=True)
    assert diff <= 1e-15


def test_herm_real_input_matches_real_solution():
    """A real symmetric matrix given to the Hermitian path: the solve meets the target
    against the real oracle's X_true (the imaginary parts stay zero)."""
    rb = _rb()
    p = workloads.make_problem(2, 300, x0="eigh")
    Xh, Xl, lh, ll, hist = oracle.refine_dd(p.A, p.X0)
    pc = workloads.Problem("real", p.A.astype(np.complex128), p.lam, None,
                           p.X0.astype(np.complex128), p.D0, {})
    A, X, D = _dev(pc)
    st, rep = rb.refine_eigvecs_herm(A, X, D, 1e-14)
    assert st == rb.REFEIG_OK, rb.strerror(st)
    Xg = rb.from_colmajor(X)
    assert float(np.max(np.abs(Xg.imag))) == 0.0
    err = float(np.max(np.abs(Xg.real - oracle.sign_align(Xg.real, Xh))))
    print(f"  iters={rep.iters} fwd={err:.2e}", flush=True)
    assert err <= 1e-14


def test_herm_rejects_unsupported_options():
    rb = _rb()
    p = workloads.hermitian_problem(1, 64)
    A, X, D = _dev(p)
    for kw in (dict(group_tau=1e-3), dict(schedule=1), dict(sparse_k=3), dict(vmode=2)):
        st, _ = rb.refine_eigvecs_herm(A, X, D, 1e-14, rb.default_opts(**kw))
        assert st == rb.REFEIG_E_ARG
