"""Parity of the GPU refinement (C ABI refine_eigvecs) with the CPU oracle.

* One iteration against the oracle's step of the proposed method (Sec. 3, exact
  products): beta and kx equal, X within the truncation budget.
* Full solves against X_true (the double-double fixed point of Algorithm 1):
  max-abs forward error <= the target, on the workload families, ragged and
  tiny sizes.
* Error paths and run-to-run determinism.
"""
import numpy as np
import pytest

import lambda_bounds
import oracle
import workloads

pytestmark = pytest.mark.gpu


def _rb():
    from paper_2602_19090_amd import binding
    return binding


def _to_dev(p):
    import torch
    rb = _rb()
    return rb.colmajor(p.A), rb.colmajor(p.X0), torch.from_numpy(np.array(p.D0)).cuda()


_XTRUE = {}


def _xtrue(p):
    key = (p.meta["digest"], p.n)
    if key not in _XTRUE:
        Xh, Xl, lh, ll, hist = oracle.refine_dd(p.A, p.X0)
        _XTRUE[key] = (Xh, lh)
    return _XTRUE[key]


def _fwd(Xg, Xt):
    return float(np.max(np.abs(Xg - oracle.sign_align(Xg, Xt))))


@pytest.mark.parametrize("cfg,n,target", [(1, 100, 1e-10), (1, 100, 1e-14), (2, 256, 1e-12),
                                          (2, 300, 1e-14), (3, 1100, 1e-14)])
def test_one_step_vs_oracle(cfg, n, target):
    _one_step_vs_oracle(cfg, n, target, 0)


@pytest.mark.parametrize("cfg,n,target", [(2, 300, 1e-14), (1, 600, 1e-8)])
def test_one_step_full_x_planes_vs_oracle(cfg, n, target):
    """kx_force = 9: X-hat kept at full precision (no X^(1) cut), against the oracle's step
    with the same plane count."""
    _one_step_vs_oracle(cfg, n, target, 9)


def _one_step_vs_oracle(cfg, n, target, kx_force):
    print(f"step cfg={cfg} n={n} target={target} kx_force={kx_force}", flush=True)
    rb = _rb()
    p = workloads.make_problem(cfg, n, x0="eigh")
    A, X, D = _to_dev(p)
    opts = rb.default_opts(fixed_iters=1, kx_force=kx_force)
    st, rep = rb.refine_eigvecs(A, X, D, target, opts)
    assert st == rb.REFEIG_OK, rb.strerror(st)
    ref = oracle.method_step(p.A, p.X0, p.D0, target / opts.delta_safety, kx_force=kx_force)
    assert rep.beta[0] == ref.beta and rep.kx[0] == ref.kx
    Xg = rb.from_colmajor(X)
    diff = float(np.max(np.abs(Xg - ref.X_hi)))
    print(f"  beta={ref.beta} kx={ref.kx} dv={rep.dv[0]} dw={rep.dw[0]} du={rep.du[0]} "
          f"|X_gpu - X_oracle|max={diff:.3e}", flush=True)
    assert diff <= target / opts.delta_safety
    _check_step_lambdas(D, ref, p.D0, target / opts.delta_safety, opts.theta)


def _check_step_lambdas(D, ref, D0, delta, theta):
    """Every eigenvalue estimate within its derived one-step bound (lambda_bounds)."""
    lam = D.cpu().numpy()
    tol = lambda_bounds.one_step_tol(ref.X1, ref.lam_h, lambda_bounds.entry_gaps(D0), delta,
                                     float(np.max(np.abs(ref.lam_h))), theta)
    ratio = np.abs(lam - ref.lam_h) / tol
    print(f"  eigenvalues: max |err| / bound = {float(np.max(ratio)):.3e}", flush=True)
    assert np.all(ratio <= 1.0)


def _check_solve_lambdas(rb, p, target, opts, rep, D, Xt, lt, cols=None):
    """Every eigenvalue estimate (or those of the columns `cols`) within its derived bound
    after a solve of rep.iters iterations: the last iteration's input comes from a solve of
    one iteration fewer with the same options (the arithmetic is the same)."""
    import torch
    K = rep.iters
    A, Xin, Din = _to_dev(p)
    if K > 1:
        o = rb.default_opts() if opts is None else type(opts).from_buffer_copy(opts)
        o.fixed_iters = K - 1
        st, _ = rb.refine_eigvecs(A, Xin, Din, target, o)
        assert st in (rb.REFEIG_OK, rb.REFEIG_NOT_CONVERGED)
    Xi = rb.from_colmajor(Xin)
    gaps = lambda_bounds.entry_gaps(Din.cpu().numpy())
    lam = D.cpu().numpy()
    if cols is not None:
        Xi, gaps, lam = Xi[:, cols], gaps[cols], lam[cols]
    theta = opts.theta if opts is not None else 0.25
    ds = opts.delta_safety if opts is not None else 8.0
    tol = lambda_bounds.solve_tol(Xi, oracle.sign_align(Xi, Xt), rep.kx[K - 1], lt, gaps,
                                  target / ds, float(np.max(np.abs(lt))), theta)
    ratio = np.abs(lam - lt) / tol
    print(f"  eigenvalues: max |err| / bound = {float(np.max(ratio)):.3e}", flush=True)
    assert np.all(ratio <= 1.0)
    del A, Xin, Din
    torch.cuda.empty_cache()


@pytest.mark.parametrize("cfg,n,x0,target", [
    (1, 100, "eigh", 1e-14), (1, 100, "eigh", 1e-8),
    (2, 512, "eigh", 1e-14), (2, 512, "eigh", 1e-11), (2, 300, "eigh", 1e-14),
    (3, 700, "eigh", 1e-14), (1, 257, "q", 1e-12)])
def test_refine_to_target(cfg, n, x0, target):
    print(f"refine cfg={cfg} n={n} x0={x0} target={target}", flush=True)
    rb = _rb()
    p = workloads.make_problem(cfg, n, x0=x0)
    Xt, lt = _xtrue(p)
    A, X, D = _to_dev(p)
    st, rep = rb.refine_eigvecs(A, X, D, target)
    r = rep.as_dict()
    err = _fwd(rb.from_colmajor(X), Xt)
    print(f"  status={st} iters={r['iters']} eps={['%.1e' % e for e in r['eps']]} "
          f"pairs={r['pairs']} fwd={err:.3e}", flush=True)
    assert st == rb.REFEIG_OK, rb.strerror(st)
    assert err <= target
    _check_solve_lambdas(rb, p, target, None, rep, D, Xt, lt)


def test_fp32_jacobi_start():
    """An FP32 cyclic-Jacobi start converges where FP32 resolves every eigenvalue gap
    (cond 1e4). At cond 1e8 it cannot (column errors up to 0.65, outside the assumption
    eps < 1/100 of Sec. 3.2): the solver must then report NOT_CONVERGED, never OK."""
    import torch
    rb = _rb()
    p = workloads.make_problem(4, 100, x0="jacobi32", cond_exp=4.0)
    Xt, _ = _xtrue(workloads.make_problem(4, 100, x0="eigh", cond_exp=4.0))
    A, X, D = _to_dev(p)
    st, rep = rb.refine_eigvecs(A, X, D, 1e-14)
    assert st == rb.REFEIG_OK, rb.strerror(st)
    assert _fwd(rb.from_colmajor(X), Xt) <= 1e-14
    p = workloads.make_problem(1, 100, x0="jacobi32")
    A, X, D = _to_dev(p)
    st, rep = rb.refine_eigvecs(A, X, D, 1e-14)
    assert st == rb.REFEIG_NOT_CONVERGED
    assert bool(torch.isfinite(X).all())


@pytest.mark.parametrize("n", [1, 2, 3, 17])
def test_tiny_sizes(n):
    rb = _rb()
    if n == 1:
        A = np.asfortranarray([[2.5]]); X0 = np.asfortranarray([[1.0]]); D0 = np.array([2.5])
        Xt = X0
    else:
        p = workloads.make_problem(2, n, x0="eigh")
        A, X0, D0 = p.A, p.X0, p.D0
        Xt, _ = _xtrue(p)
    import torch
    Ad, Xd, Dd = rb.colmajor(A), rb.colmajor(X0), torch.from_numpy(np.array(D0)).cuda()
    st, rep = rb.refine_eigvecs(Ad, Xd, Dd, 1e-14)
    assert st == rb.REFEIG_OK, rb.strerror(st)
    assert _fwd(rb.from_colmajor(Xd), Xt) <= 1e-14


def test_diagonal_matrix_stays_identity():
    import torch
    rb = _rb()
    n = 64
    A = np.asfortranarray(np.diag(np.geomspace(1.0, 1e-6, n)))
    Ad, Xd = rb.colmajor(A), rb.colmajor(np.eye(n))
    Dd = torch.from_numpy(np.diag(A).copy()).cuda()
    st, rep = rb.refine_eigvecs(Ad, Xd, Dd, 1e-14)
    assert st == rb.REFEIG_OK
    assert np.array_equal(rb.from_colmajor(Xd), np.eye(n))
    assert rep.eps[0] == 0.0


def test_error_paths():
    import torch
    rb = _rb()
    p = workloads.make_problem(2, 64, x0="eigh")
    A, X, D = _to_dev(p)
    Ab = A.clone(); Ab[3, 5] = float("nan")
    st, _ = rb.refine_eigvecs(Ab, X.clone(), D.clone(), 1e-12)
    assert st == rb.REFEIG_E_NONFINITE
    Dt = D.clone(); Dt[7] = Dt[8]
    X2 = X.clone()
    st, _ = rb.refine_eigvecs(A, X2, Dt, 1e-12)
    assert st == rb.REFEIG_E_GAP
    assert torch.equal(X2, X)                      # untouched on a negative status
    st, _ = rb.refine_eigvecs(A, X.clone(), D.clone(), -1.0)
    assert st == rb.REFEIG_E_ARG
    work = torch.empty(1024, dtype=torch.uint8, device="cuda")
    st, _ = rb.refine_eigvecs(A, X.clone(), D.clone(), 1e-12, work=work)
    assert st == rb.REFEIG_E_NOMEM
    with pytest.raises(ValueError):
        rb.workspace_bytes(8193)


def test_caller_workspace_and_determinism():
    import torch
    rb = _rb()
    p = workloads.make_problem(2, 384, x0="eigh")
    outs = []
    work = torch.empty(rb.workspace_bytes(384), dtype=torch.uint8, device="cuda")
    for w in (None, work):
        A, X, D = _to_dev(p)
        st, rep = rb.refine_eigvecs(A, X, D, 1e-13, work=w)
        assert st == rb.REFEIG_OK
        outs.append((X.cpu().numpy(), D.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_column_order_of_the_input_does_not_matter():
    """The library works on the columns in an order of its own (by gap), and every column's
    arithmetic is independent of where it sits, so permuting the input columns permutes the
    output bit for bit (n = 700 spans three 256-column blocks and a ragged tail)."""
    import torch
    rb = _rb()
    n = 700
    p = workloads.make_problem(2, n, x0="eigh")
    perm = np.random.default_rng(7).permutation(n)
    A, X, D = _to_dev(p)
    st, _ = rb.refine_eigvecs(A, X, D, 1e-13)
    assert st == rb.REFEIG_OK
    Xp = rb.colmajor(np.asfortranarray(p.X0[:, perm]))
    Dp = torch.from_numpy(np.array(p.D0)[perm].copy()).cuda()
    st, _ = rb.refine_eigvecs(A, Xp, Dp, 1e-13)
    assert st == rb.REFEIG_OK
    X0n, Xpn = rb.from_colmajor(X), rb.from_colmajor(Xp)
    assert np.array_equal(Xpn, X0n[:, perm])
    assert np.array_equal(Dp.cpu().numpy(), D.cpu().numpy()[perm])


def _golden(cfg, n):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", f"xtrue_cfg{cfg}_n{n}.npz")
    return np.load(path, allow_pickle=False)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("cfg,n,target", [(2, 4096, 1e-14), (3, 8192, 1e-14), (3, 8192, 1e-11),
                                          (3, 8192, 1e-8)])
def test_full_size_against_oracle_columns(cfg, n, target):
    """Full-size solves (the benchmark's workload at n = 8192, and its precision sweep) from an
    FP64 eigensolve start, checked on the sampled columns of the oracle's X_true
    (tests/golden/make_xtrue.py) and on every eigenvalue."""
    import torch
    rb = _rb()
    print(f"full size cfg={cfg} n={n} target={target}", flush=True)
    g = _golden(cfg, n)
    p = workloads.make_problem(cfg, n, x0="none")
    assert p.meta["digest"] == str(g["digest"]), "generator output differs from the stored matrix"
    A = rb.colmajor(p.A)
    w, V = torch.linalg.eigh(A)
    X0 = V.t().contiguous()
    D0 = w.contiguous()
    del V
    X, D = X0.clone(), D0.clone()
    st, rep = rb.refine_eigvecs(A, X, D, target)
    assert st == rb.REFEIG_OK, rb.strerror(st)
    cols = torch.from_numpy(g["cols"]).cuda()
    Xs = X[cols].cpu().numpy().T
    Xt = g["X_hi"]
    s = np.sign(np.sum(Xs * Xt, axis=0))
    err = float(np.max(np.abs(Xs - Xt * s)))
    print(f"  status {st} iters {rep.iters} eps {list(rep.eps[:rep.iters])} sampled fwd err {err:.3e}",
          flush=True)
    assert err <= target
    # eigenvalues of the sampled columns within their derived bound (lambda_bounds): the
    # last iteration's input is the solve of one iteration fewer
    K = rep.iters
    Xin, Din = X0.clone(), D0.clone()
    if K > 1:
        st1, _ = rb.refine_eigvecs(A, Xin, Din, target, rb.default_opts(fixed_iters=K - 1))
        assert st1 == rb.REFEIG_OK
    c = g["cols"]
    gaps = lambda_bounds.entry_gaps(Din.cpu().numpy())[c]
    lt = g["lam_hi"][c]
    Xi = Xin[cols].cpu().numpy().T
    tol = lambda_bounds.solve_tol(Xi, oracle.sign_align(Xi, Xt), rep.kx[K - 1], lt, gaps,
                                  target / 8.0, float(np.max(np.abs(g["lam_hi"]))))
    ratio = np.abs(D.cpu().numpy()[c] - lt) / tol
    print(f"  eigenvalues (sampled columns): max |err| / bound = {float(np.max(ratio)):.3e}",
          flush=True)
    assert np.all(ratio <= 1.0)
    if cfg == 3 and target == 1e-14:
        # the sampled columns' error against the double-double X_true (high and low words)
        err_cols = np.abs((Xs - Xt * s) - g["X_lo"] * s).max(axis=0)
        _all_columns_check(p, X, g, target, err_cols)
    del A, X, D, X0, D0, Xin, Din
    torch.cuda.empty_cache()


def _all_columns_check(p, X, g, target, err_cols):
    """Every column of the solve's X, not only the sampled ones: one double-double step of
    Algorithm 1 from X on the host (oracle/dd_numpy.py) estimates each column's forward
    error to second order; estimate plus the second-order term must be within the target.
    On the sampled columns the estimate must match the error against X_true."""
    from oracle import dd_numpy as dn
    rb = _rb()
    Xh = np.asfortranarray(rb.from_colmajor(X))
    res = dn.allcols_forward_error(p.A, Xh, g["lam_hi"])
    est, second = res["est"], res["second"]
    c = g["cols"]
    print(f"  all {Xh.shape[1]} columns: max estimated forward error {float(est.max()):.3e}, "
          f"second-order term <= {float(second.max()):.1e} ({res['seconds']:.0f} s on the host); "
          f"sampled columns: max |estimate - error| {float(np.max(np.abs(est[c] - err_cols))):.1e}",
          flush=True)
    assert np.all(np.abs(est[c] - err_cols) <= 0.02 * err_cols + 1e-17)
    assert float(np.max(est + second)) <= target


def test_batched_matches_single_calls_config4():
    """Config-4 style batch (n log-uniform in [32, 1024], cond 10^U(4,12), FP64-eigh start,
    exactly 3 iterations): the batched entry point gives each problem bit for bit what a
    single call gives, and the small members meet the target against the oracle's X_true."""
    import torch
    rb = _rb()
    ns, cs = workloads.config4_sizes(20)
    probs = [workloads.make_problem(4, int(n), index=i, cond_exp=float(c))
             for i, (n, c) in enumerate(zip(ns, cs))]
    print("batch n:", [p.n for p in probs], flush=True)
    opts = rb.default_opts(fixed_iters=3)
    target = 1e-14
    singles = []
    for p in probs:
        A, X, D = _to_dev(p)
        st, _ = rb.refine_eigvecs(A, X, D, target, opts)
        assert st == rb.REFEIG_OK, (p.n, rb.strerror(st))
        singles.append((X.cpu().numpy(), D.cpu().numpy()))
    dev = [_to_dev(p) for p in probs]
    st, reps = rb.refine_eigvecs_batched([d[0] for d in dev], [d[1] for d in dev],
                                         [d[2] for d in dev], [target] * len(probs), opts)
    assert st == rb.REFEIG_OK, rb.strerror(st)
    torch.cuda.synchronize()
    for (A, X, D), (Xs, Ds), r in zip(dev, singles, reps):
        assert r.status == rb.REFEIG_OK and r.iters == 3
        assert np.array_equal(X.cpu().numpy(), Xs) and np.array_equal(D.cpu().numpy(), Ds)
    errs = []
    for p, (A, X, D) in zip(probs, dev):
        if p.n <= 160:
            Xt, _ = _xtrue(p)
            errs.append((p.n, _fwd(rb.from_colmajor(X), Xt)))
    print("3-iteration errors (n, err):", errs, flush=True)
    assert errs and all(e <= target for _, e in errs)


def test_batched_error_paths():
    import torch
    rb = _rb()
    p = workloads.make_problem(1, 64)
    A, X, D = _to_dev(p)
    Xbad = X.clone()
    Xbad[0, 0] = float("nan")
    st, reps = rb.refine_eigvecs_batched([A, A], [X, Xbad], [D, D.clone()], [1e-13, 1e-13])
    assert st == rb.REFEIG_E_NONFINITE
    assert reps[0].status == rb.REFEIG_OK and reps[1].status == rb.REFEIG_E_NONFINITE
    with pytest.raises(ValueError):
        rb.batched_workspace_bytes([64, 0])


def _mixed_start(p, pairs, angles):
    """The FP64 eigensolve's start with some neighbouring column pairs rotated in their
    plane: strongly mixed eigenvector pairs, as a badly resolved start has."""
    X0 = p.X0.copy(order="F")
    for (a, b), t in zip(pairs, angles):
        c, s = np.cos(t), np.sin(t)
        xa, xb = X0[:, a].copy(), X0[:, b].copy()
        X0[:, a], X0[:, b] = c * xa + s * xb, -s * xa + c * xb
    return X0


@pytest.mark.parametrize("cfg,n", [(2, 300), (2, 1100), (3, 1100)])
def test_grouped_step_vs_oracle(cfg, n):
    """One step with the grouped correction (group_tau = 1e-3) against the oracle's grouped
    method step on a start with three badly mixed column pairs; spans npad < 1024 and the
    256 x 256 kernel."""
    import torch
    rb = _rb()
    target, tau = 1e-14, 1e-3
    p = workloads.make_problem(cfg, n, x0="eigh")
    pairs = [(5, 6), (n // 2, n // 2 + 1), (n - 3, n - 2)]
    X0 = _mixed_start(p, pairs, [0.3, 0.2, 0.1])
    A = rb.colmajor(p.A)
    X = rb.colmajor(X0)
    D = torch.from_numpy(np.array(p.D0)).cuda()
    opts = rb.default_opts(fixed_iters=1, group_tau=tau)
    st, rep = rb.refine_eigvecs(A, X, D, target, opts)
    assert st == rb.REFEIG_OK, rb.strerror(st)
    ref = oracle.method_step(p.A, X0, p.D0, target / opts.delta_safety, tau=tau)
    print(f"  groups gpu={rep.groups[0]} oracle={ref.groups} beta={ref.beta} kx={ref.kx}",
          flush=True)
    assert rep.groups[0] == ref.groups >= 3   # the three mixed pairs, plus any the start has
    Xg = rb.from_colmajor(X)
    diff = float(np.max(np.abs(Xg - ref.X_hi)))
    print(f"  |X_gpu - X_oracle|max={diff:.3e}", flush=True)
    assert diff <= target / opts.delta_safety


def test_grouped_solve_from_mixed_start():
    """Full solves from a start with badly mixed pairs: with grouping the target is met
    against X_true in a few iterations; the paper's first-order step needs more."""
    import torch
    rb = _rb()
    target = 1e-14
    p = workloads.make_problem(3, 700, x0="eigh")
    Xt, lt = _xtrue(p)
    X0 = _mixed_start(p, [(10, 11), (300, 301), (650, 651)], [0.35, 0.25, 0.15])
    res = {}
    for tau in (0.0, 1e-3):
        A, X = rb.colmajor(p.A), rb.colmajor(X0)
        D = torch.from_numpy(np.array(p.D0)).cuda()
        st, rep = rb.refine_eigvecs(A, X, D, target, rb.default_opts(group_tau=tau, max_iter=12))
        r = rep.as_dict()
        err = _fwd(rb.from_colmajor(X), Xt)
        res[tau] = (st, r["iters"], err)
        print(f"  tau={tau}: status={st} iters={r['iters']} groups={r['groups']} "
              f"eps={['%.1e' % e for e in r['eps']]} fwd={err:.2e}", flush=True)
    st, iters, err = res[1e-3]
    assert st == rb.REFEIG_OK and err <= target
    assert iters < res[0.0][1] or res[0.0][0] != rb.REFEIG_OK


@pytest.mark.parametrize("n", [255, 256, 257, 1023, 1024, 1025])
def test_tile_boundaries(n):
    """Orders on either side of the 256-column block and of the switch between the
    128 x 128 and 256 x 256 GEMM kernels (npad 1024), to target against X_true."""
    rb = _rb()
    target = 1e-13
    p = workloads.make_problem(2, n, x0="eigh")
    Xt, lt = _xtrue(p)
    A, X, D = _to_dev(p)
    st, rep = rb.refine_eigvecs(A, X, D, target)
    err = _fwd(rb.from_colmajor(X), Xt)
    print(f"  n={n} status={st} iters={rep.iters} fwd={err:.2e}", flush=True)
    assert st == rb.REFEIG_OK, rb.strerror(st)
    assert err <= target


def test_sparse_rule_band_matrix():
    """The sparse rule on a band matrix (half-bandwidth 3, so k = 7 nonzeros per row):
    refeig_row_nonzeros finds k; one step matches the oracle's step with xi = min(k^2, n);
    the solve reaches the target against X_true."""
    import torch
    rb = _rb()
    n, target = 600, 1e-13
    p = workloads.banded_problem(n, 3)
    A, X, D = _to_dev(p)
    k = rb.row_nonzeros(A)
    assert k == 7
    opts = rb.default_opts(fixed_iters=1, sparse_k=k)
    st, rep = rb.refine_eigvecs(A, X, D, target, opts)
    assert st == rb.REFEIG_OK, rb.strerror(st)
    ref = oracle.method_step(p.A, p.X0, p.D0, target / opts.delta_safety, xi=float(min(k * k, n)))
    assert rep.beta[0] == ref.beta and rep.kx[0] == ref.kx
    assert float(np.max(np.abs(rb.from_colmajor(X) - ref.X_hi))) <= target / opts.delta_safety
    Xt, _ = _xtrue(p)
    A, X, D = _to_dev(p)
    st, rep = rb.refine_eigvecs(A, X, D, target, rb.default_opts(sparse_k=k))
    err = _fwd(rb.from_colmajor(X), Xt)
    print(f"  sparse rule: iters={rep.iters} kx={list(rep.kx[:rep.iters])} fwd={err:.2e}", flush=True)
    assert st == rb.REFEIG_OK and err <= target


def test_adaptive_schedule():
    """The adaptive accuracy schedule (an extension beyond the paper): from a start with
    mixed pairs (errors up to 0.35) the second iteration's products aim at a looser level
    than the final delta, never above eps^4 / 100 of the first correction, the last
    iteration's products aim at the final delta, and the solve still meets the target
    against X_true in no more iterations than the paper's schedule."""
    import torch
    rb = _rb()
    target = 1e-14
    p = workloads.make_problem(3, 700, x0="eigh")
    Xt, lt = _xtrue(p)
    X0 = _mixed_start(p, [(10, 11), (300, 301), (650, 651)], [0.35, 0.25, 0.15])
    res = {}
    for sched in (0, 1):
        A, X = rb.colmajor(p.A), rb.colmajor(X0)
        D = torch.from_numpy(np.array(p.D0)).cuda()
        st, rep = rb.refine_eigvecs(A, X, D, target, rb.default_opts(schedule=sched, max_iter=12))
        r = rep.as_dict()
        err = _fwd(rb.from_colmajor(X), Xt)
        res[sched] = (st, r, err)
        print(f"  schedule={sched}: status={st} iters={r['iters']} "
              f"delta={['%.1e' % d for d in r['delta_it']]} kx={r['kx']} "
              f"eps={['%.1e' % e for e in r['eps']]} fwd={err:.2e}", flush=True)
    st, r, err = res[1]
    assert st == rb.REFEIG_OK, rb.strerror(st)
    assert err <= target
    delta = target / rb.default_opts().delta_safety
    assert r["delta_it"][0] == delta and res[0][1]["delta_it"] == [delta] * res[0][1]["iters"]
    assert delta < r["delta_it"][1] <= 0.01 * r["eps"][0] ** 4
    assert r["delta_it"][-1] == delta
    assert r["iters"] <= res[0][1]["iters"]


@pytest.mark.parametrize("cfg,n,target", [(1, 100, 1e-14), (2, 300, 1e-12), (3, 1100, 1e-14)])
def test_one_step_v_by_residues_vs_oracle(cfg, n, target):
    """vmode = 1 (V as the exact product of A's digits and X^(1) by residues and the Chinese
    remainder theorem, an alternative to the slice products): one step against the oracle's
    exact-product step, to the same bar as the slice form."""
    print(f"step vmode=1 cfg={cfg} n={n} target={target}", flush=True)
    rb = _rb()
    p = workloads.make_problem(cfg, n, x0="eigh")
    A, X, D = _to_dev(p)
    opts = rb.default_opts(fixed_iters=1, vmode=1)
    st, rep = rb.refine_eigvecs(A, X, D, target, opts)
    assert st == rb.REFEIG_OK, rb.strerror(st)
    ref = oracle.method_step(p.A, p.X0, p.D0, target / opts.delta_safety)
    assert rep.beta[0] == ref.beta and rep.kx[0] == ref.kx
    Xg = rb.from_colmajor(X)
    diff = float(np.max(np.abs(Xg - ref.X_hi)))
    print(f"  moduli={rep.pairs_p[0][0]} dv={rep.dv[0]} |X_gpu - X_oracle|max={diff:.3e}",
          flush=True)
    assert 10 <= rep.pairs_p[0][0] <= 32
    assert diff <= target / opts.delta_safety
    _check_step_lambdas(D, ref, p.D0, target / opts.delta_safety, opts.theta)


@pytest.mark.parametrize("cfg,n,target", [(3, 700, 1e-14), (2, 1025, 1e-13), (1, 257, 1e-12)])
def test_refine_v_by_residues_to_target(cfg, n, target):
    print(f"refine vmode=1 cfg={cfg} n={n} target={target}", flush=True)
    rb = _rb()
    p = workloads.make_problem(cfg, n, x0="eigh")
    Xt, lt = _xtrue(p)
    A, X, D = _to_dev(p)
    st, rep = rb.refine_eigvecs(A, X, D, target, rb.default_opts(vmode=1))
    err = _fwd(rb.from_colmajor(X), Xt)
    print(f"  status={st} iters={rep.iters} fwd={err:.3e}", flush=True)
    assert st == rb.REFEIG_OK, rb.strerror(st)
    assert err <= target


@pytest.mark.parametrize("cfg,n,target,vmode", [(3, 1024, 1e-8, 1), (3, 1024, 1e-11, 1),
                                                (3, 1100, 1e-8, 0)])
def test_loose_target_is_a_stable_fixed_point(cfg, n, target, vmode):
    """A loose target on a spectrum whose smallest gap is tiny next to max|lambda| (config 3:
    g / L about 3e-14 at n = 1024). The products' error in a column returns in the next
    iteration amplified by about max|lambda| / g_j (the amplification of the X^(1) cut of
    Sec. 4.1), so iterating past convergence must not drift above the target: the solve
    with the stopping rule, and one of 8 fixed iterations, both meet it."""
    print(f"loose target cfg={cfg} n={n} target={target} vmode={vmode}", flush=True)
    rb = _rb()
    p = workloads.make_problem(cfg, n, x0="eigh")
    Xt, lt = _xtrue(p)
    for fixed in (0, 8):
        A, X, D = _to_dev(p)
        st, rep = rb.refine_eigvecs(A, X, D, target, rb.default_opts(vmode=vmode,
                                                                     fixed_iters=fixed))
        err = _fwd(rb.from_colmajor(X), Xt)
        print(f"  fixed_iters={fixed} status={st} iters={rep.iters} "
              f"eps={['%.1e' % e for e in rep.eps[:rep.iters]]} fwd={err:.3e}", flush=True)
        assert st == rb.REFEIG_OK, rb.strerror(st)
        assert err <= target


def test_config1_slice_counts():
    """Config 1 (n = 100, cond 1e8) read as "4 INT8 slices": k_X = 4 is what the beta rule of
    Sec. 4.1 gives at target 1e-6 (internal delta 1.25e-7; the oracle's rule agrees), but 4
    digit planes of A (28 bits) cannot resolve the bottom gaps (about 2e-9 of max|lambda|).
    3 fixed iterations from the FP64 eigensolve start: the automatic plane counts meet 1e-6,
    k_A = 4 does not, and the k_A x k_X grid is printed (rows k_A = 2..14, columns k_X = 2..8)."""
    rb = _rb()
    p = workloads.make_problem(1, 100, x0="eigh")
    Xt, _ = _xtrue(p)
    target = 1e-6

    def run(**kw):
        A, X, D = _to_dev(p)
        st, rep = rb.refine_eigvecs(A, X, D, target, rb.default_opts(fixed_iters=3, **kw))
        err = _fwd(rb.from_colmajor(X), Xt) if st >= 0 else float("nan")
        return st, rep, err

    st, rep, err = run()
    print(f"  automatic: kx {list(rep.kx[:3])} dv {list(rep.dv[:3])} fwd {err:.2e}", flush=True)
    assert st == rb.REFEIG_OK and err <= target
    assert rep.kx[0] == oracle.beta_rule(p.D0, p.X0, target / 8)["kx"] == 4
    st, rep, err4 = run(ka_max=4, kx_force=4)
    print(f"  k_A = 4, k_X = 4: status {st} fwd {err4:.2e}", flush=True)
    assert not (st == rb.REFEIG_OK and err4 <= target)
    for ka in range(2, 15, 2):
        row = []
        for kx in range(2, 9):
            st, rep, e = run(ka_max=ka, kx_force=kx)
            row.append(f"{e:8.1e}" if st >= 0 else f"{'st' + str(st):>8}")
        print(f"  k_A={ka:2d}: " + " ".join(row), flush=True)


def test_server_results_match_single_calls():
    """The continuous-batching server with admission by HBM footprint: config-4 style
    requests of uneven n and mixed targets (1e-8, 1e-11, 1e-14, the serving mix), submitted
    while earlier ones run on 4 lanes from an arena that holds about three of the largest
    footprints, each come back bit for bit as a single call alone gives them (stop rule on,
    so the iteration counts differ between requests). A request whose footprint exceeds the
    arena, unknown tickets and a second wait are refused."""
    import time
    import torch
    rb = _rb()
    ns, cs = workloads.config4_sizes(24)
    probs = [workloads.make_problem(4, int(n), index=100 + i, cond_exp=float(c))
             for i, (n, c) in enumerate(zip(ns, cs))]
    targets = [(1e-8, 1e-11, 1e-14)[i % 3] for i in range(len(probs))]
    singles = []
    for p, t in zip(probs, targets):
        A, X, D = _to_dev(p)
        st, rep = rb.refine_eigvecs(A, X, D, t)
        singles.append((st, rep.iters, X.cpu().numpy(), D.cpu().numpy()))
    budget = 3 * rb.server_request_bytes(max(p.n for p in probs))
    srv = rb.Server(4, budget)
    try:
        dev = [_to_dev(p) for p in probs]
        torch.cuda.synchronize()
        t0 = time.monotonic()
        tickets = [srv.submit(A, X, D, t) for (A, X, D), t in zip(dev, targets)]
        done = [srv.wait(k) for k in tickets]
        for (A, X, D), (st1, it1, Xs, Ds), (st, rep, td), p in zip(dev, singles, done, probs):
            assert st == st1 and rep.iters == it1, (p.n, st, st1, rep.iters, it1)
            assert td >= t0
            assert np.array_equal(X.cpu().numpy(), Xs) and np.array_equal(D.cpu().numpy(), Ds)
        print("server: n", [p.n for p in probs], "iters", [r.iters for _, r, _ in done],
              flush=True)
        with pytest.raises(ValueError):
            srv.wait(tickets[0])                      # already waited for
        with pytest.raises(ValueError):
            srv.wait(10 ** 6)
    finally:
        srv.close()
    # a footprint above the arena can never start: refused at submission
    small = rb.Server(2, rb.server_request_bytes(256))
    try:
        big = workloads.make_problem(4, 700, index=999, cond_exp=6.0)
        A, X, D = _to_dev(big)
        with pytest.raises(ValueError):
            small.submit(A, X, D, 1e-14)
    finally:
        small.close()


def test_server_waits_for_the_callers_stream():
    """A request submitted right after asynchronous copies of its inputs on the caller's
    stream (no synchronisation in between) reads the copied values: the lane waits for an
    event recorded on that stream."""
    import torch
    rb = _rb()
    p = workloads.make_problem(2, 1024, x0="eigh")
    A, X0, D0 = _to_dev(p)
    X1, D1 = X0.clone(), D0.clone()
    st1, _ = rb.refine_eigvecs(A, X1, D1, 1e-13)
    assert st1 == rb.REFEIG_OK
    srv = rb.Server(2, 2 * rb.server_request_bytes(1024))
    try:
        for rep_i in range(3):
            X = torch.zeros_like(X0)
            D = torch.zeros_like(D0)
            torch.cuda.synchronize()
            X.copy_(X0)            # asynchronous on the current stream
            D.copy_(D0)
            k = srv.submit(A, X, D, 1e-13)
            st, _, _ = srv.wait(k)
            assert st == rb.REFEIG_OK, rb.strerror(st)
            assert torch.equal(X, X1) and torch.equal(D, D1), rep_i
    finally:
        srv.close()
