"""Device-side planning of the iteration (opts.plan = 0, the default) against host-side
planning (opts.plan = 1): the same plan, so bit-identical X, D and report; and a fixed-
iteration solve enqueued without any wait, captured in a HIP graph and replayed, bit-identical
to the same solve run directly."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _rb():
    from paper_2602_19090_amd import binding
    return binding


def _dev(p):
    import torch
    rb = _rb()
    return rb.colmajor(p.A), rb.colmajor(p.X0), torch.from_numpy(np.array(p.D0)).cuda()


_FIELDS = ("beta", "kx", "dv", "dw", "du", "pairs_f", "eps", "vres", "delta_it")


@pytest.mark.parametrize("cfg,n,target,kw", [
    (1, 100, 1e-14, {}), (2, 300, 1e-12, {}), (3, 1100, 1e-14, {}), (2, 1025, 1e-13, {}),
    (3, 700, 1e-8, {}), (1, 257, 1e-12, {"vmode": 0}), (3, 1024, 1e-11, {"vmode": 0}),
    (2, 64, 1e-13, {"fixed_iters": 3}), (3, 1100, 1e-14, {"kx_force": 9}),
    (1, 300, 1e-12, {"stop_rule": 1}), (2, 512, 1e-14, {"sparse_k": 7})])
def test_device_plan_matches_host_plan(cfg, n, target, kw):
    import torch
    rb = _rb()
    print(f"device vs host planning cfg={cfg} n={n} target={target} {kw}", flush=True)
    p = workloads.make_problem(cfg, n, x0="eigh")
    out = []
    for plan in (1, 0):
        A, X, D = _dev(p)
        st, rep = rb.refine_eigvecs(A, X, D, target, rb.default_opts(plan=plan, **kw))
        torch.cuda.synchronize()
        out.append((st, rep.as_dict(), X.cpu().numpy(), D.cpu().numpy()))
    (sh, rh, Xh, Dh), (sd, rd, Xd, Dd) = out
    assert sh == sd, (rb.strerror(sh), rb.strerror(sd))
    assert rh["iters"] == rd["iters"]
    for f in _FIELDS:
        assert rh[f] == rd[f], (f, rh[f], rd[f])
    assert np.array_equal(Xh, Xd) and np.array_equal(Dh, Dd)
    print(f"  status {rb.strerror(sd)} iters {rd['iters']} kx {rd['kx']} pairs "
          f"{[round(sum(x), 2) for x in rd['pairs_f']]}", flush=True)


def test_device_plan_error_paths_keep_the_last_iterate():
    """Coincident eigenvalue estimates and NaN inputs end the device-planned solve with the
    host path's status, and X, D keep their entry values."""
    import torch
    rb = _rb()
    p = workloads.make_problem(2, 200, x0="eigh")
    A, X, D = _dev(p)
    D[5] = D[6]
    X0, D0 = X.clone(), D.clone()
    st, _ = rb.refine_eigvecs(A, X, D, 1e-12)
    assert st == rb.REFEIG_E_GAP
    assert torch.equal(X, X0) and torch.equal(D, D0)
    A, X, D = _dev(p)
    X[3, 7] = float("nan")
    X0 = X.clone()
    st, _ = rb.refine_eigvecs(A, X, D, 1e-12, rb.default_opts(fixed_iters=2))
    assert st == rb.REFEIG_E_NONFINITE
    assert torch.equal(torch.nan_to_num(X), torch.nan_to_num(X0))


@pytest.mark.parametrize("cfg,n", [(3, 1024), (2, 300)])
def test_graph_captured_fixed_iterations(cfg, n):
    """A 3-iteration solve enqueued with enqueue_only (no wait, no allocation, device planning)
    is captured in a HIP graph on a side stream and replayed three times, with the inputs reset
    in between; every replay gives X, D and the report bit for bit as the direct solve."""
    import torch
    rb = _rb()
    print(f"graph capture cfg={cfg} n={n}", flush=True)
    p = workloads.make_problem(cfg, n, x0="eigh")
    A, X0, D0 = _dev(p)
    target = 1e-14
    opts = rb.default_opts(fixed_iters=3)
    work = torch.empty(rb.workspace_bytes(n, opts), dtype=torch.uint8, device="cuda")
    Xr, Dr = X0.clone(), D0.clone()
    st, rep = rb.refine_eigvecs(A, Xr, Dr, target, opts, work=work)
    assert st == rb.REFEIG_OK, rb.strerror(st)
    ref = rep.as_dict()
    eopts = rb.default_opts(fixed_iters=3, enqueue_only=1)
    X, D = X0.clone(), D0.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        st_c, _ = rb.refine_eigvecs(A, X, D, target, eopts, work=work, stream=s)
    assert st_c == rb.REFEIG_OK, rb.strerror(st_c)
    for rep_i in range(3):
        X.copy_(X0)
        D.copy_(D0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        st2, rep2 = rb.read_report(work, n, eopts)
        assert st2 == rb.REFEIG_OK, rb.strerror(st2)
        r2 = rep2.as_dict()
        assert r2["iters"] == 3
        for f in ("beta", "kx", "dv", "dw", "du", "eps", "vres"):
            assert r2[f] == ref[f], (rep_i, f, r2[f], ref[f])
        assert torch.equal(X, Xr) and torch.equal(D, Dr), rep_i
    # enqueue_only needs a caller workspace and a fixed iteration count
    assert rb.refine_eigvecs(A, X, D, target, rb.default_opts(enqueue_only=1), work=work)[0] == \
        rb.REFEIG_E_ARG
    assert rb.refine_eigvecs(A, X, D, target, eopts)[0] == rb.REFEIG_E_ARG
