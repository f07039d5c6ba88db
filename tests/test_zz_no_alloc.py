"""The entry point that allocates nothing (refine_eigvecs_noalloc, workspace in the library's
static device array) against refine_eigvecs on the same inputs: bit-identical X, D and
report, on two calls in a row, the second with a smaller input (the array keeps the first
call's contents)."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _dev(p):
    import torch
    from paper_2602_19090_amd import binding as rb
    return rb.colmajor(p.A), rb.colmajor(p.X0), torch.from_numpy(np.array(p.D0)).cuda()


def test_noalloc_matches_refine_eigvecs():
    import torch
    from paper_2602_19090_amd import binding as rb
    for cfg, n, target in [(3, 1024, 1e-14), (2, 300, 1e-12)]:
        print(f"noalloc cfg={cfg} n={n} target={target}", flush=True)
        p = workloads.make_problem(cfg, n, x0="eigh")
        A, X1, D1 = _dev(p)
        st1, r1 = rb.refine_eigvecs(A, X1, D1, target)
        A2, X2, D2 = _dev(p)
        st2, r2 = rb.refine_eigvecs_noalloc(A2, X2, D2, target)
        torch.cuda.synchronize()
        assert st1 == st2 == rb.REFEIG_OK, (rb.strerror(st1), rb.strerror(st2))
        assert r1.iters == r2.iters and list(r1.eps[:r1.iters]) == list(r2.eps[:r2.iters])
        assert torch.equal(X1, X2) and torch.equal(D1, D2)


def test_noalloc_limits():
    import torch
    from paper_2602_19090_amd import binding as rb
    p = workloads.make_problem(2, 64, x0="eigh")
    A, X, D = _dev(p)
    st, _ = rb.refine_eigvecs_noalloc(A, X, D, 1e-12, rb.default_opts(mode=rb.REFEIG_FP64_PLAIN))
    assert st == rb.REFEIG_E_ARG
    n = 1025
    A = torch.eye(n, dtype=torch.float64, device="cuda")
    X = torch.eye(n, dtype=torch.float64, device="cuda")
    D = torch.arange(n, dtype=torch.float64, device="cuda")
    st, _ = rb.refine_eigvecs_noalloc(A, X, D, 1e-12)
    assert st == rb.REFEIG_E_NOMEM
