"""Grouped batches (refine_eigvecs_batched with device planning): the solves of a batch advance
together, one launch per step and size class, the three products as persistent kernels over
a device-built list of (problem, tile, slot) items. Every problem's arithmetic is its single
call's, so X, D, the status and the plan (beta, k_X, pairs) must match the single call bit for
bit; covered: both GEMM tile sizes (npad below and from 1024), the stop test (problems that
stop at different iterations), several memory chunks, a problem above the grouped size
limit (run alone), and per-problem error statuses inside a batch."""
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _rb():
    from paper_2602_19090_amd import binding
    return binding


def _to_dev(p):
    import torch
    rb = _rb()
    return rb.colmajor(p.A), rb.colmajor(p.X0), torch.from_numpy(np.array(p.D0)).cuda()


def _singles(probs, targets, opts):
    rb = _rb()
    out = []
    for p, t in zip(probs, targets):
        A, X, D = _to_dev(p)
        st, rep = rb.refine_eigvecs(A, X, D, t, opts)
        out.append((st, X.cpu().numpy(), D.cpu().numpy(), rep))
    return out


def _check_batch(probs, targets, opts, singles):
    import torch
    rb = _rb()
    dev = [_to_dev(p) for p in probs]
    st, reps = rb.refine_eigvecs_batched([d[0] for d in dev], [d[1] for d in dev],
                                         [d[2] for d in dev], targets, opts)
    torch.cuda.synchronize()
    worst = max((s[0] for s in singles), key=lambda v: (v < 0, abs(v)))
    assert st == worst or (st >= 0 and all(s[0] >= 0 for s in singles)), (st, worst)
    for k, ((A, X, D), (s_st, Xs, Ds, srep), r) in enumerate(zip(dev, singles, reps)):
        assert r.status == s_st, (k, probs[k].n, r.status, s_st)
        assert r.iters == srep.iters, (k, probs[k].n, r.iters, srep.iters)
        it = r.iters
        assert list(r.beta[:it]) == list(srep.beta[:it]) and list(r.kx[:it]) == list(srep.kx[:it])
        assert list(r.vres[:it]) == list(srep.vres[:it])
        assert [r.pairs_f[i][q] for i in range(it) for q in range(3)] == \
            [srep.pairs_f[i][q] for i in range(it) for q in range(3)]
        assert np.array_equal(X.cpu().numpy(), Xs), (k, probs[k].n)
        assert np.array_equal(D.cpu().numpy(), Ds), (k, probs[k].n)
    return reps


def _mix():
    """Orders on both sides of the 1024 tile switch and across size classes, ragged tails,
    mixed condition numbers and targets."""
    ns = [40, 1000, 130, 1024, 257, 700, 1030, 96, 1500, 512, 33, 2100]
    probs = [workloads.make_problem(4, n, index=100 + i, cond_exp=4.0 + (i * 5) % 9)
             for i, n in enumerate(ns)]
    targets = [(1e-8, 1e-11, 1e-14)[i % 3] for i in range(len(ns))]
    return probs, targets


def test_grouped_fixed_iters_both_tiles():
    rb = _rb()
    probs, targets = _mix()
    print("grouped, fixed 3 iterations, n:", [p.n for p in probs], flush=True)
    opts = rb.default_opts(fixed_iters=3)
    singles = _singles(probs, targets, opts)
    _check_batch(probs, targets, opts, singles)


def test_grouped_stop_rule_and_chunks():
    """Default options (stop test): problems stop at different iterations, later launches skip
    them; then the same batch in chunks of at most 96 MiB of workspaces."""
    rb = _rb()
    probs, targets = _mix()
    opts = rb.default_opts()
    singles = _singles(probs, targets, opts)
    print("single-call iterations:", [s[3].iters for s in singles], flush=True)
    assert len({s[3].iters for s in singles}) > 1
    _check_batch(probs, targets, opts, singles)
    os.environ["REFEIG_GROUP_CHUNK_MIB"] = "96"
    try:
        print("chunked: workspace", rb.batched_workspace_bytes([p.n for p in probs], opts) >> 20,
              "MiB", flush=True)
        _check_batch(probs, targets, opts, singles)
    finally:
        del os.environ["REFEIG_GROUP_CHUNK_MIB"]


def test_grouped_with_a_large_member_and_errors():
    """A member above the grouped size limit (npad > 4096) runs alone; a member with a NaN in
    X and one with coinciding eigenvalue estimates fail alone with their own statuses."""
    import torch
    rb = _rb()
    ns = [300, 4200, 64, 64, 900]
    probs = [workloads.make_problem(2 if n > 1000 else 4, n, index=200 + i, cond_exp=8.0)
             for i, n in enumerate(ns)]
    targets = [1e-12] * len(ns)
    opts = rb.default_opts(fixed_iters=2)
    dev = [_to_dev(p) for p in probs]
    dev[2][1][0, 0] = float("nan")
    dev[3][2][1] = dev[3][2][0]
    single = []
    for A, X, D in dev:
        X2, D2 = X.clone(), D.clone()
        st, rep = rb.refine_eigvecs(A, X2, D2, 1e-12, opts)
        single.append((st, X2.cpu().numpy(), D2.cpu().numpy(), rep))
    assert single[2][0] == rb.REFEIG_E_NONFINITE and single[3][0] == rb.REFEIG_E_GAP
    st, reps = rb.refine_eigvecs_batched([d[0] for d in dev], [d[1] for d in dev],
                                         [d[2] for d in dev], targets, opts)
    torch.cuda.synchronize()
    assert st < 0
    for k, ((A, X, D), (s_st, Xs, Ds, srep), r) in enumerate(zip(dev, single, reps)):
        assert r.status == s_st, (k, r.status, s_st)
        if s_st >= 0:
            assert np.array_equal(X.cpu().numpy(), Xs) and np.array_equal(D.cpu().numpy(), Ds)


def test_graph_captured_batch_replays():
    """A grouped batch captured once in a HIP graph (refeig_batch_*, 3 fixed iterations) and
    replayed three times, its inputs rewritten by eager copies between the replays: every
    replay gives bit for bit what refine_eigvecs_batched gives, statuses and plans included."""
    import torch
    rb = _rb()
    probs, targets = _mix()
    opts = rb.default_opts(fixed_iters=3)
    ref = [_to_dev(p) for p in probs]
    st, rreps = rb.refine_eigvecs_batched([d[0] for d in ref], [d[1] for d in ref],
                                          [d[2] for d in ref], targets, opts)
    torch.cuda.synchronize()
    assert st == rb.REFEIG_OK
    dev = [_to_dev(p) for p in probs]
    X0 = [d[1].clone() for d in dev]
    D0 = [d[2].clone() for d in dev]
    print("batch workspace", rb.batch_workspace_bytes([p.n for p in probs], opts) >> 20, "MiB",
          flush=True)
    b = rb.Batch([d[0] for d in dev], [d[1] for d in dev], [d[2] for d in dev], targets, opts)
    try:
        for rep in range(3):
            for (A, X, D), x0, d0 in zip(dev, X0, D0):
                X.copy_(x0)
                D.copy_(d0)
            torch.cuda.synchronize()
            b.launch()
            st, sts, reps = b.results()
            assert st == rb.REFEIG_OK and all(s == rb.REFEIG_OK for s in sts), (rep, sts)
            for k, ((A, X, D), (Ar, Xr, Dr), r, rr) in enumerate(zip(dev, ref, reps, rreps)):
                assert r.iters == rr.iters == 3
                assert list(r.beta[:3]) == list(rr.beta[:3]) and list(r.kx[:3]) == list(rr.kx[:3])
                assert np.array_equal(X.cpu().numpy(), Xr.cpu().numpy()), (rep, k, probs[k].n)
                assert np.array_equal(D.cpu().numpy(), Dr.cpu().numpy()), (rep, k, probs[k].n)
            print(f"replay {rep + 1}: bit-identical", flush=True)
    finally:
        b.close()



def test_tile_choice_does_not_change_results(tmp_path):
    """Orders from 1024 run on the 256-row tile or on the 128-row tile with each entry of the
    256-row plan split in four: the batch is bit-identical to single calls either way. Then a
    batch with timing enabled on an empty cache records a choice for each of its orders."""
    rb = _rb()
    probs, targets = _mix()
    opts = rb.default_opts(fixed_iters=3)
    singles = _singles(probs, targets, opts)
    for t in ("128", "256"):
        os.environ["REFEIG_TILE"] = t
        try:
            print("tile", t, flush=True)
            _check_batch(probs, targets, opts, singles)
        finally:
            del os.environ["REFEIG_TILE"]
    cache = tmp_path / "tiles.json"
    os.environ["REFEIG_TUNE_CACHE"] = str(cache)
    try:
        _check_batch(probs[:4], targets[:4], opts, singles[:4])   # orders 40, 1000, 130, 1024
        import json
        got = json.loads(cache.read_text())
        print("tuned:", got, flush=True)
        assert any(k.endswith(":1024") for k in got) and all(v in (128, 256) for v in got.values())
    finally:
        del os.environ["REFEIG_TUNE_CACHE"]
