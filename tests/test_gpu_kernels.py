"""Bit-exact parity of the HIP splitter and INT8 slice GEMM with the CPU oracle.

Both entry points are integer work: digit planes, exponents and the INT32
slice products must equal the oracle's exactly.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _rb():
    from paper_2602_19090_amd import binding
    return binding


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _adversarial(rows, cols, seed):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((rows, cols)) * 2.0 ** rng.integers(-30, 30, (rows, cols))
    M[:, 0] = 0.0                                            # zero column
    if cols > 1:
        M[:, 1] = rng.uniform(-1, 1, rows) * 0.5
        M[rows // 2, 1] = -1.0                               # power-of-two maximum
    if cols > 2:
        M[:, 2] = 0.0
        M[0, 2] = 5e-324                                     # subnormals under a normal max
        M[-1, 2] = 3.0
    if cols > 3:
        M[:, 3] = np.nextafter(1.0, 0.0) * rng.choice([-1, 1], rows)
    return np.asfortranarray(M)


@pytest.mark.parametrize("rows,cols", [(1, 1), (7, 3), (100, 37), (300, 513), (1000, 1000)])
@pytest.mark.parametrize("k", [1, 7, 12])
def test_split_bitexact(rows, cols, k):
    print(f"split rows={rows} cols={cols} k={k}", flush=True)
    rb = _rb()
    M = _adversarial(rows, cols, rows * 7919 + cols * 31 + k)
    st, e, pl, tr = rb.split_cols(rb.colmajor(M), rows, cols, k)
    assert st == 0, rb.strerror(st)
    e_o, pl_o, tr_o = oracle.split_s7(M, k)
    np.testing.assert_array_equal(e.cpu().numpy(), e_o)
    P = rb.kblocked_to_rows(pl).cpu().numpy()
    np.testing.assert_array_equal(P[:, :cols, :rows], pl_o)
    assert not P[:, cols:, :].any() and not P[:, :, rows:].any()
    np.testing.assert_array_equal(rb.from_colmajor(tr), tr_o)


def test_split_errors():
    rb = _rb()
    M = np.asfortranarray(np.ones((10, 4)))
    M[3, 2] = np.nan
    st, *_ = rb.split_cols(rb.colmajor(M), 10, 4, 3)
    assert st == rb.REFEIG_E_NONFINITE
    M = np.asfortranarray(np.ones((10, 4)))
    M[:, 1] = 1e-150
    st, *_ = rb.split_cols(rb.colmajor(M), 10, 4, 3)
    assert st == rb.REFEIG_E_RANGE
    st, *_ = rb.split_cols(rb.colmajor(M), 10, 4, 19)
    assert st == rb.REFEIG_E_ARG


def _diag_products_oracle(Lp, Rp, kl, kr, d_min, ndiag, rows=None, cols=None):
    """Per-diagonal sums of exact int64 slice products, optionally on sampled rows/cols."""
    out = []
    for q in range(ndiag):
        d = d_min + q
        acc = None
        for s in range(max(1, d - kr), min(kl, d - 1) + 1):
            L = Lp[s - 1] if rows is None else Lp[s - 1][rows]
            R = Rp[d - s - 1] if cols is None else Rp[d - s - 1][cols]
            c = oracle.slice_gemm_i64(L, R)
            acc = c if acc is None else acc + c
        out.append(acc)
    return out


@pytest.mark.parametrize("npad,kl,kr", [(256, 1, 1), (256, 3, 5), (512, 7, 2), (512, 4, 9),
                                         (1024, 2, 3), (1536, 1, 2)])
def test_slice_gemm_bitexact(npad, kl, kr):
    print(f"gemm npad={npad} kl={kl} kr={kr}", flush=True)
    torch = _torch()
    rb = _rb()
    rng = np.random.default_rng(npad + 10 * kl + kr)
    Lp = rng.integers(-127, 128, (kl, npad, npad)).astype(np.int8)
    Rp = rng.integers(-127, 128, (kr, npad, npad)).astype(np.int8)
    ndiag = kl + kr - 1
    st, C = rb.slice_gemm(rb.rows_to_kblocked(torch.from_numpy(Lp).cuda()),
                          rb.rows_to_kblocked(torch.from_numpy(Rp).cuda()), npad, kl, kr, 2, ndiag)
    assert st == 0
    Cg = C.cpu().numpy()
    ref = _diag_products_oracle(Lp, Rp, kl, kr, 2, ndiag)
    for q in range(ndiag):
        np.testing.assert_array_equal(Cg[q].astype(np.int64), ref[q])


def test_slice_gemm_full_size_sampled():
    """n = 8192 (the benchmark's size) with the V product's plane counts (kx = 7, ka = 16,
    diagonals 2..17), checked on sampled rows and columns computed one by one."""
    torch = _torch()
    rb = _rb()
    npad, kl, kr, ndiag = 8192, 7, 16, 16
    g = torch.Generator(device="cuda").manual_seed(5)
    Lp = torch.randint(-127, 128, (kl, npad, npad), dtype=torch.int8, device="cuda", generator=g)
    Rp = torch.randint(-127, 128, (kr, npad, npad), dtype=torch.int8, device="cuda", generator=g)
    st, C = rb.slice_gemm(Lp, Rp, npad, kl, kr, 2, ndiag)
    torch.cuda.synchronize()
    assert st == 0
    rng = np.random.default_rng(6)
    rows = np.sort(rng.choice(npad, 24, replace=False))
    cols = np.sort(rng.choice(npad, 24, replace=False))
    rows[0], cols[-1] = 0, npad - 1
    ridx = torch.from_numpy(rows).cuda()
    cidx = torch.from_numpy(cols).cuda()
    Ls = rb.kblocked_to_rows(Lp)[:, ridx, :].cpu().numpy()   # the planes are read K-blocked
    Rs = rb.kblocked_to_rows(Rp)[:, cidx, :].cpu().numpy()
    ref = _diag_products_oracle(Ls, Rs, kl, kr, 2, ndiag)
    Cs = C[:, ridx][:, :, cidx].cpu().numpy()
    for q in range(ndiag):
        np.testing.assert_array_equal(Cs[q].astype(np.int64), ref[q])
    del C, Lp, Rp
    torch.cuda.empty_cache()


def test_slice_gemm_int32_extreme():
    """All digits -127 with 9 pairs on one diagonal at K = 8192: 9 * 8192 * 127^2 is within
    2^31 and must come out exactly."""
    torch = _torch()
    rb = _rb()
    npad, k = 8192, 9
    Lp = torch.full((k, npad, npad), -127, dtype=torch.int8, device="cuda")
    st, C = rb.slice_gemm(Lp, Lp, npad, k, k, 10, 1)
    torch.cuda.synchronize()
    assert st == 0
    assert int(C.min()) == int(C.max()) == 9 * 8192 * 127 * 127
    del C, Lp
    torch.cuda.empty_cache()


def test_slice_gemm_rejects_overflow_and_bad_args():
    torch = _torch()
    rb = _rb()
    Lp = torch.zeros((2, 256, 256), dtype=torch.int8, device="cuda")
    st, _ = rb.slice_gemm(Lp, Lp, 256, 2, 2, 1, 1)        # d_min < 2
    assert st == rb.REFEIG_E_ARG
    st, _ = rb.slice_gemm(Lp, Lp, 256, 2, 2, 2, 4)        # diagonal 5 > kl + kr
    assert st == rb.REFEIG_E_ARG


def test_mfma_ceiling_probe():
    """The matrix-core probe runs and reports a rate and clock in the hardware's range: at most
    the dense INT8 peak (5.0 POP/s at 2.4 GHz), the clock below the nominal 2.4 GHz."""
    from paper_2602_19090_amd import binding as rb
    for variant in (0, 1, 2):
        st, ms, pops, ghz = rb.mfma_ceiling(variant, 0.05)
        print("variant", variant, "ms", round(ms, 2), "POP/s", round(pops, 3), "GHz", round(ghz, 3),
              flush=True)
        assert st == rb.REFEIG_OK
        assert 0.3 < pops <= 5.0 and 0.5 < ghz <= 2.5 and ms > 0.0
        # the rate cannot exceed what the reported clock allows (1024 SIMDs x 2048 ops/cycle)
        assert pops <= 1024 * 2048 * ghz * 1e9 / 1e15 * 1.02
