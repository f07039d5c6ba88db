"""The FP8 ablation of the slice products (4-bit digits in FP8 E4M3 operands, the error-free
products of Sec. 2.3 with a narrower digit): integer work, so bit-exact.

* The E4M3 code of every digit in [-15, 15] decodes, by the format's own definition (sign
  bit, 4 exponent bits with bias 7, 3 mantissa bits, subnormals at exponent field 0), to that
  digit.
* The per-diagonal products equal the oracle's exact int64 slice products and the INT8
  kernel's on the same digits, across tiles and diagonals.
* At n = 8192 with 9 pairs of all-15 digits every entry is 9 * 8192 * 15^2 = 16,588,800,
  just under 2^24, the largest sum that FP32 holds exactly; 10 pairs are refused.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _rb():
    from paper_2602_19090_amd import binding
    return binding


def _decode_e4m3(b):
    b = b.astype(np.int64)
    s = np.where(b >> 7, -1.0, 1.0)
    e = (b >> 3) & 15
    m = b & 7
    normal = (1.0 + m / 8.0) * np.exp2(e - 7.0)
    sub = (m / 8.0) * 2.0 ** -6
    return s * np.where(e == 0, sub, normal)


def test_digit_codes_decode_to_the_digits():
    import torch
    rb = _rb()
    digits = np.arange(-15, 16, dtype=np.int8)
    st, codes = rb.digits_to_e4m3(torch.from_numpy(digits).cuda())
    assert st == rb.REFEIG_OK
    c = codes.cpu().numpy()
    np.testing.assert_array_equal(_decode_e4m3(c), digits.astype(np.float64))
    assert c[15] == 0                         # +0, not -0
    bad = torch.tensor([3, 16, -2], dtype=torch.int8, device="cuda")
    st, _ = rb.digits_to_e4m3(bad)
    assert st == rb.REFEIG_E_ARG


def _diag_products_oracle(Lp, Rp, kl, kr, d_min, ndiag):
    out = []
    for q in range(ndiag):
        d = d_min + q
        acc = None
        for s in range(max(1, d - kr), min(kl, d - 1) + 1):
            c = oracle.slice_gemm_i64(Lp[s - 1], Rp[d - s - 1])
            acc = c if acc is None else acc + c
        out.append(acc)
    return out


@pytest.mark.parametrize("npad,kl,kr", [(1024, 3, 4), (1280, 2, 2)])
def test_fp8_slice_products_bitexact(npad, kl, kr):
    print(f"fp8 gemm npad={npad} kl={kl} kr={kr}", flush=True)
    import torch
    rb = _rb()
    rng = np.random.default_rng(npad + kl)
    Lp = rng.integers(-15, 16, (kl, npad, npad)).astype(np.int8)
    Rp = rng.integers(-15, 16, (kr, npad, npad)).astype(np.int8)
    Lk = rb.rows_to_kblocked(torch.from_numpy(Lp).cuda())
    Rk = rb.rows_to_kblocked(torch.from_numpy(Rp).cuda())
    st1, L8 = rb.digits_to_e4m3(Lk)
    st2, R8 = rb.digits_to_e4m3(Rk)
    assert st1 == st2 == rb.REFEIG_OK
    ndiag = kl + kr - 1
    st, C8 = rb.slice_gemm_fp8(L8, R8, npad, kl, kr, 2, ndiag)
    assert st == rb.REFEIG_OK
    st, Ci = rb.slice_gemm(Lk, Rk, npad, kl, kr, 2, ndiag)
    assert st == rb.REFEIG_OK
    assert torch.equal(C8, Ci)
    Cg = C8.cpu().numpy()
    ref = _diag_products_oracle(Lp, Rp, kl, kr, 2, ndiag)
    for q in range(ndiag):
        np.testing.assert_array_equal(Cg[q].astype(np.int64), ref[q])


def test_fp8_exact_at_the_fp32_limit():
    import torch
    rb = _rb()
    npad, k = 8192, 9
    D = torch.full((k, npad, npad), 15, dtype=torch.int8, device="cuda")
    st, P8 = rb.digits_to_e4m3(D)
    assert st == rb.REFEIG_OK
    del D
    st, C = rb.slice_gemm_fp8(P8, P8, npad, k, k, 10, 1)
    torch.cuda.synchronize()
    assert st == rb.REFEIG_OK
    assert int(C.min()) == int(C.max()) == 9 * 8192 * 15 * 15
    del C
    Q8 = torch.zeros((10, npad, npad), dtype=torch.uint8, device="cuda")
    st, _ = rb.slice_gemm_fp8(Q8, Q8, npad, 10, 10, 11, 1)     # 10 pairs: over 2^24
    assert st == rb.REFEIG_E_ARG
    st, _ = rb.slice_gemm_fp8(Q8[:, :512, :512].contiguous(), Q8[:, :512, :512].contiguous(),
                              512, 2, 2, 2, 1)               # npad < 1024
    assert st == rb.REFEIG_E_ARG
    del P8, Q8
    torch.cuda.empty_cache()
