"""Bit-exact parity of the integer stages of V by residues (the default form of
V = A X^(1)) and of the splitter's other outputs, against the oracle's definitions.

* Residue planes: the digits of the oracle's split encode integers; their residues mod
  each modulus are integer work and must match exactly.
* Residue products: the GEMM's per-modulus products, stored reduced mod m_q, against the
  exact products mod m_q (also with per-block slot counts and digit levels).
* The chain digits -> residues -> products against the exact integer product of the
  digit integers (Python integers on sampled entries), at the benchmark's n = 8192.
* The transposed planes of X^(1) and the column-order read path of the splitter.
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


def _padded_planes(pl, rpad, cpad):
    """oracle planes (k, cols, rows) -> zero-padded (k, cpad, rpad)."""
    k, c, r = pl.shape
    out = np.zeros((k, cpad, rpad), dtype=np.int8)
    out[:, :c, :r] = pl
    return out


@pytest.mark.parametrize("rows,cols,k", [(100, 37, 1), (300, 513, 7), (1000, 257, 16),
                                         (256, 256, 18)])
def test_residue_planes_bitexact(rows, cols, k):
    print(f"residue planes rows={rows} cols={cols} k={k}", flush=True)
    torch = _torch()
    rb = _rb()
    rng = np.random.default_rng(rows + 3 * cols + k)
    M = np.asfortranarray(rng.standard_normal((rows, cols)) * 2.0 ** rng.integers(-8, 8, (rows, cols)))
    _, pl, _ = oracle.split_s7(M, k)
    rpad, cpad = -(-rows // 256) * 256, -(-cols // 256) * 256
    P = _padded_planes(pl, rpad, cpad)
    P[:, 0, :k] = 127                                  # extreme digit strings
    P[:, 1, :k] = -127
    mods = oracle.coprime_moduli(28)
    st, res = rb.residue_planes(rb.rows_to_kblocked(torch.from_numpy(P).cuda()), k, mods)
    torch.cuda.synchronize()
    assert st == 0, rb.strerror(st)
    got = rb.kblocked_to_rows(res).cpu().numpy()
    np.testing.assert_array_equal(got, oracle.digit_residues(P, mods))


def test_residue_planes_rejects_bad_args():
    torch = _torch()
    rb = _rb()
    P = torch.zeros((2, 256, 256), dtype=torch.int8, device="cuda")
    assert rb.residue_planes(P, 2, [255, 254])[0] == rb.REFEIG_E_ARG     # even modulus
    assert rb.residue_planes(P, 2, [257])[0] == rb.REFEIG_E_ARG          # above 255
    assert rb.residue_planes(P, 19, [255])[0] == rb.REFEIG_E_ARG         # > 18 planes


def _random_residues(rng, mods, shape):
    return np.stack([rng.integers(-(m - 1) // 2, (m - 1) // 2 + 1, shape) for m in mods]
                    ).astype(np.int8)


@pytest.mark.parametrize("npad,nmod", [(256, 5), (512, 28), (1280, 22)])
def test_residue_gemm_bitexact(npad, nmod):
    """npad 256 and 512: the 128 x 128 tile kernel; 1280: the 256 x 256 kernel (five tile
    rows, not a multiple of the 8 XCDs)."""
    print(f"residue gemm npad={npad} nmod={nmod}", flush=True)
    torch = _torch()
    rb = _rb()
    rng = np.random.default_rng(npad + nmod)
    mods = oracle.coprime_moduli(nmod)
    L = _random_residues(rng, mods, (npad, npad))
    R = _random_residues(rng, mods, (npad, npad))
    L[:, 0, :] = np.array([(m - 1) // 2 for m in mods], dtype=np.int8)[:, None]
    R[:, 0, :] = np.array([-(m - 1) // 2 for m in mods], dtype=np.int8)[:, None]
    st, C = rb.residue_gemm(rb.rows_to_kblocked(torch.from_numpy(L).cuda()),
                            rb.rows_to_kblocked(torch.from_numpy(R).cuda()), npad, mods)
    torch.cuda.synchronize()
    assert st == 0, rb.strerror(st)
    np.testing.assert_array_equal(C.cpu().numpy(), oracle.residue_product(L, R, mods))


def test_residue_gemm_levels_and_slot_counts():
    """Per 256-row block of L: a slot count (slots beyond it are not computed and keep what
    C held) and a level (the R residues of plane level * 28 + q)."""
    torch = _torch()
    rb = _rb()
    npad, nmod, nlev = 1280, 20, 3
    rng = np.random.default_rng(11)
    mods = oracle.coprime_moduli(nmod)
    L = _random_residues(rng, mods, (npad, npad))
    Rall = np.zeros((nlev * 28, npad, npad), dtype=np.int8)
    for lv in range(nlev):
        Rall[lv * 28:lv * 28 + nmod] = _random_residues(rng, mods, (npad, npad))
    vblk = np.array([[20, 0], [7, 2], [0, 1], [13, 1], [20, 2]], dtype=np.int32)
    C0 = torch.full((nmod, npad, npad), -128, dtype=torch.int8, device="cuda")
    st, C = rb.residue_gemm(rb.rows_to_kblocked(torch.from_numpy(L).cuda()),
                            rb.rows_to_kblocked(torch.from_numpy(Rall).cuda()), npad, mods,
                            vblk=vblk, out=C0)
    torch.cuda.synchronize()
    assert st == 0, rb.strerror(st)
    Cg = C.cpu().numpy()
    for b, (cnt, lv) in enumerate(vblk):
        rows = slice(256 * b, 256 * (b + 1))
        if cnt > 0:
            ref = oracle.residue_product(L[:cnt, rows], Rall[lv * 28:lv * 28 + cnt], mods[:cnt])
            np.testing.assert_array_equal(Cg[:cnt, rows], ref)
        assert (Cg[cnt:, rows] == -128).all()
    # vblk needs the 256-tile kernel; bad counts and levels are refused
    assert rb.residue_gemm(torch.zeros((1, 512, 512), dtype=torch.int8, device="cuda"),
                           torch.zeros((1, 512, 512), dtype=torch.int8, device="cuda"), 512,
                           [255], vblk=np.zeros((2, 2), np.int32))[0] == rb.REFEIG_E_ARG
    bad = vblk.copy()
    bad[1, 1] = 4
    assert rb.residue_gemm(rb.rows_to_kblocked(torch.from_numpy(L).cuda()),
                           rb.rows_to_kblocked(torch.from_numpy(Rall).cuda()), npad, mods,
                           vblk=bad)[0] == rb.REFEIG_E_ARG


def _z(digits):
    z = 0
    for d in digits:
        z = z * 128 + int(d)
    return z


def _sym(z, m):
    r = z % m
    return r - m if r > m // 2 else r


def test_residue_chain_full_size_sampled():
    """n = 8192 with the benchmark's digit counts (A: 16 digits, X^(1): 8, 22 moduli, the
    count the residue plan takes for them): digit planes -> residue planes -> residue GEMM on
    the GPU, checked on sampled rows and columns against the exact integer product of the
    digit integers, computed with Python integers."""
    torch = _torch()
    rb = _rb()
    npad, ka, kx = 8192, 16, 8
    plan = rb.host_crt_plan(npad, ka, kx)
    mods = plan["moduli"]
    assert mods == oracle.coprime_moduli(len(mods))
    g = torch.Generator(device="cuda").manual_seed(21)
    PA = torch.randint(-127, 128, (ka, npad, npad), dtype=torch.int8, device="cuda", generator=g)
    PX = torch.randint(-127, 128, (kx, npad, npad), dtype=torch.int8, device="cuda", generator=g)
    st, RA = rb.residue_planes(PA, ka, mods)
    assert st == 0
    st, RX = rb.residue_planes(PX, kx, mods)
    assert st == 0
    st, C = rb.residue_gemm(RX, RA, npad, mods)
    torch.cuda.synchronize()
    assert st == 0, rb.strerror(st)
    rng = np.random.default_rng(22)
    rows = np.sort(rng.choice(npad, 6, replace=False))
    cols = np.sort(rng.choice(npad, 6, replace=False))
    rows[0], cols[-1] = 0, npad - 1
    ridx, cidx = torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()
    dX = rb.kblocked_to_rows(PX)[:, ridx, :].cpu().numpy()      # (kx, 6, npad)
    dA = rb.kblocked_to_rows(PA)[:, cidx, :].cpu().numpy()      # (ka, 6, npad)
    # residue planes on the sampled rows (all npad entries) against the definition
    np.testing.assert_array_equal(rb.kblocked_to_rows(RX)[:, ridx, :].cpu().numpy(),
                                  oracle.digit_residues(dX, mods))
    np.testing.assert_array_equal(rb.kblocked_to_rows(RA)[:, cidx, :].cpu().numpy(),
                                  oracle.digit_residues(dA, mods))
    Cs = C[:, ridx][:, :, cidx].cpu().numpy()
    zX = [[_z(dX[:, a, k]) for k in range(npad)] for a in range(6)]
    zA = [[_z(dA[:, b, k]) for k in range(npad)] for b in range(6)]
    for a in range(6):
        for b in range(6):
            exact = sum(x * y for x, y in zip(zX[a], zA[b]))
            for q, m in enumerate(mods):
                assert int(Cs[q, a, b]) == _sym(exact, m), (a, b, q)
    del PA, PX, RA, RX, C
    torch.cuda.empty_cache()


@pytest.mark.parametrize("rows,cols,k,kT", [(100, 37, 7, 7), (300, 513, 8, 5),
                                            (1000, 1000, 9, 9), (257, 256, 3, 9)])
def test_split_transposed_planes_and_column_order(rows, cols, k, kT):
    """The splitter as the refinement runs it on X: columns read in a given working order,
    and the transposed operand planes of X^(1) (right operand of X^(1) E~)."""
    print(f"split_ex rows={rows} cols={cols} k={k} kT={kT}", flush=True)
    torch = _torch()
    rb = _rb()
    rng = np.random.default_rng(rows * 13 + cols + k)
    M = np.asfortranarray(rng.standard_normal((rows, cols)) * 2.0 ** rng.integers(-20, 20, (rows, cols)))
    M[:, 0] = 0.0
    cm = rng.permutation(cols).astype(np.int32)
    st, e, pl, tr, plT = rb.split_cols_ex(rb.colmajor(M), rows, cols, k, colmap=cm, kT=kT)
    torch.cuda.synchronize()
    assert st == 0, rb.strerror(st)
    Mp = np.asfortranarray(M[:, cm])
    e_o, pl_o, tr_o = oracle.split_s7(Mp, k)
    np.testing.assert_array_equal(e.cpu().numpy(), e_o)
    P = rb.kblocked_to_rows(pl).cpu().numpy()
    np.testing.assert_array_equal(P[:, :cols, :rows], pl_o)
    assert not P[:, cols:, :].any() and not P[:, :, rows:].any()
    np.testing.assert_array_equal(rb.from_colmajor(tr), tr_o)
    kk = max(k, kT)
    _, plT_o, _ = oracle.split_s7(Mp, kk)
    PT = rb.kblocked_to_rows(plT).cpu().numpy()                  # (kT, rows_pad, cols_pad)
    np.testing.assert_array_equal(PT[:, :rows, :cols], plT_o[:kT].transpose(0, 2, 1))
    assert not PT[:, rows:, :].any() and not PT[:, :, cols:].any()
    bad = cm.copy()
    bad[0] = cols
    assert rb.split_cols_ex(rb.colmajor(M), rows, cols, k, colmap=bad)[0] == rb.REFEIG_E_ARG
