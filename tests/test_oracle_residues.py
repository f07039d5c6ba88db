"""Pins of the oracle's residue definitions (the Chinese-remainder form of the exact
product of Sec. 2.3): Python integers decide, on inputs small enough to enumerate."""
import numpy as np
import pytest

import oracle


def test_coprime_moduli_by_hand():
    # 255 = 3*5*17, 253 = 11*23, 251 prime, 249 = 3*83 (shares 3), 247 = 13*19,
    # 245 = 5*7^2 (shares 5), 243 = 3^5, 241, 239 prime, 237 = 3*79, 235 = 5*47, 233 prime,
    # 231 = 3*7*11, 229, 227 prime, 225 = 15^2, 223 prime, 221 = 13*17, 219 = 3*73,
    # 217 = 7*31
    assert oracle.coprime_moduli(11) == [255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 217]
    from math import gcd, prod
    m = oracle.coprime_moduli(28)
    assert len(m) == 28 and all(x % 2 == 1 and 3 <= x <= 255 for x in m)
    assert all(gcd(a, b) == 1 for i, a in enumerate(m) for b in m[i + 1:])
    assert m == sorted(m, reverse=True)
    assert prod(m).bit_length() > 200


def _z(digits):
    """sum_t d_t 128^(k-1-t) as a Python integer."""
    z = 0
    for d in digits:
        z = z * 128 + int(d)
    return z


def _sym(z, m):
    r = z % m
    return r - m if r > m // 2 else r


@pytest.mark.parametrize("k", [1, 2, 7, 8, 16, 18])
def test_digit_residues_against_integers(k):
    rng = np.random.default_rng(100 + k)
    P = rng.integers(-127, 128, (k, 5, 7)).astype(np.int8)
    P[:, 0, 0] = 127
    P[:, 0, 1] = -127                       # the extreme integers
    P[:, 0, 2] = 0
    mods = oracle.coprime_moduli(28)
    R = oracle.digit_residues(P, mods)
    assert R.shape == (28, 5, 7) and R.dtype == np.int8
    for i in range(5):
        for j in range(7):
            z = _z(P[:, i, j])
            for q, m in enumerate(mods):
                assert int(R[q, i, j]) == _sym(z, m)
                assert abs(int(R[q, i, j])) <= (m - 1) // 2


def test_residue_product_is_the_exact_product_mod_m():
    """Residues of the digit integers, multiplied mod m, equal the exact integer product of
    the integers mod m (the identity the residue form of V rests on)."""
    rng = np.random.default_rng(7)
    ka, kx, K = 5, 3, 11
    PA = rng.integers(-127, 128, (ka, 4, K)).astype(np.int8)    # 4 rows, K entries each
    PX = rng.integers(-127, 128, (kx, 6, K)).astype(np.int8)    # 6 rows
    mods = oracle.coprime_moduli(9)
    C = oracle.residue_product(oracle.digit_residues(PA, mods), oracle.digit_residues(PX, mods),
                               mods)
    for i in range(4):
        for j in range(6):
            exact = sum(_z(PA[:, i, k]) * _z(PX[:, j, k]) for k in range(K))
            for q, m in enumerate(mods):
                assert int(C[q, i, j]) == _sym(exact, m)
    # and the moduli reconstruct it: |P| < M / 2 here, so the CRT value is P itself
    from math import prod
    M = prod(mods)
    exact = sum(_z(PA[:, 0, k]) * _z(PX[:, 0, k]) for k in range(K))
    assert abs(exact) < M // 2
    x = 0
    for q, m in enumerate(mods):
        Mq = M // m
        x += int(C[q, 0, 0]) * Mq * pow(Mq, -1, m)
    x %= M
    assert (x - M if x > M // 2 else x) == exact


def test_residue_product_transposition_matters():
    """A transposed operand would give another answer: the pin sees operand roles."""
    rng = np.random.default_rng(3)
    L = rng.integers(-60, 61, (1, 3, 3)).astype(np.int8)
    R = rng.integers(-60, 61, (1, 3, 3)).astype(np.int8)
    C = oracle.residue_product(L, R, [251])
    Ct = oracle.residue_product(L, np.ascontiguousarray(R.transpose(0, 2, 1)), [251])
    assert not np.array_equal(C, Ct)
