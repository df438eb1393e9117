"""Oracle pins for the multiset-equality grand product (Sec. 4.5 "Gadgets and Cost
Model": Compress(x; beta) = sum x_i beta^i and SetEq by prod (alpha - x_i)):
Python big-integer evaluation of the polynomial and the product on small tables,
the SetEq property (a row permutation leaves the total unchanged, a changed
element changes it), roots (alpha equal to a compressed row zeroes every later
running product), beta = 0 and width 1 reducing to the plain product."""
import numpy as np
import pytest

from paper_2603_03065_amd import inputs

P = inputs.P


def _table(seed, width, n):
    return inputs.canon(inputs.splitmix64(seed, np.arange(width * n, dtype=np.uint64))).reshape(width, n)


def test_against_big_integer_definition(oracle_mod):
    width, n = 5, 37
    x = _table(1, width, n)
    alpha, beta = 0x1234_5678_9ABC_DEF0 % P, 0xFEDC_BA98_7654_3210 % P
    z, total = oracle_mod.grand_product(x, alpha, beta)
    acc = 1
    for i in range(n):
        c = sum(int(x[k][i]) * pow(beta, k, P) for k in range(width)) % P   # the polynomial, not Horner
        acc = acc * ((alpha - c) % P) % P
        assert int(z[i]) == acc
    assert total == acc


def test_set_equality_property(oracle_mod):
    width, n = 3, 257
    x = _table(2, width, n)
    alpha, beta = 987654321987654321 % P, 123456789123456789 % P
    _, t0 = oracle_mod.grand_product(x, alpha, beta, want_z=False)
    perm = np.random.default_rng(3).permutation(n)
    _, t1 = oracle_mod.grand_product(np.ascontiguousarray(x[:, perm]), alpha, beta, want_z=False)
    assert t0 == t1
    y = x.copy()
    y[1, 100] = (int(y[1, 100]) + 1) % P
    _, t2 = oracle_mod.grand_product(y, alpha, beta, want_z=False)
    assert t2 != t0
    # swapping two coordinates inside a row is a different tuple
    z = x.copy()
    z[0, 7], z[1, 7] = x[1, 7], x[0, 7]
    _, t3 = oracle_mod.grand_product(z, alpha, beta, want_z=False)
    assert t3 != t0 or x[0, 7] == x[1, 7]


def test_alpha_at_a_compressed_row_zeroes_the_tail(oracle_mod):
    width, n = 2, 20
    x = _table(4, width, n)
    beta = 5
    alpha = (int(x[0][9]) + int(x[1][9]) * beta) % P
    z, total = oracle_mod.grand_product(x, alpha, beta)
    assert all(int(v) != 0 for v in z[:9]) and all(int(v) == 0 for v in z[9:]) and total == 0


def test_beta_zero_and_width_one(oracle_mod):
    n = 50
    x = _table(5, 3, n)
    alpha = 77
    _, t_beta0 = oracle_mod.grand_product(x, alpha, 0, want_z=False)
    _, t_first = oracle_mod.grand_product(np.ascontiguousarray(x[:1]), alpha, 12345, want_z=False)
    acc = 1
    for i in range(n):
        acc = acc * ((alpha - int(x[0][i])) % P) % P
    assert t_beta0 == acc == t_first


def test_empty_and_invalid(oracle_mod):
    z, total = oracle_mod.grand_product(np.zeros((2, 0), dtype=np.uint64), 3, 4)
    assert total == 1 and z.size == 0
    with pytest.raises(ValueError):
        oracle_mod.grand_product(np.zeros((0, 4), dtype=np.uint64), 3, 4)
