"""Pins for the oracle's field arithmetic and NTT against Python integers, closed
forms and the textbook DFT definition (CPU only)."""
import os
import random

import numpy as np
import pytest

from _bigint import P, dft, root

EDGE = [0, 1, 2, P - 1, P - 2, 2**32, 2**32 - 1, 2**63, 2**64 - 2**32, 12345678901234567]


def test_field_ops_edge_and_random(oracle_mod):
    o = oracle_mod
    rnd = random.Random(1)
    vals = EDGE + [rnd.randrange(P) for _ in range(300)]
    for a in vals:
        for b in (vals[:10] + [rnd.randrange(P) for _ in range(3)]):
            assert o.add(a, b) == (a + b) % P
            assert o.sub(a, b) == (a - b) % P
            assert o.mul(a, b) == (a * b) % P
    for a in vals[1:40]:
        if a % P:
            assert o.mul(a, o.inv(a)) == 1


def test_closed_form_facts(oracle_mod):
    o = oracle_mod
    # 2^64 = 2^32 - 1 and 2^96 = -1 mod p
    assert o.pow_(2, 64) == 2**32 - 1
    assert o.pow_(2, 96) == P - 1
    # p - 1 = 2^32 * 3 * 5 * 17 * 257 * 65537 and 7 generates F_p^*
    assert (P - 1) == 2**32 * 3 * 5 * 17 * 257 * 65537
    for q in (2, 3, 5, 17, 257, 65537):
        assert o.pow_(7, (P - 1) // q) != 1
    # w_{2^k} has order exactly 2^k
    for k in (1, 2, 3, 6, 12, 18, 21, 23, 32):
        w = o.root_of_unity(k)
        assert w == pow(7, (P - 1) >> k, P)
        assert o.pow_(w, 1 << k) == 1
        assert o.pow_(w, 1 << (k - 1)) == P - 1
    # small roots are powers of two: w_64 = 2^39, w_8 = 2^120, w_4 = 2^48, w_2 = 2^96
    assert o.root_of_unity(6) == pow(2, 39, P)
    assert o.root_of_unity(3) == pow(2, 120, P)
    assert o.root_of_unity(2) == pow(2, 48, P)


def test_splitmix64_published_vector(oracle_mod):
    path = os.path.join(os.path.dirname(__file__), "golden", "splitmix64.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    for seed, idx, val in rows:
        assert oracle_mod.splitmix64(int(seed), int(idx)) == int(val, 16)


def test_input_generator_uses_same_stream(oracle_mod):
    from paper_2603_03065_amd import inputs
    path = os.path.join(os.path.dirname(__file__), "golden", "splitmix64.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    for seed, idx, val in rows:
        assert int(inputs.splitmix64(int(seed), int(idx))) == int(val, 16)
    t = inputs.trace(7, 3, 2, 4)
    for c in range(2):
        for r in range(16):
            z = oracle_mod.splitmix64(7, (3 << 40) | (c << 24) | r)
            assert int(t[c, r]) == (z - P if z >= P else z)


@pytest.mark.parametrize("log_n", [0, 1, 2, 3, 5, 7])
def test_ntt_matches_direct_dft(oracle_mod, log_n):
    rnd = random.Random(log_n)
    x = [rnd.randrange(P) for _ in range(1 << log_n)]
    assert [int(v) for v in oracle_mod.ntt(x)] == dft(x)
    assert [int(v) for v in oracle_mod.ntt(x, inverse=True)] == dft(x, inverse=True)


@pytest.mark.parametrize("log_n", [1, 4, 10, 13])
def test_ntt_round_trip(oracle_mod, log_n):
    rng = np.random.default_rng(log_n)
    x = rng.integers(0, P, size=1 << log_n, dtype=np.uint64)
    y = oracle_mod.ntt(oracle_mod.ntt(x), inverse=True)
    assert np.array_equal(x, y)


@pytest.mark.parametrize("log_n", [3, 5])
def test_ntt_convolution_theorem(oracle_mod, log_n):
    n = 1 << log_n
    rnd = random.Random(99 + log_n)
    a = [rnd.randrange(P) for _ in range(n)]
    b = [rnd.randrange(P) for _ in range(n)]
    conv = [sum(a[j] * b[(k - j) % n] for j in range(n)) % P for k in range(n)]
    fa, fb = oracle_mod.ntt(a), oracle_mod.ntt(b)
    assert [int(v) for v in oracle_mod.ntt(conv)] == [int(x) * int(y) % P for x, y in zip(fa, fb)]


def test_ntt_linearity(oracle_mod):
    rnd = random.Random(5)
    n = 256
    a = [rnd.randrange(P) for _ in range(n)]
    b = [rnd.randrange(P) for _ in range(n)]
    alpha = rnd.randrange(P)
    lhs = oracle_mod.ntt([(x + alpha * y) % P for x, y in zip(a, b)])
    fa, fb = oracle_mod.ntt(a), oracle_mod.ntt(b)
    assert [int(v) for v in lhs] == [(int(x) + alpha * int(y)) % P for x, y in zip(fa, fb)]


def test_root_is_the_omega_of_the_ntt(oracle_mod):
    # X = NTT(delta_1) gives X[k] = w^k for the root the transform uses
    n = 16
    x = [0] * n
    x[1] = 1
    w = root(4)
    assert [int(v) for v in oracle_mod.ntt(x)] == [pow(w, k, P) for k in range(n)]
