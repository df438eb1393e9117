"""Pins for the oracle's coset low-degree extension: closed forms by Horner
evaluation and special cases (CPU only)."""
import random

import numpy as np
import pytest

from _bigint import P, horner, root


def _bitrev(x, bits):
    return int(format(x, f"0{bits}b")[::-1], 2) if bits else 0


def _trace_from_poly(coeffs_per_col, log_rows):
    n = 1 << log_rows
    w = root(log_rows)
    return np.array([[horner(cf, pow(w, i, P)) for i in range(n)] for cf in coeffs_per_col], dtype=np.uint64)


@pytest.mark.parametrize("log_rows,log_blowup,shift", [(0, 3, 7), (1, 3, 7), (4, 3, 7), (5, 3, 11), (3, 2, 7), (4, 0, 7), (6, 1, 3)])
def test_lde_closed_form_all_points(oracle_mod, log_rows, log_blowup, shift):
    rnd = random.Random(log_rows * 31 + log_blowup)
    n = 1 << log_rows
    coeffs = [[rnd.randrange(P) for _ in range(n)] for _ in range(3)]
    trace = _trace_from_poly(coeffs, log_rows)
    out = oracle_mod.lde(trace, log_blowup, shift)
    N = n << log_blowup
    wN = root(log_rows + log_blowup)
    for c in range(3):
        expect = [horner(coeffs[c], shift * pow(wN, k, P) % P) for k in range(N)]
        assert [int(v) for v in out[c]] == expect


def test_lde_closed_form_sampled_large(oracle_mod):
    rnd = random.Random(7)
    log_rows, log_blowup, shift = 10, 3, 7
    n = 1 << log_rows
    coeffs = [rnd.randrange(P) for _ in range(n)]
    trace = _trace_from_poly([coeffs], log_rows)
    out = oracle_mod.lde(trace, log_blowup, shift)
    wN = root(log_rows + log_blowup)
    for k in [0, 1, 2, 7, 8, 1023, 4097, (n << log_blowup) - 1] + [rnd.randrange(n << log_blowup) for _ in range(20)]:
        assert int(out[0, k]) == horner(coeffs, shift * pow(wN, k, P) % P)


def test_lde_unit_shift_reproduces_trace(oracle_mod):
    rng = np.random.default_rng(3)
    tr = rng.integers(0, P, size=(4, 256), dtype=np.uint64)
    out = oracle_mod.lde(tr, 3, 1)
    assert np.array_equal(out[:, ::8], tr)


def test_lde_constant_and_identity_columns(oracle_mod):
    log_rows, lb, s = 6, 3, 7
    n = 1 << log_rows
    w = root(log_rows)
    wN = root(log_rows + lb)
    const = np.full((1, n), 123456789, dtype=np.uint64)
    assert np.all(oracle_mod.lde(const, lb, s) == 123456789)
    ident = np.array([[pow(w, i, P) for i in range(n)]], dtype=np.uint64)   # P(x) = x
    out = oracle_mod.lde(ident, lb, s)
    assert [int(v) for v in out[0]] == [s * pow(wN, k, P) % P for k in range(n << lb)]


@pytest.mark.parametrize("log_rows,log_blowup", [(0, 3), (3, 3), (7, 3), (5, 1)])
def test_lde_bitrev_is_permutation_of_natural(oracle_mod, log_rows, log_blowup):
    rng = np.random.default_rng(log_rows)
    tr = rng.integers(0, P, size=(3, 1 << log_rows), dtype=np.uint64)
    nat = oracle_mod.lde(tr, log_blowup, 7, oracle_mod.NATURAL)
    rev = oracle_mod.lde(tr, log_blowup, 7, oracle_mod.BITREV)
    bits = log_rows + log_blowup
    perm = [_bitrev(k, bits) for k in range(1 << bits)]
    assert np.array_equal(rev, nat[:, perm])


def test_lde_rejects_invalid(oracle_mod):
    tr = np.zeros((1, 4), dtype=np.uint64)
    with pytest.raises(ValueError):
        oracle_mod.lde(tr, 3, 0)
    with pytest.raises(ValueError):
        oracle_mod.lde(tr, 3, P)


def test_eval_columns_matches_horner(oracle_mod):
    rnd = random.Random(21)
    cf = [[rnd.randrange(P) for _ in range(37)] for _ in range(3)]
    xs = [0, 1, P - 1, rnd.randrange(P), rnd.randrange(P)]
    out = oracle_mod.eval_columns(np.array(cf, dtype=np.uint64), xs)
    for c in range(3):
        assert [int(v) for v in out[c]] == [horner(cf[c], x) for x in xs]


def test_interpolate_then_eval_reproduces_lde(oracle_mod):
    rng = np.random.default_rng(22)
    tr = rng.integers(0, P, size=(2, 64), dtype=np.uint64)
    lde = oracle_mod.lde(tr, 3, 7)
    cf = oracle_mod.interpolate(tr)
    wN = root(9)
    ks = [0, 3, 100, 511]
    got = oracle_mod.eval_columns(cf, [7 * pow(wN, k, P) % P for k in ks])
    assert np.array_equal(got, lde[:, ks])
