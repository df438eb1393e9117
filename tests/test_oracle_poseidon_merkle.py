"""Pins for the oracle's Poseidon permutation, sponge, compression and Merkle
tree: S-box invertibility, the MDS property of the derived matrix (with the
minor counter itself pinned by closed-form counts), round trips through an
independently written inverse permutation, and MerkleOpen path recomputation."""
import math
import random

import numpy as np
import pytest

from _bigint import D_INV7, P, InversePoseidon, det

TOTAL_SQUARE_SUBMATRICES = math.comb(24, 12) - 1      # 2 704 155 for a 12 x 12 matrix


def test_sbox_is_a_bijection(oracle_mod):
    assert math.gcd(7, P - 1) == 1
    assert D_INV7 == 10540996611094048183
    rnd = random.Random(2)
    for x in [0, 1, P - 1, 2**32] + [rnd.randrange(P) for _ in range(200)]:
        assert oracle_mod.pow_(oracle_mod.pow_(x, 7), D_INV7) == x


def test_minor_counter_closed_forms(oracle_mod):
    # identity: a submatrix (R, C) is nonsingular iff R == C, so 2^12 - 1 are nonsingular
    ident = np.eye(12, dtype=np.uint64)
    assert oracle_mod.singular_minor_count(ident) == TOTAL_SQUARE_SUBMATRICES - (2**12 - 1)
    # all-ones: only the 144 1x1 minors are nonsingular
    ones = np.ones((12, 12), dtype=np.uint64)
    assert oracle_mod.singular_minor_count(ones) == TOTAL_SQUARE_SUBMATRICES - 144


def test_det12_matches_gaussian_elimination(oracle_mod):
    rnd = random.Random(11)
    for _ in range(3):
        m = [[rnd.randrange(P) for _ in range(12)] for _ in range(12)]
        assert oracle_mod.det12(np.array(m, dtype=np.uint64)) == det(m)
    m = [[rnd.randrange(256) for _ in range(12)] for _ in range(12)]
    m[5] = list(m[2])                                      # two equal rows
    assert oracle_mod.det12(np.array(m, dtype=np.uint64)) == 0 == det(m)


def test_minor_counter_finds_a_planted_singular_2x2(oracle_mod):
    # circulant with a_0 = 2, a_1 = 4, a_11 = 1: rows 0,1 x cols 0,1 = [[2,4],[1,2]], det 0
    circ = [2, 4, 3, 5, 7, 11, 13, 17, 19, 23, 29, 1]
    m = np.array([[circ[(j - i) % 12] for j in range(12)] for i in range(12)], dtype=np.uint64)
    assert oracle_mod.singular_minor_count(m) >= 1


def test_derived_constants_are_well_formed(poseidon):
    rc, circ, mds = poseidon.rc, poseidon.circ, poseidon.mds
    assert rc.shape == (30, 12) and np.all(rc < np.uint64(P))
    assert len(set(int(v) for v in rc.ravel())) == 360
    assert np.all((circ >= 1) & (circ <= 255))
    for i in range(12):
        for j in range(12):
            assert mds[i, j] == circ[(j - i) % 12]
    assert poseidon.mds_attempts >= 1


def test_derived_mds_is_mds(oracle_mod, poseidon):
    # every square submatrix of the derived matrix is nonsingular over F_p
    assert oracle_mod.singular_minor_count(poseidon.mds) == 0
    assert oracle_mod.det12(poseidon.mds) == det([[int(v) for v in r] for r in poseidon.mds]) != 0


def test_round_constants_follow_the_stream(oracle_mod, poseidon):
    # accepted SplitMix64 outputs (z < p) in order fill rc round-major
    vals, i = [], 0
    while len(vals) < 360:
        z = oracle_mod.splitmix64(poseidon.seed, i)
        i += 1
        if z < P:
            vals.append(z)
    assert [int(v) for v in poseidon.rc.ravel()] == vals


def test_permutation_round_trips_through_independent_inverse(poseidon):
    inv = InversePoseidon(poseidon.rc, poseidon.mds)
    rnd = random.Random(4)
    states = [[0] * 12, [P - 1] * 12, list(range(12))] + [[rnd.randrange(P) for _ in range(12)] for _ in range(40)]
    out = poseidon.permute(np.array(states, dtype=np.uint64))
    for s, o in zip(states, out):
        assert inv([int(v) for v in o]) == s


def test_permutation_is_not_trivial(poseidon):
    out = poseidon.permute(np.zeros((2, 12), dtype=np.uint64))
    assert not np.array_equal(out[0], np.zeros(12, dtype=np.uint64))
    one = np.zeros((1, 12), dtype=np.uint64)
    one[0, 11] = 1
    assert not np.array_equal(poseidon.permute(one)[0], out[0])


@pytest.mark.parametrize("length", [1, 4, 7, 8, 9, 12, 16, 17, 20, 135])
def test_sponge_structure_via_inverse(poseidon, length):
    """Undo the last permutation of the sponge: lanes 0..k-1 must hold the last
    chunk (k elements) and the other lanes the state after the previous chunks;
    for the first chunk that previous state is zero (overwrite absorption, zero
    IV, elements in column order). Run over lengths, this checks every step."""
    inv = InversePoseidon(poseidon.rc, poseidon.mds)
    rnd = random.Random(length)
    row = [rnd.randrange(P) for _ in range(length)]
    final = [int(v) for v in poseidon.sponge_state(np.array(row, dtype=np.uint64))]
    q_last = 8 * ((length - 1) // 8)
    last = row[q_last:]
    before = inv(final)
    assert before[:len(last)] == last
    prev = [int(v) for v in poseidon.sponge_state(np.array(row[:q_last], dtype=np.uint64))]
    assert before[len(last):] == prev[len(last):]
    if q_last == 0:
        assert prev == [0] * 12


def test_sponge_empty_row_is_zero_state(poseidon):
    assert np.all(poseidon.sponge_state(np.zeros(0, dtype=np.uint64)) == 0)


def test_compress_via_inverse(poseidon):
    inv = InversePoseidon(poseidon.rc, poseidon.mds)
    rnd = random.Random(8)
    l = [rnd.randrange(P) for _ in range(4)]
    r = [rnd.randrange(P) for _ in range(4)]
    st = poseidon.compress_state(np.array(l, dtype=np.uint64), np.array(r, dtype=np.uint64))
    assert inv([int(v) for v in st]) == l + r + [0, 0, 0, 0]


def test_leaf_digest_is_sponge_of_stored_row(poseidon):
    rng = np.random.default_rng(5)
    mat = rng.integers(0, P, size=(11, 32), dtype=np.uint64)
    dig = poseidon.leaf_digests(mat)
    for k in (0, 5, 31):
        assert np.array_equal(dig[k], poseidon.sponge_state(mat[:, k])[:4])


@pytest.mark.parametrize("log_leaves", range(1, 9))
def test_merkle_open_every_leaf(oracle_mod, poseidon, log_leaves):
    rng = np.random.default_rng(log_leaves)
    n_cols = 3 + log_leaves
    mat = rng.integers(0, P, size=(n_cols, 1 << log_leaves), dtype=np.uint64)
    for h in sorted({0, min(2, log_leaves), log_leaves}):
        cap, tree = poseidon.merkle_commit(mat, h, want_tree=True)
        leaves = tree[: 1 << log_leaves]
        assert np.array_equal(leaves, poseidon.leaf_digests(mat))
        for i in range(1 << log_leaves):
            path = oracle_mod.merkle_path(tree, log_leaves, h, i)
            node, ci = poseidon.merkle_open(leaves[i], i, path)
            assert np.array_equal(node, cap[ci])
        if h == log_leaves:
            assert np.array_equal(cap, leaves)


def test_cap_consistency(poseidon):
    """The cap-0 root equals the root of the cap-h nodes folded pairwise."""
    rng = np.random.default_rng(9)
    mat = rng.integers(0, P, size=(9, 64), dtype=np.uint64)
    root = poseidon.merkle_commit(mat, 0)
    for h in (1, 2, 3, 6):
        level = [row for row in poseidon.merkle_commit(mat, h)]
        while len(level) > 1:
            level = [poseidon.compress_state(level[2 * k], level[2 * k + 1])[:4] for k in range(len(level) // 2)]
        assert np.array_equal(level[0], root[0])


def test_commit_equals_lde_then_merkle(oracle_mod, poseidon):
    rng = np.random.default_rng(12)
    tr = rng.integers(0, P, size=(10, 32), dtype=np.uint64)
    cap, lde, tree = poseidon.commit(tr, 3, 7, oracle_mod.BITREV, 2, want_lde=True, want_tree=True)
    assert np.array_equal(lde, oracle_mod.lde(tr, 3, 7, oracle_mod.BITREV))
    assert np.array_equal(cap, poseidon.merkle_commit(lde, 2))
