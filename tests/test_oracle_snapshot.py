"""Oracle pins for the snapshot commitment (Sec. 4.3 "Snapshot Commitments"):
a transcription of the section's equations over the separately pinned sponge and
compression, and structural facts every correct implementation has — which inputs
each output depends on, the list and slot indices being absorbed, MerkleOpen of a
list's digest reaching the top-level root, and the one-list one-slot case."""
import numpy as np
import pytest

from paper_2603_03065_amd import inputs

P = inputs.P


def _mtree(poseidon, leaves):
    """MerkleTree over a list of 4-element digests (power-of-two count) to one root."""
    level = [np.asarray(x, dtype=np.uint64) for x in leaves]
    while len(level) > 1:
        level = [poseidon.compress_state(level[2 * k], level[2 * k + 1])[:4] for k in range(len(level) // 2)]
    return level[0]


def _by_definition(poseidon, log_lists, log_slots, m, dim, k, s):
    n_list, n = 1 << log_lists, 1 << log_slots
    N = n_list * n
    roots, hashes = [], []
    for i in range(n_list):
        leaves = []
        for j in range(n):
            t = i * n + j
            rec = [i, j, s["flag"][t], s["item"][t]] + [s["codes"][mm][t] for mm in range(m)]
            leaves.append(poseidon.sponge_state(np.array(rec, dtype=np.uint64))[:4])
        root_i = _mtree(poseidon, leaves)
        roots.append(root_i)
        seq = np.concatenate([np.array([i], dtype=np.uint64), s["centroids"][i], root_i])
        hashes.append(poseidon.sponge_state(seq)[:4])
    root_mk = _mtree(poseidon, hashes)
    root_cb = poseidon.sponge_state(s["codebooks"].reshape(-1))[:4]
    assert N == len(s["flag"])
    return root_mk, root_cb, np.array(roots), np.array(hashes)


def _commit(poseidon, shape, s):
    return poseidon.snapshot_commit(*shape, s["flag"], s["item"], s["codes"], s["centroids"], s["codebooks"])


@pytest.mark.parametrize("shape", [(0, 0, 1, 1, 1), (1, 2, 2, 4, 3), (2, 3, 8, 16, 4), (3, 1, 3, 9, 2)])
def test_snapshot_matches_the_equations(poseidon, shape):
    s = inputs.snapshot(31, *shape)
    got = _commit(poseidon, shape, s)
    want = _by_definition(poseidon, *shape, s)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)


def test_one_list_one_slot(poseidon):
    shape = (0, 0, 2, 2, 1)
    s = inputs.snapshot(32, *shape)
    mk, cb, roots, hashes = _commit(poseidon, shape, s)
    leaf = poseidon.sponge_state(np.array([0, 0, s["flag"][0], s["item"][0], s["codes"][0][0], s["codes"][1][0]],
                                          dtype=np.uint64))[:4]
    assert np.array_equal(roots[0], leaf)          # a one-leaf tree is its leaf
    assert np.array_equal(mk, hashes[0])


def test_dependencies_are_local(poseidon):
    shape = (2, 3, 4, 8, 4)
    s = inputs.snapshot(33, *shape)
    mk, cb, roots, hashes = _commit(poseidon, shape, s)
    n = 1 << shape[1]

    def changed(mutate):
        t = {k: v.copy() for k, v in s.items()}
        mutate(t)
        return _commit(poseidon, shape, t)

    def lists_differing(r2):
        return [i for i in range(len(roots)) if not np.array_equal(roots[i], r2[i])]

    # a record field of list 2: that list's root and hash, and the top root
    for field, pos in (("flag", 2 * n + 5), ("item", 2 * n + 1)):
        mk2, cb2, r2, h2 = changed(lambda t: t[field].__setitem__(pos, (int(t[field][pos]) + 1) % P))
        assert lists_differing(r2) == [2] and not np.array_equal(mk, mk2) and np.array_equal(cb, cb2)
    mk2, cb2, r2, h2 = changed(lambda t: t["codes"].__setitem__((3, 1 * n + 7), (int(t["codes"][3][n + 7]) + 1) % P))
    assert lists_differing(r2) == [1] and np.array_equal(cb, cb2)
    # slot order inside a list matters
    def swap(t):
        a, b = 3 * n + 0, 3 * n + 1
        for key in ("flag", "item"):
            t[key][[a, b]] = t[key][[b, a]]
        t["codes"][:, [a, b]] = t["codes"][:, [b, a]]
    mk2, _, r2, _ = changed(swap)
    assert lists_differing(r2) == [3] and not np.array_equal(mk, mk2)
    # a centroid coordinate: only that list's hash and the top root
    mk2, cb2, r2, h2 = changed(lambda t: t["centroids"].__setitem__((0, 7), (int(t["centroids"][0][7]) + 1) % P))
    assert lists_differing(r2) == [] and not np.array_equal(hashes[0], h2[0])
    assert all(np.array_equal(hashes[i], h2[i]) for i in range(1, len(hashes))) and not np.array_equal(mk, mk2)
    # a codebook coordinate: only the codebook digest
    mk2, cb2, r2, h2 = changed(lambda t: t["codebooks"].__setitem__((3, 3, 1), (int(t["codebooks"][3][3][1]) + 1) % P))
    assert np.array_equal(mk, mk2) and not np.array_equal(cb, cb2)


def test_indices_are_absorbed(poseidon):
    """Two lists with identical records and centroids still get different list roots
    and digests (i and j enter every hash)."""
    shape = (1, 2, 2, 2, 2)
    s = inputs.snapshot(34, *shape)
    n = 1 << shape[1]
    for key in ("flag", "item"):
        s[key][n:] = s[key][:n]
    s["codes"][:, n:] = s["codes"][:, :n]
    s["centroids"][1] = s["centroids"][0]
    mk, cb, roots, hashes = _commit(poseidon, shape, s)
    assert not np.array_equal(roots[0], roots[1]) and not np.array_equal(hashes[0], hashes[1])


def test_list_digest_opens_to_the_top_root(poseidon, oracle_mod):
    shape = (3, 2, 2, 4, 2)
    s = inputs.snapshot(35, *shape)
    mk, cb, roots, hashes = _commit(poseidon, shape, s)
    # the tree over the list digests, stored level by level, gives each list's path
    levels = [hashes]
    while len(levels[-1]) > 1:
        lv = levels[-1]
        levels.append(np.array([poseidon.compress_state(lv[2 * k], lv[2 * k + 1])[:4] for k in range(len(lv) // 2)]))
    tree = np.concatenate(levels)
    for i in range(1 << shape[0]):
        path = oracle_mod.merkle_path(tree, shape[0], 0, i)
        node, ci = poseidon.merkle_open(hashes[i], i, path)
        assert ci == 0 and np.array_equal(node, mk)


def test_invalid_arguments(poseidon):
    s = inputs.snapshot(36, 1, 1, 2, 4, 2)
    with pytest.raises(ValueError):
        poseidon.snapshot_commit(1, 1, 3, 4, 2, s["flag"], s["item"], s["codes"], s["centroids"], s["codebooks"])
