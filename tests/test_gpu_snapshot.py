"""GPU: the snapshot commitment (list roots, root_mk, root_cb) equals the oracle's,
bit for bit, on small shapes that span the kernels' special cases and on the
full SIFT1M zk-opt layout (1024 lists x 2048 slots, M = 8, D = 128, K = 256)."""
import numpy as np
import pytest

from paper_2603_03065_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def v3db():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2603_03065_amd as m
    m.lib()
    return m


def _run(v3db, poseidon, shape, seed):
    import torch
    s = inputs.snapshot(seed, *shape)
    d = {k: v3db.to_device(np.ascontiguousarray(v)) for k, v in s.items()}
    with v3db.Context(0) as ctx:
        mk, cb, roots = ctx.snapshot_commit(*shape, d["flag"], d["item"], d["codes"], d["centroids"], d["codebooks"])
        torch.cuda.synchronize()
        got = (v3db.to_host(mk), v3db.to_host(cb), v3db.to_host(roots))
    want = poseidon.snapshot_commit(*shape, s["flag"], s["item"], s["codes"], s["centroids"], s["codebooks"])
    return got, want


# (log_lists, log_slots, M, D, K): one list of one slot; one slot per list; one list;
# records of one permutation (M <= 4) and of two or more; centroid sequences shorter
# and longer than a permutation's rate; codebooks of one and of many permutations;
# list trees of 2^15 and 2^16 leaves (both Merkle kernels)
SHAPES = [(0, 0, 1, 1, 1), (3, 0, 2, 2, 3), (0, 5, 4, 8, 2), (2, 3, 8, 16, 4), (4, 2, 5, 5, 9),
          (5, 4, 12, 24, 16), (1, 16, 8, 32, 8), (7, 9, 8, 128, 256)]


@pytest.mark.parametrize("shape", SHAPES)
def test_snapshot_matches_oracle(v3db, poseidon, oracle_mod, shape):
    oracle_mod.set_threads(0)
    (mk, cb, roots), (omk, ocb, oroots, _) = _run(v3db, poseidon, shape, 40 + shape[0])
    assert np.array_equal(roots, oroots)
    assert np.array_equal(mk, omk)
    assert np.array_equal(cb, ocb)


def test_snapshot_sift1m_zkopt_full(v3db, poseidon, oracle_mod):
    """1024 lists x 2048 slots (N = 2^21 records), M = 8, D = 128, K = 256."""
    oracle_mod.set_threads(0)
    shape = (10, 11, 8, 128, 256)
    (mk, cb, roots), (omk, ocb, oroots, _) = _run(v3db, poseidon, shape, 50)
    assert np.array_equal(roots, oroots)
    assert np.array_equal(mk, omk)
    assert np.array_equal(cb, ocb)


def test_snapshot_rejects_bad_shapes(v3db):
    import torch
    z = torch.zeros(16, dtype=torch.int64, device="cuda")
    with v3db.Context(0) as ctx:
        with pytest.raises(v3db.V3dbError, match="multiple"):
            ctx.snapshot_commit(1, 1, 3, 4, 2, z, z, z, z, z)
        with pytest.raises(v3db.V3dbError, match="limits"):
            ctx.snapshot_commit(14, 13, 1, 1, 1, z, z, z, z, z)


def test_snapshot_gist1m_zkopt_full(v3db, poseidon, oracle_mod):
    """512 lists x 4096 slots (N = 2^21 records), M = 8, D = 960, K = 256: centroid
    sponges of 965 words and a codebook digest of 30 720 chained permutations."""
    oracle_mod.set_threads(0)
    shape = (9, 12, 8, 960, 256)
    (mk, cb, roots), (omk, ocb, oroots, _) = _run(v3db, poseidon, shape, 7)
    assert np.array_equal(roots, oroots)
    assert np.array_equal(mk, omk)
    assert np.array_equal(cb, ocb)
