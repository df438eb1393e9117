"""GPU: the allocation-free Merkle commitment (v3db_merkle_commit_noalloc, tree levels in
the library's static device scratch) gives the cap v3db_merkle_commit gives with its
pooled scratch, on two calls in a row on one context (the second with fewer leaves,
fewer columns and another cap height), and the oracle's cap; sizes beyond the static
scratch are refused."""
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


def test_noalloc_commit_matches_pooled_commit(v3db, poseidon):
    import torch
    with v3db.Context(0) as ctx:
        # 2^20 leaves, cap height 0: the largest tree the static scratch holds
        for (C, L, h, seed) in [(24, 20, 0, 71), (9, 13, 3, 72)]:
            mat = inputs.trace_torch(seed, 0, C, L, device="cuda")
            want = ctx.merkle_commit(mat, h)
            got = torch.full((1 << h, 4), -1, dtype=torch.int64, device="cuda")
            ctx.merkle_commit_noalloc(mat, h, got)
            torch.cuda.synchronize()
            assert np.array_equal(v3db.to_host(got), v3db.to_host(want)), f"{C} x 2^{L}, cap {h}"
            if L <= 13:
                ocap = poseidon.merkle_commit(v3db.to_host(mat), h)
                assert np.array_equal(v3db.to_host(got), ocap)


def test_noalloc_commit_refuses_trees_beyond_its_scratch(v3db):
    import torch
    with v3db.Context(0) as ctx:
        mat = torch.zeros((1, 1 << 21), dtype=torch.int64, device="cuda")
        cap = torch.zeros((1, 4), dtype=torch.int64, device="cuda")
        with pytest.raises(v3db.V3dbError, match="static scratch"):
            ctx.merkle_commit_noalloc(mat, 0, cap)
        with pytest.raises(v3db.V3dbError, match="cap_height"):
            ctx.merkle_commit_noalloc(mat[:, :8], 4, torch.zeros((16, 4), dtype=torch.int64, device="cuda"))
