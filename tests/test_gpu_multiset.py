"""GPU: the multiset-equality grand product (running products of alpha minus the
compressed rows) equals the oracle's, element by element, across tile and scan
boundaries, and at 2^24 rows in the launch configuration the benchmark times."""
import numpy as np
import pytest

from paper_2603_03065_amd import inputs

pytestmark = pytest.mark.gpu
P = inputs.P


@pytest.fixture(scope="module")
def v3db():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2603_03065_amd as m
    m.lib()
    return m


def _table(seed, width, n):
    return inputs.canon(inputs.splitmix64(seed, np.arange(width * n, dtype=np.uint64))).reshape(width, n)


# sizes around one tile (4096 rows), several tiles with a ragged tail, and more
# tiles than the partial scan has threads (1024)
@pytest.mark.parametrize("width,n", [(1, 1), (3, 7), (4, 4095), (4, 4096), (2, 4097), (5, 100_003),
                                     (1, 4096 * 1024 + 5), (8, 1 << 16)])
def test_grand_product_matches_oracle(v3db, oracle_mod, width, n):
    import torch
    x = _table(60 + width, width, n)
    alpha, beta = int(inputs.splitmix64(61, n)) % P, int(inputs.splitmix64(62, n)) % P
    with v3db.Context(0) as ctx:
        z, total = ctx.grand_product(v3db.to_device(x), alpha, beta)
        _, total_only = ctx.grand_product(v3db.to_device(x), alpha, beta, want_z=False)
        torch.cuda.synchronize()
        z, total, total_only = v3db.to_host(z), int(v3db.to_host(total)[0]), int(v3db.to_host(total_only)[0])
    oz, ot = oracle_mod.grand_product(x, alpha, beta)
    assert np.array_equal(z, oz)
    assert total == ot == total_only


def test_grand_product_set_equality_and_edge_cases(v3db, oracle_mod):
    import torch
    width, n = 3, 9000
    x = _table(70, width, n)
    alpha, beta = 1234567, 7654321
    perm = np.random.default_rng(71).permutation(n)
    with v3db.Context(0) as ctx:
        _, t0 = ctx.grand_product(v3db.to_device(x), alpha, beta, want_z=False)
        _, t1 = ctx.grand_product(v3db.to_device(np.ascontiguousarray(x[:, perm])), alpha, beta, want_z=False)
        # alpha equal to a compressed row: zero from that row on
        a0 = (int(x[0][5000]) + int(x[1][5000]) * beta + int(x[2][5000]) * beta * beta) % P
        z, tz = ctx.grand_product(v3db.to_device(x), a0, beta)
        # no rows
        _, te = ctx.grand_product(torch.empty((2, 0), dtype=torch.int64, device="cuda"), 5, 6)
        torch.cuda.synchronize()
        t0, t1 = int(v3db.to_host(t0)[0]), int(v3db.to_host(t1)[0])
        z, tz, te = v3db.to_host(z), int(v3db.to_host(tz)[0]), int(v3db.to_host(te)[0])
    assert t0 == t1 == oracle_mod.grand_product(x, alpha, beta, want_z=False)[1]
    assert (z[:5000] != 0).all() and (z[5000:] == 0).all() and tz == 0
    assert te == 1


def test_grand_product_fullsize_2p24(v3db, oracle_mod):
    """2^24 rows of 4-element tuples: every running product against the oracle."""
    import torch
    width, n = 4, 1 << 24
    x = _table(80, width, n)
    alpha, beta = int(inputs.splitmix64(81, 0)) % P, int(inputs.splitmix64(82, 0)) % P
    with v3db.Context(0) as ctx:
        z, total = ctx.grand_product(v3db.to_device(x), alpha, beta)
        torch.cuda.synchronize()
        z, total = v3db.to_host(z), int(v3db.to_host(total)[0])
    oz, ot = oracle_mod.grand_product(x, alpha, beta)
    assert np.array_equal(z, oz) and total == ot
