"""GPU: extensions of columns made of edge values of the field, against the oracle element
by element. The butterflies' carry and borrow paths (sums that reach 2^64 or p, differences
that borrow, shift products of values near 2^64) are exercised by constant columns of
0, 1, p - 1, 2^32 - 1, 2^63 and p - 2^32, a column alternating 0 and p - 1, and columns
whose every element is drawn from those values (seeded); at 2^12 rows (one tile per pass)
and 2^18 rows (the 80 x 2^18 workload's transform sizes), both layouts, blowup 8, and then
committed (leaf digests and cap against the oracle's) at 2^12 rows."""
import numpy as np
import pytest

from paper_2603_03065_amd import inputs

pytestmark = pytest.mark.gpu
P = inputs.P
EDGES = [0, 1, P - 1, 2**32 - 1, 2**63, P - 2**32, P - 2]


@pytest.fixture(scope="module")
def v3db():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2603_03065_amd as m
    m.lib()
    return m


def _edge_columns(log_rows, n_mixed=3, seed=1234):
    n = 1 << log_rows
    cols = [np.full(n, v, dtype=np.uint64) for v in (0, 1, P - 1, 2**32 - 1, 2**63, P - 2**32)]
    alt = np.zeros(n, dtype=np.uint64)
    alt[1::2] = P - 1
    cols.append(alt)
    z = inputs.splitmix64(seed, np.arange(n_mixed * n, dtype=np.uint64)).reshape(n_mixed, n)
    ev = np.array(EDGES, dtype=np.uint64)
    for k in range(n_mixed):
        cols.append(ev[(z[k] % np.uint64(len(EDGES))).astype(np.int64)])
    return np.stack(cols)


@pytest.mark.parametrize("log_rows", [12, 18])
@pytest.mark.parametrize("layout", [0, 1], ids=["natural", "bitrev"])
def test_edge_value_columns_extend_like_the_oracle(v3db, oracle_mod, log_rows, layout):
    import torch
    oracle_mod.set_threads(0)
    tr = _edge_columns(log_rows)
    with v3db.Context(0) as ctx:
        out = ctx.lde(v3db.to_device(tr), 3, 7, layout)
        torch.cuda.synchronize()
        got = v3db.to_host(out)
    want = oracle_mod.lde(tr, 3, 7, layout)
    for c in range(tr.shape[0]):
        assert np.array_equal(got[c], want[c]), f"column {c} (first values {tr[c][:2]})"
    # a constant column extends to the same constant
    for c, v in enumerate((0, 1, P - 1, 2**32 - 1, 2**63, P - 2**32)):
        assert np.all(got[c] == np.uint64(v)), f"constant column {v}"


def test_edge_value_trace_commits_like_the_oracle(v3db, poseidon):
    import torch
    tr = _edge_columns(12)
    with v3db.Context(0) as ctx:
        N = 1 << 15
        job = v3db.Job(trace=v3db.to_device(tr), log_blowup=3, cap_height=3,
                       lde=torch.empty((tr.shape[0], N), dtype=torch.int64, device="cuda"),
                       tree=torch.empty((2 * N - 8, 4), dtype=torch.int64, device="cuda"))
        ctx.commit(job)
        torch.cuda.synchronize()
        cap, tree = v3db.to_host(job.cap), v3db.to_host(job.tree)
    ocap, _, otree = poseidon.commit(tr, 3, 7, 0, 3, want_tree=True)
    assert np.array_equal(tree, otree)
    assert np.array_equal(cap, ocap)
