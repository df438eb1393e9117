"""GPU parity at full workload sizes, in the launch configuration the benchmark
times (one job through v3db_commit_batch with caller-provided LDE and tree).

The oracle cannot hash 2^21..2^23 rows in a test, so it checks what it can
compute one by one: whole LDE columns, LDE rows at sampled indices (Horner
evaluation of the oracle's interpolants at the row's coset point, every column),
the leaf digest of each sampled row (oracle sponge over that row), sampled
Merkle nodes at every level (oracle compression of the stored children), the
top levels in full, and the cap (the stored level at the cap height)."""
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


def _bitrev(k, bits):
    return int(format(k, f"0{bits}b")[::-1], 2)


def _run_fullsize(v3db, oracle_mod, poseidon, C, L, h, layout, seed, cols_full, n_rows_sampled, rng_seed):
    import torch
    b = 3
    logN = L + b
    N = 1 << logN
    tr = inputs.trace(seed, 0, C, L)
    with v3db.Context(0) as ctx:
        job = v3db.Job(trace=v3db.to_device(tr), log_blowup=b, cap_height=h, shift=7, layout=layout,
                       lde=torch.empty((C, N), dtype=torch.int64, device="cuda"),
                       tree=torch.empty((2 * N - (1 << h), 4), dtype=torch.int64, device="cuda"))
        ctx.commit(job)
        torch.cuda.synchronize()
        cap = v3db.to_host(job.cap)
        tree = v3db.to_host(job.tree)
        lde_cols = {c: v3db.to_host(job.lde[c]) for c in cols_full}
        rng = np.random.default_rng(rng_seed)
        rows = sorted(set([0, N - 1] + [int(x) for x in rng.integers(0, N, n_rows_sampled)]))
        lde_rows = {k: v3db.to_host(job.lde[:, k].contiguous()) for k in rows}
        del job
        torch.cuda.empty_cache()

    # whole columns against the oracle's LDE
    for c in cols_full:
        assert np.array_equal(lde_cols[c], oracle_mod.lde(tr[c:c + 1], b, 7, layout)[0]), f"column {c}"
    # sampled rows: every column's interpolant at the row's coset point
    coeffs = oracle_mod.interpolate(tr)
    wN = oracle_mod.root_of_unity(logN)
    pts = [7 * pow(wN, _bitrev(k, logN) if layout else k, P) % P for k in rows]
    vals = oracle_mod.eval_columns(coeffs, pts)
    leaves = tree[:N]
    for i, k in enumerate(rows):
        assert np.array_equal(lde_rows[k], vals[:, i]), f"LDE row {k}"
        assert np.array_equal(leaves[k], poseidon.sponge_state(vals[:, i])[:4]), f"leaf {k}"
    # tree: sampled nodes of every level, the top levels in full, the cap
    off, cnt = 0, N
    lvl = logN
    rng = np.random.default_rng(rng_seed + 1)
    while lvl > h:
        above = cnt // 2
        idx = range(above) if above <= 1024 else sorted(set(int(x) for x in rng.integers(0, above, 64)))
        for k in idx:
            want = poseidon.compress_state(tree[off + 2 * k], tree[off + 2 * k + 1])[:4]
            assert np.array_equal(tree[off + cnt + k], want), f"level {lvl - 1} node {k}"
        off += cnt
        cnt = above
        lvl -= 1
    assert np.array_equal(cap, tree[off:off + cnt])


def test_fullsize_80x2p18_natural_cap4(v3db, oracle_mod, poseidon):
    oracle_mod.set_threads(0)
    _run_fullsize(v3db, oracle_mod, poseidon, C=80, L=18, h=4, layout=0, seed=2, cols_full=[0, 37, 79],
                  n_rows_sampled=6, rng_seed=20)


def test_fullsize_135x2p20_bitrev_cap4(v3db, oracle_mod, poseidon):
    oracle_mod.set_threads(0)
    _run_fullsize(v3db, oracle_mod, poseidon, C=135, L=20, h=4, layout=1, seed=3, cols_full=[134],
                  n_rows_sampled=3, rng_seed=30)


def _run_sampled_only(v3db, oracle_mod, poseidon, C, L, b, h, layout, seed, n_rows_sampled, rng_seed):
    """Largest extensions the library accepts (2^26 rows): sampled rows, leaves and nodes only."""
    import torch
    logN = L + b
    N = 1 << logN
    tr = inputs.trace(seed, 0, C, L)
    with v3db.Context(0) as ctx:
        job = v3db.Job(trace=v3db.to_device(tr), log_blowup=b, cap_height=h, shift=7, layout=layout,
                       lde=torch.empty((C, N), dtype=torch.int64, device="cuda"),
                       tree=torch.empty((2 * N - (1 << h), 4), dtype=torch.int64, device="cuda"))
        ctx.commit(job)
        torch.cuda.synchronize()
        rng = np.random.default_rng(rng_seed)
        rows = sorted(set([0, 1, N - 1] + [int(x) for x in rng.integers(0, N, n_rows_sampled)]))
        lde_rows = {k: v3db.to_host(job.lde[:, k].contiguous()) for k in rows}
        leaves = {k: v3db.to_host(job.tree[k]) for k in rows}
        total = 2 * N - (1 << h)                  # digests in the tree
        lvl_h = total - (1 << h)                  # offset of the cap level
        lvl_h1 = lvl_h - (1 << (h + 1))           # offset of the level below it
        top = v3db.to_host(job.tree[lvl_h:total])
        below = v3db.to_host(job.tree[lvl_h1:lvl_h])
        cap = v3db.to_host(job.cap)
        del job
        torch.cuda.empty_cache()
    coeffs = oracle_mod.interpolate(tr)
    wN = oracle_mod.root_of_unity(logN)
    pts = [7 * pow(wN, _bitrev(k, logN) if layout else k, P) % P for k in rows]
    vals = oracle_mod.eval_columns(coeffs, pts)
    for i, k in enumerate(rows):
        assert np.array_equal(lde_rows[k], vals[:, i]), f"LDE row {k}"
        assert np.array_equal(leaves[k], poseidon.sponge_state(vals[:, i])[:4]), f"leaf {k}"
    # the cap is the level above its children, folded pairwise
    assert np.array_equal(cap, top)
    for k in range(1 << h):
        assert np.array_equal(cap[k], poseidon.compress_state(below[2 * k], below[2 * k + 1])[:4])


@pytest.mark.parametrize("C,L,b,h,layout", [(2, 23, 3, 1, 0), (1, 24, 2, 0, 1)])
def test_max_extension_2p26_rows(v3db, oracle_mod, poseidon, C, L, b, h, layout):
    oracle_mod.set_threads(0)
    _run_sampled_only(v3db, oracle_mod, poseidon, C, L, b, h, layout, seed=7, n_rows_sampled=3, rng_seed=L)
