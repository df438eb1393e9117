"""GPU: the batched commit path (phase launches over many traces, captured as a
HIP graph) gives exactly the caps, trees and LDEs of committing each trace alone,
and those match the oracle."""
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


@pytest.fixture()
def ctx(v3db):
    c = v3db.Context(0)
    yield c
    c.close()


def _host(v3db, t):
    import torch
    torch.cuda.synchronize()
    return v3db.to_host(t)


def _jobs(v3db, trs, h=2, layout=0, with_buffers=False, b=3):
    import torch
    jobs = []
    for tr in trs:
        C, n = tr.shape
        N = n << b
        j = v3db.Job(trace=v3db.to_device(tr), log_blowup=b, cap_height=min(h, (n << b).bit_length() - 1),
                     layout=layout)
        if with_buffers:
            j.lde = torch.empty((C, N), dtype=torch.int64, device="cuda")
            j.tree = torch.empty((2 * N - (1 << j.cap_height), 4), dtype=torch.int64, device="cuda")
        jobs.append(j)
    return jobs


def _small_mix(n_traces, max_log_rows=11, seed_stream=inputs.BATCH_SHAPE_STREAM):
    shapes = [(min(lr, max_log_rows), nc) for lr, nc in inputs.batch_shapes(n_traces, seed_stream)]
    return [inputs.trace(4, t, nc, lr) for t, (lr, nc) in enumerate(shapes)]


def test_batched_equals_oracle_with_buffers(v3db, ctx, poseidon):
    trs = _small_mix(7, max_log_rows=9) + [inputs.trace(4, 99, 1, 0), inputs.trace(4, 98, 3, 1)]
    jobs = _jobs(v3db, trs, h=2, with_buffers=True)
    ctx.commit_batch(jobs)
    for tr, j in zip(trs, jobs):
        cap, lde, tree = poseidon.commit(tr, 3, 7, 0, j.cap_height, want_lde=True, want_tree=True)
        assert np.array_equal(_host(v3db, j.lde), lde)
        assert np.array_equal(_host(v3db, j.tree), tree)
        assert np.array_equal(_host(v3db, j.cap), cap)


def test_batched_equals_per_trace(v3db, ctx):
    trs = _small_mix(24, max_log_rows=12)
    batched = [_host(v3db, c) for c in ctx.commit_batch(_jobs(v3db, trs))]
    ctx.set_batching(False)
    single = [_host(v3db, c) for c in ctx.commit_batch(_jobs(v3db, trs))]
    for a, b in zip(batched, single):
        assert np.array_equal(a, b)


def test_mixed_layouts_and_cap_heights(v3db, ctx, poseidon):
    trs = _small_mix(4, max_log_rows=8)
    jobs = _jobs(v3db, trs[:2], h=0) + _jobs(v3db, trs[2:3], h=2, layout=1) + _jobs(v3db, trs[3:], h=64)
    ctx.commit_batch(jobs)
    for tr, j in zip(trs, jobs):
        assert np.array_equal(_host(v3db, j.cap), poseidon.commit(tr, 3, 7, j.layout, j.cap_height)[0])


def test_graph_replay_with_new_data(v3db, ctx, poseidon):
    shapes = [(6, 9), (8, 20), (5, 1)]
    for rep in range(3):
        trs = [inputs.trace(40 + rep, t, nc, lr) for t, (lr, nc) in enumerate(shapes)]
        jobs = _jobs(v3db, trs, h=1)
        ctx.commit_batch(jobs)
        for tr, j in zip(trs, jobs):
            assert np.array_equal(_host(v3db, j.cap), poseidon.commit(tr, 3, 7, 0, 1)[0])


def test_graph_cache_eviction(v3db, ctx, poseidon):
    """Ten distinct lists of two traces (a batch needs two natural-layout jobs), each
    committed three times in an interleaved order: a list's first call runs without a
    graph, its second captures one, its third replays it; with more lists than the 8
    graphs kept, earlier graphs are evicted while later ones are in use, and the first
    list comes back at the end. Every cap against the oracle."""
    lists = [[(3 + k % 5, 2 + k), (4 + k % 3, 3)] for k in range(10)]
    order = [k for r in range(3) for k in range(10)] + [0, 0]
    for step, k in enumerate(order):
        trs = [inputs.trace(50 + step, t, nc, lr) for t, (lr, nc) in enumerate(lists[k])]
        jobs = _jobs(v3db, trs, h=0)
        ctx.commit_batch(jobs)
        for tr, j in zip(trs, jobs):
            assert np.array_equal(_host(v3db, j.cap), poseidon.commit(tr, 3, 7, 0, 0)[0]), f"call {step}, list {k}"


def test_small_group_cap_splits_batch(v3db, ctx):
    trs = _small_mix(10, max_log_rows=10)
    ref = [_host(v3db, c) for c in ctx.commit_batch(_jobs(v3db, trs))]
    ctx.set_batch_group_bytes(1 << 20)     # every job in a group of its own or few
    got = [_host(v3db, c) for c in ctx.commit_batch(_jobs(v3db, trs))]
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


def test_other_blowups_batched(v3db, ctx, poseidon):
    for b in (0, 1, 2, 4):
        trs = [inputs.trace(60 + b, t, 5 + t, 4 + t) for t in range(3)]
        jobs = _jobs(v3db, trs, h=1, b=b, with_buffers=True)
        ctx.commit_batch(jobs)
        for tr, j in zip(trs, jobs):
            cap, lde, _ = poseidon.commit(tr, b, 7, 0, j.cap_height, want_lde=True)
            assert np.array_equal(_host(v3db, j.lde), lde)
            assert np.array_equal(_host(v3db, j.cap), cap)


def test_batch_of_64_mixed_traces_workload(v3db, ctx, poseidon):
    """The batch workload: 64 traces, log rows uniform in 10..18, columns uniform in
    20..135, blowup 8, cap height 2. Every batched cap equals the same trace
    committed alone; the smallest traces are also checked against the oracle."""
    import torch
    shapes = inputs.batch_shapes(64)
    trs = [inputs.trace(4, t, nc, lr) for t, (lr, nc) in enumerate(shapes)]
    jobs = _jobs(v3db, trs, h=2)
    caps = [_host(v3db, c) for c in ctx.commit_batch(jobs)]
    del jobs
    torch.cuda.empty_cache()
    ctx.set_batching(False)
    for t in range(64):
        j = _jobs(v3db, [trs[t]], h=2)[0]
        ctx.commit(j)
        assert np.array_equal(caps[t], _host(v3db, j.cap)), f"trace {t} shape {shapes[t]}"
    smallest = sorted(range(64), key=lambda t: (shapes[t][0], shapes[t][1]))[:3]
    for t in smallest:
        assert np.array_equal(caps[t], poseidon.commit(trs[t], 3, 7, 0, 2)[0]), f"trace {t} shape {shapes[t]}"
