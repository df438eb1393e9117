"""GPU: the FRI commit phase (pair-leaf trees and caps of every round, arity-2
folds) equals the oracle's, word for word, over shapes that span one-block and
many-block folds, cap heights from 0 to the last round's limit, and a 2^22-point
codeword; the 2^21-point extension of the headline commitment is folded too."""
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


def _run(v3db, poseidon, f0, shift, betas, h):
    import torch
    with v3db.Context(0) as ctx:
        folded, caps, trees = ctx.fri_commit(v3db.to_device(f0), shift, betas, h, want_trees=True)
        _, caps2, _ = ctx.fri_commit(v3db.to_device(f0), shift, betas, h)   # trees in scratch
        torch.cuda.synchronize()
        got = (v3db.to_host(folded), v3db.to_host(caps), v3db.to_host(trees), v3db.to_host(caps2))
    want = poseidon.fri_commit(f0, shift, betas, h, want_trees=True)
    return got, want


@pytest.mark.parametrize("log_n,rounds,h,shift", [(1, 1, 0, 7), (5, 3, 2, 7), (8, 8, 0, 3), (11, 6, 4, 7),
                                                   (16, 10, 6, 5), (20, 12, 8, 7)])
def test_fri_commit_matches_oracle(v3db, poseidon, oracle_mod, log_n, rounds, h, shift):
    oracle_mod.set_threads(0)
    f0 = inputs.canon(inputs.splitmix64(100 + log_n, np.arange(1 << log_n, dtype=np.uint64)))
    betas = [int(b) % P for b in inputs.splitmix64(101, np.arange(rounds, dtype=np.uint64))]
    (folded, caps, trees, caps2), (ofolded, ocaps, otrees) = _run(v3db, poseidon, f0, shift, betas, h)
    assert np.array_equal(folded, ofolded)
    assert np.array_equal(trees, otrees)
    assert np.array_equal(caps, ocaps) and np.array_equal(caps2, ocaps)


def test_fri_commit_2p22(v3db, poseidon, oracle_mod):
    oracle_mod.set_threads(0)
    log_n, rounds, h = 22, 16, 4
    f0 = inputs.canon(inputs.splitmix64(110, np.arange(1 << log_n, dtype=np.uint64)))
    betas = [int(b) % P for b in inputs.splitmix64(111, np.arange(rounds, dtype=np.uint64))]
    (folded, caps, trees, caps2), (ofolded, ocaps, otrees) = _run(v3db, poseidon, f0, 7, betas, h)
    assert np.array_equal(folded, ofolded) and np.array_equal(caps, ocaps) and np.array_equal(trees, otrees)


def test_fri_over_the_committed_extension(v3db, poseidon, oracle_mod):
    """Folding a column of the headline commitment's extension (80 x 2^18 -> 2^21,
    shift 7): the codeword is low-degree (rate 1/8), so after 18 rounds the last
    codeword of 8 values is constant (degree < 1), and every fold matches the oracle."""
    import torch
    tr = inputs.trace(2, 0, 1, 18)
    with v3db.Context(0) as ctx:
        lde = ctx.lde(v3db.to_device(tr), 3, 7, 0)
        betas = [int(b) % P for b in inputs.splitmix64(120, np.arange(18, dtype=np.uint64))]
        folded, caps, _ = ctx.fri_commit(lde[0].contiguous(), 7, betas, 2)
        torch.cuda.synchronize()
        folded, caps, f0 = v3db.to_host(folded), v3db.to_host(caps), v3db.to_host(lde[0])
    last = folded[-8:]
    assert (last == last[0]).all()
    ofolded, ocaps, _ = poseidon.fri_commit(f0, 7, betas, 2)
    assert np.array_equal(folded, ofolded) and np.array_equal(caps, ocaps)


def test_fri_rejects_bad_arguments(v3db):
    import torch
    f = torch.zeros(16, dtype=torch.int64, device="cuda")
    with v3db.Context(0) as ctx:
        with pytest.raises(v3db.V3dbError, match="rounds"):
            ctx.fri_commit(f, 7, [1, 2, 3], 2)
        with pytest.raises(v3db.V3dbError, match="shift"):
            ctx.fri_commit(f, P, [1], 0)


def test_fri_calls_of_different_sizes_on_one_context(v3db, poseidon, oracle_mod):
    """Back-to-back calls on one context whose round tables differ in size (the batched
    trees' job table grows, then is reused for a smaller call), the middle one on
    another stream: every call equals the oracle."""
    import torch
    oracle_mod.set_threads(0)
    shapes = [(9, 3, 2), (14, 10, 3), (7, 2, 1)]   # (log_n, rounds, cap height)
    side = torch.cuda.Stream()
    with v3db.Context(0) as ctx:
        outs = []
        for k, (log_n, rounds, h) in enumerate(shapes):
            f0 = inputs.canon(inputs.splitmix64(130 + k, np.arange(1 << log_n, dtype=np.uint64)))
            betas = [int(b) % P for b in inputs.splitmix64(140 + k, np.arange(rounds, dtype=np.uint64))]
            stream = side if k == 1 else None
            d = v3db.to_device(f0)
            if stream is not None:
                stream.wait_stream(torch.cuda.current_stream())
                # the codeword is read on the side stream: its block must not be handed
                # to the next call's upload (on the default stream) before that work ends
                d.record_stream(stream)
            folded, caps, trees = ctx.fri_commit(d, 7, betas, h, want_trees=True, stream=stream)
            outs.append((f0, betas, h, folded, caps, trees, d))
        torch.cuda.synchronize()
        for f0, betas, h, folded, caps, trees, _ in outs:
            ofolded, ocaps, otrees = poseidon.fri_commit(f0, 7, betas, h, want_trees=True)
            assert np.array_equal(v3db.to_host(folded), ofolded)
            assert np.array_equal(v3db.to_host(caps), ocaps)
            assert np.array_equal(v3db.to_host(trees), otrees)
