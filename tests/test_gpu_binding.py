"""GPU: the binding refuses caller-supplied buffers that are too small, of the wrong
dtype or not contiguous before anything reaches the library (which writes through raw
pointers), and nothing it refuses leaves work behind: the next call on the same
context gives the oracle's result."""
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


def test_short_or_malformed_buffers_are_refused(v3db, poseidon):
    import torch
    tr = inputs.trace(70, 0, 3, 6)
    d = v3db.to_device(tr)
    N = 64 << 3
    with v3db.Context(0) as ctx:
        with pytest.raises(ValueError, match="out"):
            ctx.lde(d, 3, out=torch.empty((3, N - 1), dtype=torch.int64, device="cuda"))
        with pytest.raises(ValueError, match="expected a contiguous int64"):
            ctx.lde(d, 3, out=torch.empty((3, N), dtype=torch.int32, device="cuda"))
        with pytest.raises(ValueError, match="expected a contiguous int64"):
            ctx.lde(d, 3, out=torch.empty((N, 3), dtype=torch.int64, device="cuda").t())
        mat = ctx.lde(d, 3)
        with pytest.raises(ValueError, match="tree"):
            ctx.merkle_commit(mat, 2, tree=torch.empty((2 * N - 5, 4), dtype=torch.int64, device="cuda"))
        with pytest.raises(ValueError, match="cap"):
            ctx.merkle_commit(mat, 2, cap=torch.empty((3, 4), dtype=torch.int64, device="cuda"))
        job = v3db.Job(trace=d, log_blowup=3, cap_height=1,
                       lde=torch.empty((3, N // 2), dtype=torch.int64, device="cuda"))
        with pytest.raises(ValueError, match="job 0 lde"):
            ctx.commit(job)
        with pytest.raises(ValueError, match="states"):
            ctx.poseidon_permute(torch.empty((5,), dtype=torch.int32, device="cuda"))
        # the context is intact
        job = v3db.Job(trace=d, log_blowup=3, cap_height=1)
        ctx.commit(job)
        torch.cuda.synchronize()
        assert np.array_equal(v3db.to_host(job.cap), poseidon.commit(tr, 3, 7, 0, 1)[0])
