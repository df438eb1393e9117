"""GPU: requests served through the continuous-batching server (several slots,
batches of mixed shapes overlapping on the device) give exactly the cap each
trace gets when committed alone, and the oracle's cap."""
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


def test_served_equals_alone_and_oracle(v3db, poseidon):
    import torch
    rng_shapes = [(6 + (k * 5) % 6, 3 + (k * 7) % 38) for k in range(40)] + [(13, 80), (12, 135)]
    traces = [inputs.trace(5, k, C, L) for k, (L, C) in enumerate(rng_shapes)]
    pinned = [torch.from_numpy(t.view(np.int64)).pin_memory() for t in traces]
    with v3db.Context(0) as ctx:
        with v3db.Server(ctx, slots=3, hbm_budget=2 << 30, max_batch=8) as srv:
            tickets = [srv.submit(p, cap_height=2 if L + 3 >= 2 else 0) for p, (L, C) in zip(pinned, rng_shapes)]
            srv.drain()
            res = [srv.poll(t) for t in tickets]
            stats = srv.stats()
        assert all(r[0] == 0 for r in res)
        assert stats["hbm_peak"] <= 2 << 30 and stats["hbm_in_use"] == 0
        assert max(r[2]["batch_size"] for r in res) > 1
        assert len({r[2]["slot"] for r in res}) > 1
        for k, (tr, r) in enumerate(zip(traces, res)):
            job = v3db.Job(trace=v3db.to_device(tr), log_blowup=3, cap_height=2)
            ctx.commit(job)
            torch.cuda.synchronize()
            assert np.array_equal(r[1], v3db.to_host(job.cap)), f"request {k}"
        for k in range(0, 40, 7):
            assert np.array_equal(res[k][1], poseidon.commit(traces[k], 3, 7, 0, 2)[0]), f"request {k}"


def test_server_isolates_an_injected_failure(v3db):
    import torch
    traces = [inputs.trace(6, k, 9, 8) for k in range(6)]
    with v3db.Context(0) as ctx:
        with v3db.Server(ctx, slots=2, hbm_budget=1 << 30) as srv:
            tickets = [srv.submit(t, flags=v3db.REQ_FAIL_INJECT if k == 2 else 0) for k, t in enumerate(traces)]
            srv.drain()
            res = [srv.poll(t) for t in tickets]
        assert res[2][0] == 5 and all(r[0] == 0 for k, r in enumerate(res) if k != 2)
        for k in (0, 5):
            job = v3db.Job(trace=v3db.to_device(traces[k]), log_blowup=3, cap_height=2)
            ctx.commit(job)
            torch.cuda.synchronize()
            assert np.array_equal(res[k][1], v3db.to_host(job.cap))
