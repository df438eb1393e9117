"""The serving scheduler's policy on the host, with the simulated executor (no
GPU): admission in arrival order by HBM budget, continuous batching over slots,
failure isolation, queue limits, latency stamps."""
import time

import numpy as np
import pytest


@pytest.fixture(scope="module")
def v3db():
    import paper_2603_03065_amd as m
    m.lib()
    return m


def _footprint(C, L, b=3, h=2):
    g = lambda x: (x + (2 << 20) - 1) // (2 << 20) * (2 << 20)       # arena granularity
    n, N = 1 << L, 1 << (L + b)
    return g(C * n * 8) + g(C * N * 8) + g((2 * N - (1 << h)) * 32) + g((1 << h) * 32) + g(C * n * 8)


def _trace(C, L):
    return np.zeros((C, 1 << L), dtype=np.uint64)


def test_all_complete_with_ordered_stamps(v3db):
    with v3db.Server(None, slots=3, hbm_budget=8 << 30, sim_ns_per_element=0.5) as srv:
        keep = [_trace(20, 12) for _ in range(30)]
        tickets = [srv.submit(t, cap_height=2) for t in keep]
        srv.drain()
        res = [srv.poll(t) for t in tickets]
        assert all(r is not None and r[0] == 0 for r in res)
        for _, cap, tm in res:
            assert tm["t_arrive"] <= tm["t_admit"] <= tm["t_done"]
            assert cap.shape == (4, 4)
        st = srv.stats()
        assert st["completed"] == 30 and st["failed"] == 0 and st["hbm_in_use"] == 0


def test_budget_is_never_exceeded_and_fifo(v3db):
    big = _footprint(80, 14)
    budget = int(2.5 * big)                       # at most two big requests admitted at once
    with v3db.Server(None, slots=4, hbm_budget=budget, sim_ns_per_element=2.0) as srv:
        keep = [_trace(80, 14) for _ in range(10)]
        tickets = [srv.submit(t) for t in keep]
        srv.drain()
        res = [srv.poll(t) for t in tickets]
        st = srv.stats()
        assert st["hbm_peak"] <= budget and st["pool_bytes"] <= budget + (2 << 20)
        assert st["hbm_peak"] >= big
        admits = [r[2]["t_admit"] for r in res]
        assert admits == sorted(admits)            # arrival order
        assert max(r[2]["batch_size"] for r in res) <= 2


def test_continuous_batching_admits_late_arrivals(v3db):
    # a long request occupies slot 0; requests that arrive later are batched on free slots
    with v3db.Server(None, slots=2, hbm_budget=16 << 30, sim_ns_per_element=20.0) as srv:
        keep = [_trace(40, 14)] + [_trace(8, 10) for _ in range(12)]
        t0 = srv.submit(keep[0])
        time.sleep(0.002)
        rest = [srv.submit(t) for t in keep[1:]]
        srv.drain()
        first = srv.poll(t0)
        others = [srv.poll(t) for t in rest]
        assert first[2]["slot"] == 0
        assert all(o[2]["t_admit"] < first[2]["t_done"] for o in others[:1])   # admitted while slot 0 ran
        assert max(o[2]["batch_size"] for o in others) > 1


def test_failure_is_isolated(v3db):
    with v3db.Server(None, slots=2, hbm_budget=8 << 30, sim_ns_per_element=0.5) as srv:
        keep = [_trace(16, 11) for _ in range(9)]
        tickets = [srv.submit(t, flags=v3db.REQ_FAIL_INJECT if i == 4 else 0) for i, t in enumerate(keep)]
        srv.drain()
        res = [srv.poll(t) for t in tickets]
        assert res[4][0] == 5                      # DEVICE
        assert all(r[0] == 0 for i, r in enumerate(res) if i != 4)
        st = srv.stats()
        assert st["failed"] == 1 and st["completed"] == 9 and st["hbm_in_use"] == 0


def test_rejections(v3db):
    with v3db.Server(None, slots=1, hbm_budget=64 << 20, max_queue=2, sim_ns_per_element=1e4) as srv:
        with pytest.raises(v3db.V3dbError) as e:
            srv.submit(_trace(80, 16))             # alone bigger than the budget
        assert e.value.name == "OUT_OF_MEMORY"
        with pytest.raises(v3db.V3dbError) as e:
            srv.submit(_trace(4, 8), shift=0)
        assert e.value.name == "INVALID_ARG"
        keep = [_trace(4, 12) for _ in range(8)]
        ok, busy = 0, 0
        for t in keep:
            try:
                srv.submit(t)
                ok += 1
            except v3db.V3dbError as ex:
                assert ex.name == "BUSY"
                busy += 1
        assert busy > 0
        srv.drain()


def test_latency_counts_from_arrival_stamp(v3db):
    with v3db.Server(None, slots=1, hbm_budget=8 << 30, sim_ns_per_element=0.1) as srv:
        t = _trace(8, 10)
        stamp = v3db.clock() - 0.5                   # arrived half a second before submission
        tk = srv.submit(t, t_arrive=stamp)
        srv.drain()
        st, cap, tm = srv.poll(tk)
        assert tm["t_arrive"] == stamp and tm["t_done"] - tm["t_arrive"] >= 0.5
