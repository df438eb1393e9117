"""The seeded input generators: the torch form of the trace generator draws the same
values as the numpy form (on the CPU here; the GPU tests compare it on the device)."""
import numpy as np
import pytest

from paper_2603_03065_amd import inputs


@pytest.mark.parametrize("seed,trace_id,n_cols,log_rows", [(5, 0, 3, 10), (5, 5850, 80, 12), (3, 0, 7, 8),
                                                         (4, 63, 20, 11), (0xFFFFFFFFFFFFFFFF, 1, 2, 9)])
def test_trace_torch_equals_trace(seed, trace_id, n_cols, log_rows):
    a = inputs.trace(seed, trace_id, n_cols, log_rows)
    b = inputs.trace_torch(seed, trace_id, n_cols, log_rows, device="cpu").numpy().view(np.uint64)
    assert np.array_equal(a, b)
    assert int(a.max()) < inputs.P


def test_canon_boundary_values():
    z = np.array([0, inputs.P - 1, inputs.P, inputs.P + 1, 2**64 - 1], dtype=np.uint64)
    assert inputs.canon(z).tolist() == [0, inputs.P - 1, 0, 1, 2**32 - 2]


def test_serve_sample_holds_every_big_request():
    reqs = inputs.serve_requests(120.0, 50.0)
    chk = set(inputs.serve_checked(reqs))
    big = [i for i, r in enumerate(reqs) if r[1:] == inputs.SERVE_BIG_SHAPE]
    assert set(big) <= chk and 250 < len(big) < 350
    small = chk - set(big)
    assert 60 < len(small) < 180          # about 2 % of about 6000
