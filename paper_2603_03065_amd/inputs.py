"""Seeded synthetic inputs, shared by the GPU path's tests/benchmarks and the oracle's.

This module holds no arithmetic of the method: it only draws uniform Goldilocks
field elements and workload shapes from a counter-based SplitMix64 stream, so the
same trace can be rebuilt anywhere from (seed, trace_id, col, row).

Element (seed, trace_id, col, row) = canon(SplitMix64(seed, (trace_id << 40) | (col << 24) | row)),
where SplitMix64(seed, i) is output i of the generator started at `seed` (the state
advances by 0x9E3779B97F4A7C15 before each output, then the published finaliser
mixes it) and canon(z) = z - p if z >= p else z.
"""
from __future__ import annotations

import numpy as np

P = 0xFFFFFFFF00000001
_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, idx) -> np.ndarray:
    """Vectorised SplitMix64 output idx (0-based) for a stream started at seed."""
    i = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (i + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def canon(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    return np.where(z >= np.uint64(P), z - np.uint64(P), z)


def trace(seed: int, trace_id: int, n_cols: int, log_rows: int, col0: int = 0) -> np.ndarray:
    """Column-major trace [n_cols][2^log_rows] of uniform field elements."""
    assert log_rows <= 24 and col0 + n_cols <= (1 << 16)
    rows = np.arange(1 << log_rows, dtype=np.uint64)
    out = np.empty((n_cols, 1 << log_rows), dtype=np.uint64)
    base = np.uint64(trace_id) << np.uint64(40)
    for c in range(n_cols):
        idx = base | (np.uint64(col0 + c) << np.uint64(24)) | rows
        out[c] = canon(splitmix64(seed, idx))
    return out


def states(seed: int, count: int) -> np.ndarray:
    """count random Poseidon states [count][12], uniform in [0, p)."""
    return canon(splitmix64(seed, np.arange(count * 12, dtype=np.uint64))).reshape(count, 12)


# ---- workload shapes ---------------------------------------------------------

BATCH_SHAPE_STREAM = 0x5634_0004


def batch_shapes(n_traces: int = 64, stream: int = BATCH_SHAPE_STREAM):
    """(log_rows, n_cols) per trace of the batched workload: log_rows uniform in
    10..18 and columns uniform in 20..135, drawn from a SplitMix64 stream."""
    out = []
    for t in range(n_traces):
        lr = 10 + int(splitmix64(stream, 2 * t)) % 9
        nc = 20 + int(splitmix64(stream, 2 * t + 1)) % 116
        out.append((lr, nc))
    return out


def uniform01(stream: int, i) -> np.ndarray:
    """Uniform doubles in [0, 1) from the top 53 bits of SplitMix64(stream, i)."""
    return (splitmix64(stream, i) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


# ---- IVF-PQ snapshots ----------------------------------------------------------

def _fixed_point(seed: int, kind: int, count: int) -> np.ndarray:
    """count signed 16-bit fixed-point coordinates in the field: magnitude uniform in
    [0, 2^16 - 1], negative values as p - |v| (the paper's encoding scales every
    coordinate into [-(2^16 - 1), 2^16 - 1])."""
    z = splitmix64(seed, (np.uint64(kind) << np.uint64(56)) | np.arange(count, dtype=np.uint64))
    mag = z & np.uint64(0xFFFF)
    neg = ((z >> np.uint64(16)) & np.uint64(1)).astype(bool) & (mag != 0)
    return np.where(neg, np.uint64(P) - mag, mag)


def snapshot(seed: int, log_lists: int, log_slots: int, m: int, dim: int, k: int):
    """A synthetic fixed-shape IVF-PQ snapshot: n_list = 2^log_lists lists of
    n = 2^log_slots slots, each list holding count_i valid records (uniform in
    [3n/4, n], the rest padding), M PQ codes per record, D-dimensional centroids
    and M x K codebooks of D/M coordinates.
    Returns dict(flag [N], item [N], codes [M][N], centroids [n_list][D],
    codebooks [M][K][D/M]) with records in list-major order (t = i * n + j)."""
    n_list, n = 1 << log_lists, 1 << log_slots
    N = n_list * n
    cnt = splitmix64(seed, (np.uint64(1) << np.uint64(56)) | np.arange(n_list, dtype=np.uint64))
    counts = n - (cnt % np.uint64(n // 4 + 1)).astype(np.int64)
    j = np.tile(np.arange(n, dtype=np.int64), n_list)
    valid = j < np.repeat(counts, n)
    flag = valid.astype(np.uint64)
    rid = splitmix64(seed, (np.uint64(2) << np.uint64(56)) | np.arange(N, dtype=np.uint64)) >> np.uint64(24)
    item = np.where(valid, rid + np.uint64(1), np.uint64(0))
    z = splitmix64(seed, (np.uint64(3) << np.uint64(56)) | np.arange(m * N, dtype=np.uint64)).reshape(m, N)
    codes = np.where(valid[None, :], z % np.uint64(k), np.uint64(0))
    centroids = _fixed_point(seed, 4, n_list * dim).reshape(n_list, dim)
    codebooks = _fixed_point(seed, 5, k * dim).reshape(m, k, dim // m)
    return {"flag": flag, "item": item, "codes": codes, "centroids": centroids, "codebooks": codebooks}


# ---- serving workload -----------------------------------------------------------

SERVE_ARRIVAL_STREAM = 0x5634_0005   # exponential inter-arrival gaps
SERVE_BIG_STREAM = 0x5634_0105       # u' < 0.05: an 80 x 2^18 request (cap height 4)
SERVE_SHAPE_STREAM = 0x5634_0205     # otherwise the batch workload's shape distribution
SERVE_SAMPLE_STREAM = 0x5634_0305    # the seeded 2 % sample of requests checked against stored caps
SERVE_TRACE_SEED = 5                 # request i's trace is trace(5, i, n_cols, log_rows)
SERVE_BIG_SHAPE = (18, 80, 4)        # (log_rows, n_cols, cap_height)


def serve_requests(seconds: float = 120.0, rate: float = 50.0):
    """Seeded open-loop arrivals: list of (t_arrive_s, log_rows, n_cols, cap_height)
    for request index i = 0, 1, ... Gaps are -ln(1 - u) / rate with u from
    SERVE_ARRIVAL_STREAM; a request is 80 cols x 2^18 rows with cap height 4 when
    u' < 0.05 (SERVE_BIG_STREAM), otherwise log rows 10 + (z mod 9) and columns
    20 + (z' mod 116) with cap height 2 (SERVE_SHAPE_STREAM, outputs 2i and 2i + 1)."""
    import math
    out, t, i = [], 0.0, 0
    while True:
        u = float(uniform01(SERVE_ARRIVAL_STREAM, i))
        t += -math.log(1.0 - u) / rate
        if t >= seconds:
            return out
        if float(uniform01(SERVE_BIG_STREAM, i)) < 0.05:
            L, C, h = SERVE_BIG_SHAPE
        else:
            L = 10 + int(splitmix64(SERVE_SHAPE_STREAM, 2 * i)) % 9
            C = 20 + int(splitmix64(SERVE_SHAPE_STREAM, 2 * i + 1)) % 116
            h = 2
        out.append((t, L, C, h))
        i += 1


def serve_checked(requests):
    """Indices of the requests whose caps are stored as expected values: a seeded 2 %
    sample (u < 0.02 on SERVE_SAMPLE_STREAM) and every 80 x 2^18 request."""
    return [i for i, (_, L, C, h) in enumerate(requests)
            if float(uniform01(SERVE_SAMPLE_STREAM, i)) < 0.02 or (L, C, h) == SERVE_BIG_SHAPE]


# ---- the same traces drawn on a torch device ---------------------------------------

def trace_torch(seed: int, trace_id: int, n_cols: int, log_rows: int, device="cuda", col0: int = 0):
    """trace() drawn with torch int64 operations on `device` (same values, as the raw
    bits of an int64 tensor [n_cols][2^log_rows]): for workloads too large to draw on
    the host in time. int64 multiplication wraps modulo 2^64 like uint64, right shifts
    are made logical by masking, and z >= p (as unsigned) is z in [p - 2^64, 0) as signed."""
    import torch
    assert log_rows <= 24 and col0 + n_cols <= (1 << 16)

    def s64(x: int) -> int:
        return x - (1 << 64) if x >= 1 << 63 else x

    def srl(z, k: int):
        return (z >> k) & ((1 << (64 - k)) - 1)

    rows = torch.arange(1 << log_rows, dtype=torch.int64, device=device)
    cols = torch.arange(col0, col0 + n_cols, dtype=torch.int64, device=device)
    idx = (trace_id << 40) | (cols[:, None] << 24) | rows[None, :]
    z = (idx + 1) * s64(0x9E3779B97F4A7C15) + s64(seed & ((1 << 64) - 1))
    z = (z ^ srl(z, 30)) * s64(0xBF58476D1CE4E5B9)
    z = (z ^ srl(z, 27)) * s64(0x94D049BB133111EB)
    z = z ^ srl(z, 31)
    big = (z < 0) & (z >= s64(P))
    return torch.where(big, z - s64(P), z)
