"""Python binding for libv3db (trace commitment on MI355X / gfx950).

Thin argument marshalling over the C ABI in include/v3db.h: every step of the
commitment runs in the library's HIP kernels. PyTorch supplies device memory
and streams only: field elements live in int64 tensors used as raw 64-bit words
(values >= 2^63 appear negative in torch and are the same bits), passed to the
library as data pointers, with the current torch stream as the HIP stream.

If libv3db.so has not been built, or was built from other sources than the tree
holds, this module raises on first use; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libv3db.so")

P = 0xFFFFFFFF00000001
POSEIDON_SEED = 260303065
NATURAL, BITREV = 0, 1

_STATUS = {
    0: "OK", 1: "INVALID_ARG", 2: "UNSUPPORTED", 3: "NONCANONICAL",
    4: "OUT_OF_MEMORY", 5: "DEVICE", 6: "BUSY",
}


class V3dbError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"v3db {_STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = _STATUS.get(status, str(status))


class _Job(ctypes.Structure):
    _fields_ = [
        ("d_trace", ctypes.c_void_p),
        ("n_cols", ctypes.c_uint32),
        ("log_rows", ctypes.c_uint32),
        ("log_blowup", ctypes.c_uint32),
        ("cap_height", ctypes.c_uint32),
        ("shift", ctypes.c_uint64),
        ("layout", ctypes.c_int),
        ("d_lde", ctypes.c_void_p),
        ("d_tree", ctypes.c_void_p),
        ("d_cap", ctypes.c_void_p),
    ]


class _ServerCfg(ctypes.Structure):
    _fields_ = [
        ("slots", ctypes.c_uint32),
        ("max_batch", ctypes.c_uint32),
        ("max_queue", ctypes.c_uint32),
        ("hbm_budget_bytes", ctypes.c_size_t),
        ("sim_ns_per_element", ctypes.c_double),
    ]


class _Request(ctypes.Structure):
    _fields_ = [
        ("h_trace", ctypes.c_void_p),
        ("n_cols", ctypes.c_uint32),
        ("log_rows", ctypes.c_uint32),
        ("log_blowup", ctypes.c_uint32),
        ("cap_height", ctypes.c_uint32),
        ("shift", ctypes.c_uint64),
        ("h_cap", ctypes.c_void_p),
        ("t_arrive", ctypes.c_double),
        ("flags", ctypes.c_uint32),
    ]


class _Timing(ctypes.Structure):
    _fields_ = [
        ("t_arrive", ctypes.c_double),
        ("t_admit", ctypes.c_double),
        ("t_done", ctypes.c_double),
        ("batch_size", ctypes.c_uint32),
        ("slot", ctypes.c_uint32),
        ("t_dev_start", ctypes.c_double),
        ("t_dev_end", ctypes.c_double),
    ]


class _Stats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_uint64),
        ("completed", ctypes.c_uint64),
        ("failed", ctypes.c_uint64),
        ("batches", ctypes.c_uint64),
        ("hbm_in_use", ctypes.c_size_t),
        ("hbm_peak", ctypes.c_size_t),
        ("pool_bytes", ctypes.c_size_t),
    ]


class _Schedule(ctypes.Structure):
    _fields_ = [
        ("log_rows", ctypes.c_uint32),
        ("log_blowup", ctypes.c_uint32),
        ("split_log", ctypes.c_uint32),
        ("tile_cap", ctypes.c_uint32 * 3),
        ("chunk_cols", ctypes.c_uint32),
        ("time_us", ctypes.c_double),
    ]


@dataclass
class Schedule:
    """How one (log_rows, log_blowup) extension is cut into kernels (see v3db_schedule)."""
    log_rows: int
    log_blowup: int
    split_log: int
    tile_cap: tuple
    chunk_cols: int
    time_us: float = 0.0

    @staticmethod
    def _from(c: "_Schedule") -> "Schedule":
        return Schedule(c.log_rows, c.log_blowup, c.split_log, tuple(c.tile_cap), c.chunk_cols, c.time_us)

    def _to(self) -> "_Schedule":
        return _Schedule(self.log_rows, self.log_blowup, self.split_log, (ctypes.c_uint32 * 3)(*self.tile_cap),
                         self.chunk_cols, self.time_us)


class _Snapshot(ctypes.Structure):
    _fields_ = [
        ("log_lists", ctypes.c_uint32),
        ("log_slots", ctypes.c_uint32),
        ("m", ctypes.c_uint32),
        ("dim", ctypes.c_uint32),
        ("k", ctypes.c_uint32),
        ("d_flag", ctypes.c_void_p),
        ("d_item", ctypes.c_void_p),
        ("d_codes", ctypes.c_void_p),
        ("d_centroids", ctypes.c_void_p),
        ("d_codebooks", ctypes.c_void_p),
    ]


_lib = None


def lib():
    """Load libv3db.so (after torch, so both share torch's HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (its libamdhip64 must be the one the library binds to)
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(python paper_2603_03065_amd/build.py)")
    L = ctypes.CDLL(LIB_PATH)
    # a library built from other sources than the tree's would run other kernels than
    # the ones read, tested and measured here: refuse it
    from .build import source_digest
    built = getattr(L, "v3db_build_digest", None)
    if built is not None:
        built.restype, built.argtypes = ctypes.c_char_p, []
        built = built().decode()
    if built != source_digest():
        raise ImportError(f"{LIB_PATH} was built from other sources than csrc/ and include/v3db.h "
                          "hold now; rebuild it with __graft_entry__.build()")
    vp, u32, u64, sz, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t, ctypes.c_int
    sig = {
        "v3db_ctx_create": (i32, [i32, u64, sz, ctypes.POINTER(vp)]),
        "v3db_ctx_destroy": (None, [vp]),
        "v3db_last_error": (ctypes.c_char_p, []),
        "v3db_build_digest": (ctypes.c_char_p, []),
        "v3db_poseidon_constants": (i32, [vp, vp, vp, ctypes.POINTER(u32)]),
        "v3db_ctx_hash_path": (i32, [vp]),
        "v3db_derive_poseidon_constants": (i32, [u64, vp, vp, ctypes.POINTER(u32)]),
        "v3db_lde": (i32, [vp, vp, u32, u32, u32, u64, i32, vp, vp]),
        "v3db_poseidon_permute": (i32, [vp, vp, sz, vp]),
        "v3db_merkle_commit": (i32, [vp, vp, u32, u32, u32, vp, vp, vp]),
        "v3db_merkle_commit_noalloc": (i32, [vp, vp, u32, u32, u32, vp, vp]),
        "v3db_commit_batch": (i32, [vp, ctypes.POINTER(_Job), sz, vp]),
        "v3db_commit_batch_scratch_bytes": (sz, [ctypes.POINTER(_Job), sz]),
        "v3db_profile_enable": (i32, [vp, i32]),
        "v3db_set_option": (i32, [vp, i32, u64]),
        "v3db_clock": (ctypes.c_double, []),
        "v3db_server_create": (i32, [vp, ctypes.POINTER(_ServerCfg), ctypes.POINTER(vp)]),
        "v3db_server_submit": (i32, [vp, ctypes.POINTER(_Request), ctypes.POINTER(u64)]),
        "v3db_server_poll": (i32, [vp, u64, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(_Timing)]),
        "v3db_server_drain": (i32, [vp]),
        "v3db_server_stats_get": (i32, [vp, ctypes.POINTER(_Stats)]),
        "v3db_server_destroy": (None, [vp]),
        "v3db_profile_read": (i32, [vp, vp, vp]),
        "v3db_autotune_lde": (i32, [vp, u32, u32, u32, i32, ctypes.POINTER(_Schedule)]),
        "v3db_open_batch": (i32, [vp, vp, u32, u32, vp, u32, vp, sz, vp, vp, vp]),
        "v3db_snapshot_commit": (i32, [vp, ctypes.POINTER(_Snapshot), vp, vp, vp, vp]),
        "v3db_grand_product": (i32, [vp, vp, u32, u64, u64, u64, vp, vp, vp]),
        "v3db_fri_commit": (i32, [vp, vp, u32, u64, vp, u32, u32, vp, vp, vp, vp]),
        "v3db_verify_batch": (i32, [vp, vp, u32, u32, u32, vp, sz, vp, vp, vp, vp]),
        "v3db_get_schedule": (i32, [vp, u32, u32, ctypes.POINTER(_Schedule)]),
        "v3db_set_schedule": (i32, [vp, ctypes.POINTER(_Schedule)]),
        "v3db_schedules_save": (i32, [vp, ctypes.c_char_p, ctypes.POINTER(sz)]),
        "v3db_schedules_load": (i32, [vp, ctypes.c_char_p, ctypes.POINTER(sz)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(status: int):
    if status != 0:
        raise V3dbError(status, lib().v3db_last_error().decode(errors="replace"))


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _ptr(t, numel: Optional[int] = None, device=None, what: str = "tensor") -> Optional[int]:
    """Device pointer of a contiguous int64 CUDA tensor; with numel, the tensor must hold at
    least that many words, and with device, live on that device (the library writes through
    raw pointers, so a short or misplaced buffer is refused here)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.int64 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{what}: expected a contiguous int64 CUDA tensor")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{what}: holds {t.numel()} words, needs {numel}")
    if device is not None and t.device.index != device:
        raise ValueError(f"{what}: on cuda:{t.device.index}, the context is on cuda:{device}")
    return t.data_ptr()


def to_device(a: np.ndarray, device="cuda"):
    """uint64 numpy array -> int64 torch tensor on the device (same bits)."""
    import torch
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return torch.from_numpy(a.view(np.int64)).to(device)


def to_host(t) -> np.ndarray:
    """int64 torch tensor -> uint64 numpy array (same bits)."""
    return t.detach().cpu().contiguous().numpy().view(np.uint64)


def derive_poseidon_constants(seed: int = POSEIDON_SEED):
    """Host-only: (rc [30][12], circ [12], attempts) a context with this seed uses."""
    rc = np.zeros((30, 12), dtype=np.uint64)
    circ = np.zeros(12, dtype=np.uint64)
    att = ctypes.c_uint32(0)
    _check(lib().v3db_derive_poseidon_constants(seed, rc.ctypes.data, circ.ctypes.data, ctypes.byref(att)))
    return rc, circ, int(att.value)


@dataclass
class Job:
    """One trace to commit; tensors are int64 on the device."""
    trace: object                      # [n_cols][2^log_rows]
    log_blowup: int = 3
    cap_height: int = 0
    shift: int = 7
    layout: int = NATURAL
    lde: object = None                 # [n_cols][N] or None (scratch)
    tree: object = None                # [2N - 2^h][4] or None
    cap: object = None                 # [2^h][4]; allocated if None


class Context:
    """A device context: resident Poseidon constants and twiddle tables."""

    def __init__(self, device: int = 0, seed: int = POSEIDON_SEED, hbm_budget: int = 0):
        L = lib()
        h = ctypes.c_void_p()
        _check(L.v3db_ctx_create(device, seed, hbm_budget, ctypes.byref(h)))
        self._h = h
        self.device = device
        self.seed = seed

    def close(self):
        if getattr(self, "_h", None):
            lib().v3db_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def handle(self):
        return self._h

    @property
    def hash_path(self) -> str:
        """'mfma' (int8 matrix cores) or 'valu': the form of the permutation's linear
        layer the bulk hashing kernels of this context use (results are identical)."""
        return {1: "mfma", 0: "valu"}[lib().v3db_ctx_hash_path(self._h)]

    def poseidon_constants(self):
        rc = np.zeros((30, 12), dtype=np.uint64)
        circ = np.zeros(12, dtype=np.uint64)
        att = ctypes.c_uint32(0)
        _check(lib().v3db_poseidon_constants(self._h, rc.ctypes.data, circ.ctypes.data, ctypes.byref(att)))
        return rc, circ, int(att.value)

    def lde(self, trace, log_blowup: int, shift: int = 7, layout: int = NATURAL, out=None, stream=None):
        import torch
        n_cols, n = trace.shape
        log_rows = n.bit_length() - 1
        if 1 << log_rows != n:
            raise ValueError("rows must be a power of two")
        if out is None:
            out = torch.empty((n_cols, n << log_blowup), dtype=torch.int64, device=trace.device)
        d = self.device
        _check(lib().v3db_lde(self._h, _ptr(trace, n_cols * n, d, "trace"), n_cols, log_rows, log_blowup, shift,
                              layout, _ptr(out, (n_cols * n) << log_blowup, d, "out"), _stream(stream)))
        return out

    def poseidon_permute(self, states, stream=None):
        """In place on a [count][12] tensor."""
        count = states.numel() // 12
        _check(lib().v3db_poseidon_permute(self._h, _ptr(states, 12 * count, self.device, "states"), count,
                                           _stream(stream)))
        return states

    def merkle_commit(self, mat, cap_height: int, tree=None, cap=None, stream=None):
        import torch
        n_cols, nl = mat.shape
        log_leaves = nl.bit_length() - 1
        if 1 << log_leaves != nl:
            raise ValueError("leaf count must be a power of two")
        if cap is None:
            cap = torch.empty((1 << cap_height, 4), dtype=torch.int64, device=mat.device)
        d = self.device
        tree_words = ((2 << log_leaves) - (1 << cap_height)) * 4 if cap_height <= log_leaves else None
        _check(lib().v3db_merkle_commit(self._h, _ptr(mat, n_cols * nl, d, "mat"), n_cols, log_leaves, cap_height,
                                        _ptr(tree, tree_words, d, "tree"),
                                        _ptr(cap, (1 << cap_height) * 4 if cap_height < 63 else None, d, "cap"),
                                        _stream(stream)))
        return cap

    def merkle_commit_noalloc(self, mat, cap_height: int, cap, stream=None):
        """merkle_commit whose tree levels live in the library's static device scratch
        (v3db_merkle_commit_noalloc): allocates nothing; cap must be given."""
        n_cols, nl = mat.shape
        log_leaves = nl.bit_length() - 1
        if 1 << log_leaves != nl:
            raise ValueError("leaf count must be a power of two")
        d = self.device
        _check(lib().v3db_merkle_commit_noalloc(self._h, _ptr(mat, n_cols * nl, d, "mat"), n_cols, log_leaves,
                                                cap_height,
                                                _ptr(cap, (1 << cap_height) * 4 if cap_height < 63 else None, d,
                                                     "cap"), _stream(stream)))
        return cap

    def open_batch(self, mat, tree, cap_height: int, idx, rows=None, paths=None, stream=None):
        """Rows idx[q] of the committed matrix mat ([C][2^L]) and their authentication paths
        ([Q][L - cap_height][4], leaf level first) from the stored tree."""
        import torch
        n_cols, nl = mat.shape
        log_leaves = nl.bit_length() - 1
        q = idx.numel()
        if rows is None:
            rows = torch.empty((q, n_cols), dtype=torch.int64, device=mat.device)
        if paths is None:
            paths = torch.empty((q, max(log_leaves - cap_height, 0), 4), dtype=torch.int64, device=mat.device)
        d = self.device
        depth = max(log_leaves - cap_height, 0)
        tree_words = ((2 << log_leaves) - (1 << cap_height)) * 4 if cap_height <= log_leaves else None
        _check(lib().v3db_open_batch(self._h, _ptr(mat, n_cols * nl, d, "mat"), n_cols, log_leaves,
                                     _ptr(tree, tree_words, d, "tree"), cap_height, _ptr(idx, q, d, "idx"), q,
                                     _ptr(rows, q * n_cols, d, "rows"),
                                     _ptr(paths, q * depth * 4, d, "paths") if paths.numel() else None,
                                     _stream(stream)))
        return rows, paths

    def verify_batch(self, rows, paths, idx, cap, log_leaves: int, cap_height: int, ok=None, stream=None):
        """1 where row q and path q reproduce cap entry idx[q] >> (log_leaves - cap_height), else 0."""
        import torch
        q, n_cols = rows.shape
        if ok is None:
            ok = torch.empty((q,), dtype=torch.int32, device=rows.device)
        if ok.dtype != torch.int32 or not ok.is_cuda or not ok.is_contiguous() or ok.numel() < q:
            raise ValueError(f"ok: expected a contiguous int32 CUDA tensor of at least {q} entries")
        d = self.device
        depth = max(log_leaves - cap_height, 0)
        _check(lib().v3db_verify_batch(self._h, _ptr(rows, q * n_cols, d, "rows"), n_cols, log_leaves, cap_height,
                                       _ptr(idx, q, d, "idx"), q,
                                       _ptr(paths, q * depth * 4, d, "paths") if paths.numel() else None,
                                       _ptr(cap, (1 << cap_height) * 4 if cap_height < 63 else None, d, "cap"),
                                       ok.data_ptr(), _stream(stream)))
        return ok

    def snapshot_commit(self, log_lists: int, log_slots: int, m: int, dim: int, k: int, flag, item, codes,
                        centroids, codebooks, list_roots=None, stream=None):
        """Commitment (root_mk, root_cb) of a fixed-shape IVF-PQ snapshot held in device
        tensors: flag, item [N]; codes [m][N]; centroids [n_list][dim]; codebooks
        [m][k][dim/m]. Returns (root_mk [4], root_cb [4], list_roots [n_list][4])."""
        import torch
        dev = flag.device
        if list_roots is None:
            list_roots = torch.empty((1 << log_lists, 4), dtype=torch.int64, device=dev)
        mk = torch.empty((4,), dtype=torch.int64, device=dev)
        cb = torch.empty((4,), dtype=torch.int64, device=dev)
        d = self.device
        # sizes are checked for shapes the library accepts; it reports the others itself
        valid = m >= 1 and k >= 1 and dim >= 1 and dim % m == 0 and log_lists + log_slots <= 26 and m <= 65535 \
            and k * dim < 1 << 32
        N, nl = (1 << (log_lists + log_slots), 1 << log_lists) if valid else (None, None)
        need = (lambda x: x) if valid else (lambda x: None)
        sn = _Snapshot(log_lists, log_slots, m, dim, k, _ptr(flag, need(N), d, "flag"), _ptr(item, need(N), d, "item"),
                       _ptr(codes, need(m * N if valid else 0), d, "codes"),
                       _ptr(centroids, need(nl * dim if valid else 0), d, "centroids"),
                       _ptr(codebooks, need(k * dim), d, "codebooks"))
        _check(lib().v3db_snapshot_commit(self._h, ctypes.byref(sn), _ptr(list_roots, need(4 * nl if valid else 0), d,
                                                                          "list_roots"),
                                          _ptr(mk), _ptr(cb), _stream(stream)))
        return mk, cb, list_roots

    def grand_product(self, cols, alpha: int, beta: int, z=None, want_z: bool = True, stream=None):
        """Running products z_i = prod_{j<=i} (alpha - Compress(row j; beta)) of a column-major
        table cols [width][n] (int64 device tensor); returns (z or None, total [1])."""
        import torch
        width, n = cols.shape
        if want_z and z is None:
            z = torch.empty((n,), dtype=torch.int64, device=cols.device)
        total = torch.empty((1,), dtype=torch.int64, device=cols.device)
        d = self.device
        _check(lib().v3db_grand_product(self._h, _ptr(cols, width * n, d, "cols") if n else None, width, n, alpha % P,
                                        beta % P, _ptr(z, n, d, "z") if (want_z and n) else None,
                                        _ptr(total, 1, d, "total"), _stream(stream)))
        return (z if want_z else None), total

    def fri_commit(self, codeword, shift: int, betas, cap_height: int, folded=None, trees=None, caps=None,
                   want_trees: bool = False, stream=None):
        """FRI commit phase over a codeword (int64 device tensor of 2^L values on the coset shift *
        <w_{2^L}>), one round per challenge in betas. Returns (folded f_1..f_R concatenated,
        caps [R][2^h][4], trees concatenated or None)."""
        import torch
        n = codeword.numel()
        log_n = n.bit_length() - 1
        b = np.ascontiguousarray(np.asarray(betas, dtype=np.uint64))
        rounds = b.size
        dev = codeword.device
        if folded is None:
            folded = torch.empty((n - (n >> rounds),), dtype=torch.int64, device=dev)
        if caps is None:
            caps = torch.empty((rounds, 1 << cap_height, 4), dtype=torch.int64, device=dev)
        if want_trees and trees is None:
            words = sum(((n >> r) - (1 << cap_height)) * 4 for r in range(rounds))
            trees = torch.empty((words,), dtype=torch.int64, device=dev)
        d = self.device
        ok = rounds <= log_n and cap_height < 63
        _check(lib().v3db_fri_commit(self._h, _ptr(codeword, n, d, "codeword"), log_n, shift, b.ctypes.data, rounds,
                                     cap_height, _ptr(folded, n - (n >> rounds) if ok else None, d, "folded"),
                                     _ptr(trees, sum(((n >> r) - (1 << cap_height)) * 4 for r in range(rounds))
                                          if ok and cap_height + rounds <= log_n else None, d, "trees"),
                                     _ptr(caps, rounds * (1 << cap_height) * 4 if ok else None, d, "caps"),
                                     _stream(stream)))
        return folded, caps, trees

    @staticmethod
    def _jobs(jobs: Sequence[Job], device=None):
        import torch
        arr = (_Job * len(jobs))()
        for i, j in enumerate(jobs):
            n_cols, n = j.trace.shape
            log_rows = n.bit_length() - 1
            if 1 << log_rows != n:
                raise ValueError("rows must be a power of two")
            if j.cap is None:
                j.cap = torch.empty((1 << j.cap_height, 4), dtype=torch.int64, device=j.trace.device)
            logN = log_rows + j.log_blowup
            ok = 0 <= j.cap_height <= logN < 63
            arr[i] = _Job(_ptr(j.trace, n_cols * n, device, f"job {i} trace"), n_cols, log_rows, j.log_blowup,
                          j.cap_height, j.shift, j.layout,
                          _ptr(j.lde, n_cols << logN if ok else None, device, f"job {i} lde"),
                          _ptr(j.tree, ((2 << logN) - (1 << j.cap_height)) * 4 if ok else None, device,
                               f"job {i} tree"),
                          _ptr(j.cap, (1 << j.cap_height) * 4 if ok else None, device, f"job {i} cap"))
        return arr

    def commit_batch(self, jobs: Sequence[Job], stream=None):
        arr = self._jobs(jobs, self.device)
        _check(lib().v3db_commit_batch(self._h, arr, len(jobs), _stream(stream)))
        return [j.cap for j in jobs]

    def profile_enable(self, on: bool = True):
        _check(lib().v3db_profile_enable(self._h, 1 if on else 0))

    def profile_read(self):
        """{phase: (milliseconds, intervals)} since the last read, for lde / leaf / merkle."""
        ms = np.zeros(4, dtype=np.float64)
        cnt = np.zeros(4, dtype=np.uint64)
        _check(lib().v3db_profile_read(self._h, ms.ctypes.data, cnt.ctypes.data))
        return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(("lde", "leaf", "merkle", "batch"))}

    def set_batching(self, on: bool):
        """False: commit_batch runs each job with its own launch sequence (the baseline)."""
        _check(lib().v3db_set_option(self._h, 0, 1 if on else 0))

    def set_batch_group_bytes(self, n: int):
        _check(lib().v3db_set_option(self._h, 1, n))

    def commit(self, job: Job, stream=None):
        return self.commit_batch([job], stream)[0]

    def autotune_lde(self, log_rows: int, log_blowup: int, n_cols: int, layout: int = NATURAL) -> Schedule:
        """Time candidate schedules for the shape on the device and install the fastest."""
        out = _Schedule()
        _check(lib().v3db_autotune_lde(self._h, log_rows, log_blowup, n_cols, layout, ctypes.byref(out)))
        return Schedule._from(out)

    def get_schedule(self, log_rows: int, log_blowup: int) -> Schedule:
        out = _Schedule()
        _check(lib().v3db_get_schedule(self._h, log_rows, log_blowup, ctypes.byref(out)))
        return Schedule._from(out)

    def set_schedule(self, s: Schedule):
        c = s._to()
        _check(lib().v3db_set_schedule(self._h, ctypes.byref(c)))

    def save_schedules(self, path: str) -> int:
        n = ctypes.c_size_t()
        _check(lib().v3db_schedules_save(self._h, os.fsencode(path), ctypes.byref(n)))
        return n.value

    def load_schedules(self, path: str) -> int:
        n = ctypes.c_size_t()
        _check(lib().v3db_schedules_load(self._h, os.fsencode(path), ctypes.byref(n)))
        return n.value


def commit_batch_scratch_bytes(jobs: Sequence[Job]) -> int:
    arr = Context._jobs(jobs)
    return int(lib().v3db_commit_batch_scratch_bytes(arr, len(jobs)))


REQ_FAIL_INJECT = 1


def clock() -> float:
    """Seconds on the monotonic clock the server stamps requests with."""
    return float(lib().v3db_clock())


class Server:
    """Continuous-batching commit server (see v3db_server_* in include/v3db.h).

    submit() takes a host trace (a contiguous uint64 numpy array or an int64 CPU
    tensor, ideally pinned) and returns a ticket; the caller keeps the trace alive
    until the request is done. Results land in a per-request host cap array.
    """

    def __init__(self, ctx: Optional[Context], slots: int = 4, hbm_budget: int = 64 << 30, max_batch: int = 0,
                 max_queue: int = 0, sim_ns_per_element: float = 0.0):
        cfg = _ServerCfg(slots, max_batch, max_queue, hbm_budget, sim_ns_per_element)
        h = ctypes.c_void_p()
        _check(lib().v3db_server_create(ctx.handle if ctx is not None else None, ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._ctx = ctx
        self._keep = {}

    def submit(self, trace, log_blowup: int = 3, cap_height: int = 2, shift: int = 7, t_arrive: float = -1.0,
               flags: int = 0, shape=None):
        """trace: host [n_cols][2^log_rows] (uint64 numpy or int64 CPU tensor), or with shape=(n_cols,
        log_rows) any object exposing a data pointer via .ctypes.data / .data_ptr() of that many words."""
        if shape is None:
            n_cols, n = trace.shape
            log_rows = int(n).bit_length() - 1
        else:
            n_cols, log_rows = shape
        ptr = trace.data_ptr() if hasattr(trace, "data_ptr") else trace.ctypes.data
        cap = np.zeros((1 << cap_height, 4), dtype=np.uint64)
        req = _Request(ptr, n_cols, log_rows, log_blowup, cap_height, shift, cap.ctypes.data, t_arrive, flags)
        ticket = ctypes.c_uint64(0)
        _check(lib().v3db_server_submit(self._h, ctypes.byref(req), ctypes.byref(ticket)))
        self._keep[int(ticket.value)] = (trace, cap)
        return int(ticket.value)

    def poll(self, ticket: int):
        """None while running; else (status, cap, timing dict)."""
        done, st, t = ctypes.c_int(0), ctypes.c_int(0), _Timing()
        _check(lib().v3db_server_poll(self._h, ticket, ctypes.byref(done), ctypes.byref(st), ctypes.byref(t)))
        if not done.value:
            return None
        _, cap = self._keep.pop(ticket)
        timing = {"t_arrive": t.t_arrive, "t_admit": t.t_admit, "t_done": t.t_done,
                  "batch_size": int(t.batch_size), "slot": int(t.slot),
                  "t_dev_start": t.t_dev_start, "t_dev_end": t.t_dev_end}
        return int(st.value), cap, timing

    def drain(self):
        _check(lib().v3db_server_drain(self._h))

    def stats(self):
        s = _Stats()
        _check(lib().v3db_server_stats_get(self._h, ctypes.byref(s)))
        return {f: int(getattr(s, f)) for f, _ in _Stats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib().v3db_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
