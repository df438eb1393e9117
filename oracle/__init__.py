"""Reference oracle (CPU) for the trace-commitment phase: Goldilocks coset LDE,
Poseidon row hashing, Merkle tree and cap.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package. The plain C implementation
lives in ``oracle.c`` (see ``oracle.h`` for the passages of the paper each part
follows); this module compiles it with gcc and exposes numpy wrappers. It shares
no code with the GPU library and does not import it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

P = 0xFFFFFFFF00000001
WIDTH, RATE, DIGEST, ROUNDS = 12, 8, 4, 30
NATURAL, BITREV = 0, 1


def build(verbose: bool = False) -> str:
    """Compile oracle.c into liboracle.so next to it (gcc, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", LIB + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("seed", ctypes.c_uint64),
        ("rc", (ctypes.c_uint64 * WIDTH) * ROUNDS),
        ("circ", ctypes.c_uint64 * WIDTH),
        ("mds", (ctypes.c_uint64 * WIDTH) * WIDTH),
        ("mds_attempts", ctypes.c_uint32),
        ("stream_next", ctypes.c_uint64),
    ]


_lib = None
_U64P = ctypes.POINTER(ctypes.c_uint64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    lib = ctypes.CDLL(LIB)
    u64, u32, i32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
    pp = ctypes.POINTER(_Params)
    sig = {
        "or_add": (u64, [u64, u64]),
        "or_sub": (u64, [u64, u64]),
        "or_mul": (u64, [u64, u64]),
        "or_pow": (u64, [u64, u64]),
        "or_inv": (u64, [u64]),
        "or_root_of_unity": (u64, [u32]),
        "or_splitmix64": (u64, [u64, u64]),
        "or_ntt": (None, [_U64P, u32, i32]),
        "or_lde": (i32, [_U64P, u32, u32, u32, u64, i32, _U64P]),
        "or_interpolate": (i32, [_U64P, u32, u32, _U64P]),
        "or_eval_columns": (None, [_U64P, u32, u64, _U64P, u32, _U64P]),
        "or_poseidon_params_init": (i32, [u64, pp]),
        "or_singular_minor_count": (u64, [_U64P]),
        "or_det12": (u64, [_U64P]),
        "or_poseidon_permute_batch": (None, [pp, _U64P, ctypes.c_size_t]),
        "or_sponge_state": (None, [pp, _U64P, u32, _U64P]),
        "or_compress_state": (None, [pp, _U64P, _U64P, _U64P]),
        "or_leaf_digests": (i32, [pp, _U64P, u32, u32, _U64P]),
        "or_merkle_commit": (i32, [pp, _U64P, u32, u32, u32, _U64P, _U64P]),
        "or_merkle_path": (i32, [_U64P, u32, u32, u64, _U64P]),
        "or_merkle_open": (None, [pp, _U64P, u64, _U64P, u32, _U64P, ctypes.POINTER(u64)]),
        "or_commit": (i32, [pp, _U64P, u32, u32, u32, u64, i32, u32, _U64P, _U64P, _U64P]),
        "or_snapshot_commit": (i32, [pp, u32, u32, u32, u32, u32, _U64P, _U64P, _U64P, _U64P, _U64P, _U64P, _U64P,
                                     _U64P, _U64P]),
        "or_grand_product": (i32, [_U64P, u32, u64, u64, u64, _U64P, _U64P]),
        "or_fri_commit": (i32, [pp, _U64P, u32, u64, _U64P, u32, u32, _U64P, _U64P, _U64P]),
        "or_set_threads": (i32, [i32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_U64P)


def _u64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint64))


# ---------------------------------------------------------------- field

def add(a: int, b: int) -> int:
    return int(_load().or_add(a, b))


def sub(a: int, b: int) -> int:
    return int(_load().or_sub(a, b))


def mul(a: int, b: int) -> int:
    return int(_load().or_mul(a, b))


def pow_(a: int, e: int) -> int:
    return int(_load().or_pow(a, e))


def inv(a: int) -> int:
    return int(_load().or_inv(a))


def root_of_unity(log_n: int) -> int:
    return int(_load().or_root_of_unity(log_n))


def splitmix64(seed: int, i: int) -> int:
    return int(_load().or_splitmix64(seed, i))


def set_threads(n: int = 0) -> int:
    return int(_load().or_set_threads(n))


# ---------------------------------------------------------------- NTT / LDE

def ntt(x, inverse: bool = False) -> np.ndarray:
    a = _u64(x).copy()
    n = a.size
    log_n = n.bit_length() - 1
    assert 1 << log_n == n
    _load().or_ntt(_ptr(a), log_n, 1 if inverse else 0)
    return a


def interpolate(trace: np.ndarray) -> np.ndarray:
    t = _u64(trace)
    c, n = t.shape
    out = np.empty_like(t)
    rc = _load().or_interpolate(_ptr(t), c, n.bit_length() - 1, _ptr(out))
    assert rc == 0
    return out


def lde(trace: np.ndarray, log_blowup: int, shift: int, layout: int = NATURAL) -> np.ndarray:
    """trace [C][n] -> LDE [C][n << log_blowup]."""
    t = _u64(trace)
    c, n = t.shape
    log_rows = n.bit_length() - 1
    out = np.empty((c, n << log_blowup), dtype=np.uint64)
    rc = _load().or_lde(_ptr(t), c, log_rows, log_blowup, shift, layout, _ptr(out))
    if rc != 0:
        raise ValueError("oracle lde: invalid arguments")
    return out


def eval_columns(coeffs: np.ndarray, points) -> np.ndarray:
    """out[c][i] = P_c(points[i]) for the coefficient rows of coeffs [C][n]."""
    cf = _u64(coeffs)
    x = _u64(points)
    out = np.empty((cf.shape[0], x.size), dtype=np.uint64)
    _load().or_eval_columns(_ptr(cf), cf.shape[0], cf.shape[1], _ptr(x), x.size, _ptr(out))
    return out


# ---------------------------------------------------------------- Poseidon

class Poseidon:
    """Constants derived from a seed, plus the primitive operations."""

    def __init__(self, seed: int):
        self._p = _Params()
        rc = _load().or_poseidon_params_init(seed, ctypes.byref(self._p))
        if rc != 0:
            raise RuntimeError("no MDS draw passed")
        self.seed = seed

    @property
    def rc(self) -> np.ndarray:
        return np.ctypeslib.as_array(self._p.rc).copy()

    @property
    def circ(self) -> np.ndarray:
        return np.ctypeslib.as_array(self._p.circ).copy()

    @property
    def mds(self) -> np.ndarray:
        return np.ctypeslib.as_array(self._p.mds).copy()

    @property
    def mds_attempts(self) -> int:
        return int(self._p.mds_attempts)

    @property
    def stream_next(self) -> int:
        return int(self._p.stream_next)

    def permute(self, states) -> np.ndarray:
        s = _u64(states).reshape(-1, WIDTH).copy()
        _load().or_poseidon_permute_batch(ctypes.byref(self._p), _ptr(s), s.shape[0])
        return s

    def sponge_state(self, row) -> np.ndarray:
        r = _u64(row)
        out = np.zeros(WIDTH, dtype=np.uint64)
        _load().or_sponge_state(ctypes.byref(self._p), _ptr(r) if r.size else None, r.size, _ptr(out))
        return out

    def compress_state(self, left, right) -> np.ndarray:
        l, r = _u64(left), _u64(right)
        out = np.zeros(WIDTH, dtype=np.uint64)
        _load().or_compress_state(ctypes.byref(self._p), _ptr(l), _ptr(r), _ptr(out))
        return out

    def snapshot_commit(self, log_lists: int, log_slots: int, m: int, dim: int, k: int, flag, item, codes,
                        centroids, codebooks):
        """Sec. 4.3 snapshot commitment: returns (root_mk, root_cb, list_roots, list_hashes).
        flag, item: [N]; codes: [M][N]; centroids: [n_list][D]; codebooks: [M][K][D/M]
        (canonical flattening), N = n_list * n."""
        n_list = 1 << log_lists
        args = [_u64(a).reshape(-1) for a in (flag, item, codes, centroids, codebooks)]
        roots = np.empty((n_list, DIGEST), dtype=np.uint64)
        hashes = np.empty((n_list, DIGEST), dtype=np.uint64)
        mk = np.empty(DIGEST, dtype=np.uint64)
        cb = np.empty(DIGEST, dtype=np.uint64)
        rc = _load().or_snapshot_commit(ctypes.byref(self._p), log_lists, log_slots, m, dim, k,
                                        *[_ptr(a) for a in args], _ptr(roots), _ptr(hashes), _ptr(mk), _ptr(cb))
        if rc != 0:
            raise ValueError("oracle snapshot_commit: invalid arguments")
        return mk, cb, roots, hashes

    def fri_commit(self, codeword, shift: int, betas, cap_height: int, want_trees: bool = False):
        """FRI commit phase over a codeword of 2^L values on the coset shift * <w_{2^L}>: per round
        the pair-leaf tree's cap, then the fold with betas[r]. Returns (folded f_1..f_R
        concatenated, caps [R][2^h][4], trees concatenated or None)."""
        f = _u64(codeword)
        n = f.size
        log_n = n.bit_length() - 1
        b = _u64(betas)
        rounds = b.size
        folded = np.empty(n - (n >> rounds), dtype=np.uint64)
        caps = np.empty((rounds, 1 << cap_height, DIGEST), dtype=np.uint64)
        words = sum(((n >> r) - (1 << cap_height)) * DIGEST for r in range(rounds))
        trees = np.empty(words, dtype=np.uint64) if want_trees else None
        rc = _load().or_fri_commit(ctypes.byref(self._p), _ptr(f), log_n, shift, _ptr(b), rounds, cap_height,
                                   _ptr(folded), _ptr(trees) if trees is not None else None, _ptr(caps))
        if rc != 0:
            raise ValueError("oracle fri_commit: invalid arguments")
        return folded, caps, trees

    def leaf_digests(self, mat: np.ndarray) -> np.ndarray:
        m = _u64(mat)
        c, nl = m.shape
        out = np.empty((nl, DIGEST), dtype=np.uint64)
        assert _load().or_leaf_digests(ctypes.byref(self._p), _ptr(m), c, nl.bit_length() - 1, _ptr(out)) == 0
        return out

    def merkle_commit(self, mat: np.ndarray, cap_height: int, want_tree: bool = False):
        m = _u64(mat)
        c, nl = m.shape
        log_leaves = nl.bit_length() - 1
        cap = np.empty((1 << cap_height, DIGEST), dtype=np.uint64)
        tree = np.empty((2 * nl - (1 << cap_height), DIGEST), dtype=np.uint64) if want_tree else None
        rc = _load().or_merkle_commit(ctypes.byref(self._p), _ptr(m), c, log_leaves, cap_height,
                                      _ptr(tree) if tree is not None else None, _ptr(cap))
        if rc != 0:
            raise ValueError("oracle merkle_commit: invalid arguments")
        return (cap, tree) if want_tree else cap

    def merkle_open(self, leaf, index: int, path: np.ndarray):
        p = _u64(path).reshape(-1, DIGEST)
        node = np.zeros(DIGEST, dtype=np.uint64)
        cap_index = ctypes.c_uint64(0)
        _load().or_merkle_open(ctypes.byref(self._p), _ptr(_u64(leaf)), index,
                               _ptr(p) if p.size else None, p.shape[0], _ptr(node), ctypes.byref(cap_index))
        return node, int(cap_index.value)

    def commit(self, trace: np.ndarray, log_blowup: int, shift: int, layout: int, cap_height: int,
               want_lde: bool = False, want_tree: bool = False):
        t = _u64(trace)
        c, n = t.shape
        log_rows = n.bit_length() - 1
        N = n << log_blowup
        cap = np.empty((1 << cap_height, DIGEST), dtype=np.uint64)
        lde_out = np.empty((c, N), dtype=np.uint64) if want_lde else None
        tree = np.empty((2 * N - (1 << cap_height), DIGEST), dtype=np.uint64) if want_tree else None
        rc = _load().or_commit(ctypes.byref(self._p), _ptr(t), c, log_rows, log_blowup, shift, layout,
                               cap_height, _ptr(lde_out) if lde_out is not None else None,
                               _ptr(tree) if tree is not None else None, _ptr(cap))
        if rc != 0:
            raise ValueError("oracle commit: invalid arguments")
        return cap, lde_out, tree


def grand_product(cols, alpha: int, beta: int, want_z: bool = True):
    """Running products z_i = prod_{j<=i} (alpha - Compress(row j; beta)) of a column-major
    table [width][n]; returns (z or None, total)."""
    c = _u64(cols)
    if c.ndim == 1:
        c = c.reshape(1, -1)
    width, n = c.shape
    z = np.empty(n, dtype=np.uint64) if want_z else None
    total = np.zeros(1, dtype=np.uint64)
    rc = _load().or_grand_product(_ptr(c) if c.size else None, width, n, alpha, beta,
                                  _ptr(z) if (z is not None and n) else None, _ptr(total))
    if rc != 0:
        raise ValueError("oracle grand_product: invalid arguments")
    return z, int(total[0])


def merkle_path(tree: np.ndarray, log_leaves: int, cap_height: int, index: int) -> np.ndarray:
    t = _u64(tree)
    path = np.zeros((max(log_leaves - cap_height, 0), DIGEST), dtype=np.uint64)
    rc = _load().or_merkle_path(_ptr(t), log_leaves, cap_height, index, _ptr(path) if path.size else None)
    assert rc == 0
    return path


def singular_minor_count(m) -> int:
    a = _u64(m).reshape(WIDTH, WIDTH)
    return int(_load().or_singular_minor_count(_ptr(a)))


def det12(m) -> int:
    a = _u64(m).reshape(WIDTH, WIDTH)
    return int(_load().or_det12(_ptr(a)))
