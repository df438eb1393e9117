"""The C-ABI library: it loads, exports every entry point include/v3db.h
declares, and its host-only logic (argument checks that need no device, constant
derivation) behaves; no kernel runs here."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "v3db.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(v3db_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def v3db():
    import paper_2603_03065_amd as m
    m.lib()
    return m


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("v3db_lde", "v3db_poseidon_permute", "v3db_merkle_commit", "v3db_commit_batch",
                     "v3db_ctx_create", "v3db_ctx_destroy", "v3db_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(v3db):
    lib = v3db.lib()
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", v3db.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (v3db_\w+)", out))
    assert set(_declared()) <= exported


def test_library_constants_match_oracle(v3db, poseidon):
    rc, circ, attempts = v3db.derive_poseidon_constants(poseidon.seed)
    assert np.array_equal(rc, poseidon.rc)
    assert np.array_equal(circ, poseidon.circ)
    assert attempts == poseidon.mds_attempts


def test_library_constants_other_seeds(v3db, oracle_mod):
    for seed in (0, 1, 2**63 + 5):
        o = oracle_mod.Poseidon(seed)
        rc, circ, attempts = v3db.derive_poseidon_constants(seed)
        assert np.array_equal(rc, o.rc) and np.array_equal(circ, o.circ) and attempts == o.mds_attempts


def test_scratch_size_is_host_logic(v3db):
    lib = v3db.lib()
    J = v3db._Job
    jobs = (J * 2)()
    jobs[0] = J(None, 8, 12, 3, 0, 7, 0, None, None, None)
    jobs[1] = J(None, 80, 10, 3, 2, 7, 0, None, None, None)
    b = lib.v3db_commit_batch_scratch_bytes(jobs, 2)
    # two natural-layout jobs are batched: Y (n words per column), LDE and tree of
    # every job coexist, each rounded up to 256 bytes
    def batched(C, L, h):
        y = C * (1 << L) * 8
        lde = C * (1 << (L + 3)) * 8
        tree = ((2 << (L + 3)) - (1 << h)) * 32
        return (y + lde + tree + 255) // 256 * 256
    assert b == batched(8, 12, 0) + batched(80, 10, 2)
    # a lone job is committed alone: its LDE, then a region shared by Y and the tree
    one = lib.v3db_commit_batch_scratch_bytes(jobs, 1)
    assert one == 8 * (1 << 15) * 8 + max(8 * (1 << 12) * 8, ((2 << 15) - 1) * 32)


def test_null_context_is_rejected_without_device(v3db):
    lib = v3db.lib()
    assert lib.v3db_lde(None, None, 1, 1, 3, 7, 0, None, None) == 1
    assert b"NULL ctx" in lib.v3db_last_error()
    assert lib.v3db_commit_batch(None, None, 0, None) == 1
    assert lib.v3db_poseidon_permute(None, None, 0, None) == 1


def test_schedule_calls_reject_null_arguments_without_device(v3db):
    lib = v3db.lib()
    s = v3db._Schedule(12, 3, 6, (ctypes.c_uint32 * 3)(4, 4, 4), 8, 0.0)
    assert lib.v3db_autotune_lde(None, 12, 3, 8, 0, None) == 1
    assert b"NULL ctx" in lib.v3db_last_error()
    assert lib.v3db_get_schedule(None, 12, 3, ctypes.byref(s)) == 1
    assert lib.v3db_set_schedule(None, ctypes.byref(s)) == 1
    assert lib.v3db_schedules_save(None, b"/dev/null", None) == 1
    assert lib.v3db_schedules_load(None, b"/dev/null", None) == 1


def test_open_and_verify_reject_bad_arguments_without_device(v3db):
    lib = v3db.lib()
    assert lib.v3db_open_batch(None, None, 1, 4, None, 0, None, 1, None, None, None) == 1
    assert b"NULL ctx" in lib.v3db_last_error()
    assert lib.v3db_verify_batch(None, None, 1, 4, 0, None, 1, None, None, None, None) == 1
    assert b"NULL ctx" in lib.v3db_last_error()


def test_snapshot_commit_rejects_bad_arguments_without_device(v3db):
    lib = v3db.lib()
    assert lib.v3db_snapshot_commit(None, None, None, None, None, None) == 1
    assert b"NULL ctx" in lib.v3db_last_error()


def test_grand_product_rejects_bad_arguments_without_device(v3db):
    lib = v3db.lib()
    assert lib.v3db_grand_product(None, None, 1, 4, 1, 2, None, None, None) == 1
    assert b"NULL ctx" in lib.v3db_last_error()


def test_fri_commit_rejects_bad_arguments_without_device(v3db):
    lib = v3db.lib()
    assert lib.v3db_fri_commit(None, None, 4, 7, None, 1, 0, None, None, None, None) == 1
    assert b"NULL ctx" in lib.v3db_last_error()


def test_library_is_built_from_the_tree_sources(v3db, tmp_path):
    """The library reports the digest of the sources it was built from, and the loader
    refuses a library whose digest differs from the tree's."""
    from paper_2603_03065_amd.build import source_digest
    assert v3db.lib().v3db_build_digest().decode() == source_digest()
    # a copy of the package whose header differs from the one the library was built with
    import shutil
    import subprocess
    import sys
    pkg = tmp_path / "paper_2603_03065_amd"
    shutil.copytree(os.path.dirname(v3db.LIB_PATH), pkg, ignore=shutil.ignore_patterns("_build", "__pycache__"))
    (tmp_path / "include").mkdir()
    (tmp_path / "include" / "v3db.h").write_text(open(HEADER).read() + "\n/* edited */\n")
    code = ("import paper_2603_03065_amd as m\n"
            "try:\n    m.lib()\nexcept ImportError as e:\n    print('refused:', e)\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=tmp_path, capture_output=True, text=True, timeout=300)
    assert "refused:" in r.stdout and "rebuild" in r.stdout, r.stdout + r.stderr
