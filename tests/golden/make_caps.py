#!/usr/bin/env python3
"""Write the expected commitments of every commit workload, computed by the CPU oracle.

Each entry is one trace committed as the paper states it (§4.3: comm = MerkleTree of
Hash = Poseidon over each stored row of the extended trace; the extension is the FFT
over a power-of-two domain of §2.1), with the readings fixed for this project (field,
roots, shift 7, blowup 8, rate-8 sponge, 4-element digests, the circulant of seed
260303065). Only `oracle/` computes; `paper_2603_03065_amd.inputs` only draws the
seeded traces and workload shapes.

Files (JSON, hex strings of canonical u64 words):
  caps_small.json   8 cols x 2^12 rows, natural, cap height 0                  (seed 1)
  caps_80x2p18.json 80 cols x 2^18 rows, natural, cap height 4                 (seed 2)
  caps_135x2p20.json 135 cols x 2^20 rows, bit-reversed, cap height 4          (seed 3)
  caps_batch64.json the 64 traces of the batch workload, natural, cap height 2 (seed 4, trace t)
  caps_serve.json   the checked requests of the serving workload (a seeded 2 % sample
                    and every 80 x 2^18 request; seed 5, trace = request index)
For the single traces and the batch every entry also holds SHA-256 digests of the
whole extension ([C][N] column-major u64 little-endian), of the leaf digests
([N][4]) and of the whole stored tree ([2N - 2^h][4], leaves first).

Usage: python tests/golden/make_caps.py small 80x2p18 135x2p20 batch64 serve
(the serving file is rewritten after every request, so an interrupted run keeps what
it finished and a rerun skips the requests already present).
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2603_03065_amd import inputs  # noqa: E402

SEED = 260303065
SHIFT = 7
LOG_BLOWUP = 3
CITE = ("comm = MerkleTree(Hash(row_0), ..., Hash(row_{N-1})) over the rows of the coset extension "
        "(paper §4.3 'Snapshot Commitments' for Hash/MerkleTree, §2.1 for the FFT over a power-of-two domain); "
        "computed by oracle/ only")

SINGLES = {
    # name: (n_cols, log_rows, layout, cap_height, data seed)
    "small": (8, 12, oracle.NATURAL, 0, 1),
    "80x2p18": (80, 18, oracle.NATURAL, 4, 2),
    "135x2p20": (135, 20, oracle.BITREV, 4, 3),
}


def hexs(a) -> list:
    return [[f"{int(v):016x}" for v in row] for row in np.asarray(a).reshape(-1, 4)]


def sha(a: np.ndarray) -> str:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return hashlib.sha256(a.view(np.uint8).data).hexdigest()


def commit_entry(pos, seed, trace_id, n_cols, log_rows, layout, cap_height, digests=True):
    tr = inputs.trace(seed, trace_id, n_cols, log_rows)
    t0 = time.time()
    cap, lde, tree = pos.commit(tr, LOG_BLOWUP, SHIFT, layout, cap_height, want_lde=digests, want_tree=digests)
    e = {"seed": seed, "trace_id": trace_id, "n_cols": n_cols, "log_rows": log_rows, "log_blowup": LOG_BLOWUP,
         "shift": SHIFT, "layout": "bitrev" if layout == oracle.BITREV else "natural", "cap_height": cap_height,
         "cap": hexs(cap)}
    if digests:
        N = 1 << (log_rows + LOG_BLOWUP)
        e["lde_sha256"] = sha(lde)
        e["leaves_sha256"] = sha(tree[:N])
        e["tree_sha256"] = sha(tree)
        del lde, tree
    print(f"  {n_cols} x 2^{log_rows} (seed {seed}, trace {trace_id}): {time.time() - t0:.1f} s", flush=True)
    return e


def write(name, doc):
    path = os.path.join(HERE, f"caps_{name}.json")
    with open(path + ".tmp", "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")
    os.replace(path + ".tmp", path)


def header(what):
    return {"what": what, "cite": CITE, "poseidon_seed": SEED, "written_by": "tests/golden/make_caps.py"}


def main(parts):
    pos = oracle.Poseidon(SEED)
    print(f"oracle threads: {oracle.set_threads(0)}", flush=True)
    for part in parts:
        print(f"{part}:", flush=True)
        if part in SINGLES:
            C, L, layout, h, seed = SINGLES[part]
            doc = header(f"single trace {C} cols x 2^{L} rows, blowup 8")
            doc["entries"] = [commit_entry(pos, seed, 0, C, L, layout, h)]
            write(part, doc)
        elif part == "batch64":
            doc = header("the 64 traces of the batch workload (inputs.batch_shapes), blowup 8, natural, cap height 2")
            doc["entries"] = [commit_entry(pos, 4, t, C, L, oracle.NATURAL, 2)
                              for t, (L, C) in enumerate(inputs.batch_shapes(64))]
            write(part, doc)
        elif part == "serve":
            reqs = inputs.serve_requests(120.0, 50.0)
            checked = inputs.serve_checked(reqs)
            path = os.path.join(HERE, "caps_serve.json")
            doc = header("checked requests of the serving workload (inputs.serve_requests(120, 50), "
                         "inputs.serve_checked): a seeded 2 % sample and every 80 x 2^18 request")
            doc["entries"] = {}
            if os.path.exists(path):
                with open(path) as f:
                    doc["entries"] = json.load(f).get("entries", {})
            # the sampled requests first (mostly small), then the large ones
            order = sorted(checked, key=lambda i: (reqs[i][1:4] == inputs.SERVE_BIG_SHAPE, i))
            for i in order:
                if str(i) in doc["entries"]:
                    continue
                _, L, C, h = reqs[i]
                doc["entries"][str(i)] = commit_entry(pos, inputs.SERVE_TRACE_SEED, i, C, L, oracle.NATURAL, h,
                                                      digests=False)
                write("serve", doc)
            print(f"  {len(doc['entries'])} of {len(checked)} requests stored", flush=True)
        else:
            raise SystemExit(f"unknown part {part!r}")


if __name__ == "__main__":
    main(sys.argv[1:] or ["small", "80x2p18", "135x2p20", "batch64", "serve"])
