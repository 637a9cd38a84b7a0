"""Write ``digests.json``: oracle results for the larger workloads.

Each entry holds, per nonterminal, the number of pairs in R_A and a SHA-256 of
the packed result (uint64 little-endian, shape [|N|, n, ceil(n/64)], bit j%64 of
word j//64 of row i set iff (i, j) in R_A).  Only the oracle and the seeded
generators are called.  The 16384-node case takes tens of minutes on one core:

    python tests/golden/make_digests.py            # all but the 16384-node case
    python tests/golden/make_digests.py --full     # also the 16384-node case
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import worklist  # noqa: E402
from workloads import configs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "digests.json")

CASES = {
    "hierarchy4096_samegen": lambda: configs.config2(),
    "hierarchy4096_rev_samegen": lambda: configs.config2(reverse=True),
    "er16384_induced1024_dyck": lambda: configs.config3_induced(1024),
    "er1024_dyck": lambda: configs.config3(1024),
    "er2048_dyck": lambda: configs.config3(2048),
    "er4096_dyck": lambda: configs.config3(4096),
}
FULL = {"er16384_dyck": lambda: configs.config3(16384)}


def digest(bits: np.ndarray) -> dict:
    counts = [int(np.unpackbits(np.ascontiguousarray(b).view(np.uint8)).sum()) for b in bits]
    return {"counts": counts, "sha256": hashlib.sha256(np.ascontiguousarray(bits).astype("<u8").tobytes()).hexdigest()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--full", action="store_true")
    ap.add_argument("--only", default=None)
    args = ap.parse_args()
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    todo = dict(CASES)
    if args.full:
        todo.update(FULL)
    if args.only:
        todo = {k: v for k, v in {**CASES, **FULL}.items() if k == args.only}
    for name, mk in todo.items():
        inst = mk()
        t = time.time()
        bits = worklist.closure(inst.n, inst.edges, inst.grammar)
        d = digest(bits)
        d.update({"n": inst.n, "edges": int(len(inst.edges)), "grammar": inst.grammar.name,
                  "oracle_seconds": round(time.time() - t, 2)})
        data[name] = d
        print(name, d, flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
