"""Write ``digests.json``: oracle results for the larger workloads.

Relational closures come from the worklist oracle; the conjunctive case (Dyck
conjoined with a^n b^n on the ER recipe at n = 8192, the conclusion's
conjunctive generalisation) from the conjunctive Algorithm 1 oracle, which
also stores its loop count.  Single-path lengths (section 5) on the ER Dyck
recipe at n = 2048 and 4096 come from the C transcription of the single-path
oracle: per nonterminal the number of present cells and the sum of their
lengths, the loop count, and a SHA-256 of the uint32 lengths (little-endian,
shape [|N|, n, n], 0 for an absent cell).

Each entry holds, per nonterminal, the number of pairs in R_A and a SHA-256 of
the packed result (uint64 little-endian, shape [|N|, n, ceil(n/64)], bit j%64 of
word j//64 of row i set iff (i, j) in R_A).  Only the oracle and the seeded
generators are called.  The 16384-node case takes tens of minutes on one core:

    python tests/golden/make_digests.py            # all but the 16384-node case
    python tests/golden/make_digests.py --full     # also the 16384-node and conjunctive cases
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

from oracle import conjunctive, single_path, worklist  # noqa: E402
from workloads import configs, grammars  # noqa: E402

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
# conjunctive grammars: (graph, grammar)
CONJ = {"er8192_dyck_and_anbn": lambda: (configs.config3(8192), grammars.dyck_and_anbn())}
# single-path lengths
SP = {"sp_er2048_dyck": lambda: configs.config3(2048), "sp_er4096_dyck": lambda: configs.config3(4096)}


def length_digest(L: np.ndarray) -> dict:
    return {"counts": [int((x > 0).sum()) for x in L], "length_sums": [int(x.astype(np.int64).sum()) for x in L],
            "sha256": hashlib.sha256(np.ascontiguousarray(L).astype("<u4").tobytes()).hexdigest()}


def digest(bits: np.ndarray) -> dict:
    counts = [int(np.unpackbits(np.ascontiguousarray(b).view(np.uint8)).sum()) for b in bits]
    return {"counts": counts, "sha256": hashlib.sha256(np.ascontiguousarray(bits).astype("<u8").tobytes()).hexdigest()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--full", action="store_true")
    ap.add_argument("--only", default=None)
    args = ap.parse_args()
    todo = dict(CASES)
    if args.full:
        todo.update(FULL)
        todo.update(CONJ)
        todo.update(SP)
    if args.only:
        todo = {k: v for k, v in {**CASES, **FULL, **CONJ, **SP}.items() if k == args.only}
    for name, mk in todo.items():
        t = time.time()
        if name in SP:
            inst = mk()
            g = inst.grammar
            L, loops, rc = single_path.lengths_native(inst.n, inst.edges, g)
            assert rc == 0, rc
            d = length_digest(L)
            d["jacobi_loops"] = int(loops)
        elif name in CONJ:
            inst, g = mk()
            dense, loops = conjunctive.closure(inst.n, inst.edges, g)
            d = digest(worklist.pack(dense))
            d["jacobi_loops"] = int(loops)
        else:
            inst = mk()
            g = inst.grammar
            d = digest(worklist.closure(inst.n, inst.edges, g))
        d.update({"n": inst.n, "edges": int(len(inst.edges)), "grammar": g.name,
                  "oracle_seconds": round(time.time() - t, 2)})
        print(name, d, flush=True)
        data = json.load(open(OUT)) if os.path.exists(OUT) else {}  # merge with entries written meanwhile
        data[name] = d
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
