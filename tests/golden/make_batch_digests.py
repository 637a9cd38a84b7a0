"""Write ``batch_digests.json``: per-instance oracle results of the 512-instance
batch workload (seed 4) and of the first 600 requests of the serving stream
(seed 5: the 100 warm-up and 500 measured requests the benchmark submits), as
pair counts and SHA-256 of the packed result (same layout as
``digests.json``).  Only the oracle and the seeded generators are called.

    python tests/golden/make_batch_digests.py                 # both sets
    python tests/golden/make_batch_digests.py --only serve600 # one set, merged
    python tests/golden/make_batch_digests.py --jobs 6        # worker processes
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import worklist  # noqa: E402
from workloads import configs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch_digests.json")

SETS = {
    "batch512": lambda: configs.config4(),
    "serve600": lambda: configs.config5(count=600)[0],
}


def digest(bits):
    counts = [int(np.unpackbits(np.ascontiguousarray(b).view(np.uint8)).sum()) for b in bits]
    return {"counts": counts, "sha256": hashlib.sha256(np.ascontiguousarray(bits).astype("<u8").tobytes()).hexdigest()}


_CACHE = {}


def _insts(name):
    if name not in _CACHE:
        _CACHE[name] = SETS[name]()
    return _CACHE[name]


def _one(args):
    name, k = args
    inst = _insts(name)[k]
    d = digest(worklist.closure(inst.n, inst.edges, inst.grammar))
    d.update({"n": inst.n, "tag": inst.tag})
    return k, d


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", choices=sorted(SETS), default=None)
    ap.add_argument("--jobs", type=int, default=1)
    args = ap.parse_args()
    out = json.load(open(OUT)) if os.path.exists(OUT) else {}
    t0 = time.time()
    for name in ([args.only] if args.only else sorted(SETS)):
        insts = _insts(name)
        rows = [None] * len(insts)
        # largest first, so the pool's tail is short
        order = sorted(range(len(insts)), key=lambda k: -insts[k].n)
        with ProcessPoolExecutor(max_workers=max(1, args.jobs)) as ex:
            for done, (k, d) in enumerate(ex.map(_one, [(name, k) for k in order])):
                rows[k] = d
                if done % 50 == 0:
                    print(name, done, f"{time.time() - t0:.0f}s", flush=True)
        out[name] = rows
        if name == "serve600":
            out.pop("serve200", None)  # superseded: its rows are the first 200 of serve600
        with open(OUT, "w") as f:
            json.dump(out, f, indent=0, sort_keys=True)
    print("done", f"{time.time() - t0:.0f}s")


if __name__ == "__main__":
    main()
