"""Write ``batch_digests.json``: per-instance oracle results of the 512-instance
batch workload (seed 4) and of the first 200 requests of the serving stream
(seed 5), as pair counts and SHA-256 of the packed result (same layout as
``digests.json``).  Only the oracle and the seeded generators are called.

    python tests/golden/make_batch_digests.py
"""
from __future__ import annotations

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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch_digests.json")


def digest(bits):
    counts = [int(np.unpackbits(np.ascontiguousarray(b).view(np.uint8)).sum()) for b in bits]
    return {"counts": counts, "sha256": hashlib.sha256(np.ascontiguousarray(bits).astype("<u8").tobytes()).hexdigest()}


def main():
    out = {}
    t0 = time.time()
    for name, insts in (("batch512", configs.config4()), ("serve200", configs.config5(count=200)[0])):
        rows = []
        for k, inst in enumerate(insts):
            d = digest(worklist.closure(inst.n, inst.edges, inst.grammar))
            d.update({"n": inst.n, "tag": inst.tag})
            rows.append(d)
            if k % 50 == 0:
                print(name, k, f"{time.time() - t0:.0f}s", flush=True)
        out[name] = rows
    with open(OUT, "w") as f:
        json.dump(out, f, indent=0, sort_keys=True)
    print("done", f"{time.time() - t0:.0f}s")


if __name__ == "__main__":
    main()
