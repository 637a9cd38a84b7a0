"""The C oracles (worklist closure, single-path lengths, bit-packed Algorithm
1 on two OpenMP threads) built with AddressSanitizer and
UndefinedBehaviorSanitizer (host code only; a small C driver feeds them the
cases): no report on the worked example, ragged random graphs, empty and
one-node graphs and a grammar without binary rules, and the same outputs as
the ordinary builds."""
from __future__ import annotations

import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import bitset, single_path, worklist
from workloads import configs, grammars, graphs

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")


def _fnv(buf: bytes) -> int:
    h = 1469598103934665603
    for c in buf:
        h = ((h ^ c) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


def _cases():
    we = configs.worked_example()
    out = [(we.n, we.edges, we.grammar)]
    for k, (n, m) in enumerate([(1, 1), (63, 150), (64, 200), (65, 190), (130, 400)]):
        n, e = graphs.erdos_renyi(n, min(m, n * max(n - 1, 1)) if n > 1 else 0, 90 + k, labels=2)
        out.append((n, e, grammars.dyck() if k % 2 else grammars.anbn()))
    n, e = graphs.hierarchy(100, 5, roots=2, reverse=True)
    out.append((n, e, grammars.same_generation()))
    out.append((0, np.zeros((0, 3), np.int32), grammars.dyck()))
    out.append((1, np.array([[0, 0, 0]], np.int32), grammars.transitive_closure()))
    out.append((40, graphs.erdos_renyi(40, 90, 7, labels=2)[1],
                grammars.CNF(("S",), ("a", "b"), ((0, 0),), (), "only_terms")))
    return out


def test_oracles_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    exe = tmp_path / "driver"
    r = subprocess.run(["gcc", "-std=gnu11", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp",
                        "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        os.path.join(HERE, "native", "oracle_sanitize_driver.c"),
                        os.path.join(ORACLE, "cfpq_worklist.c"), os.path.join(ORACLE, "cfpq_single_path.c"),
                        os.path.join(ORACLE, "cfpq_bitset.c"), "-o", str(exe)], capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in r.stderr:
        pytest.skip("gcc without sanitizer runtimes: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    cases = _cases()
    lines = []
    for n, e, g in cases:
        e = np.asarray(e, np.int32).reshape(-1, 3)
        lines.append(f"{n} {len(e)} {g.n_nonterminals} {g.n_terminals} {len(g.term)} {len(g.bin)}")
        lines += [" ".join(str(int(x)) for x in row) for row in e]
        lines += [f"{a} {x}" for a, x in g.term]
        lines += [f"{a} {b} {c}" for a, b, c in g.bin]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe)], input="\n".join(lines) + "\n", capture_output=True, text=True, env=env,
                         timeout=300)
    assert run.returncode == 0, run.stderr[-2000:]
    assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr, run.stderr[-2000:]
    got = run.stdout.split("\n")
    for (n, e, g), line in zip(cases, got):
        rc1, rc2, rc3, loops, loops3, h1, h2, h3 = line.split()
        bits = worklist.closure(n, e, g)
        L, loops_c, rc = single_path.lengths_native(n, e, g)
        _, loops_b, _ = bitset.closure(n, e, g)
        assert int(rc1) == 0 and int(rc2) == rc and int(loops) == loops_c
        assert int(rc3) == 0 and int(loops3) == loops_b
        assert int(h1, 16) == _fnv(np.ascontiguousarray(bits).tobytes())
        assert int(h2, 16) == _fnv(np.ascontiguousarray(L).tobytes())
        assert int(h3, 16) == int(h1, 16)  # the same relations in the same layout
