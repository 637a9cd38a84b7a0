"""Pins of the bit-packed Algorithm 1 (``oracle/cfpq_bitset.c``), CPU only.

It is a second CPU implementation of the closure (the benchmark times it on
all host cores), so it is held to what the paper and the mathematics fix, not
to itself: the printed result and loop count of the section 4.3 example, the
two-cycle closed form with Lemma 3's loop count, brute force on tiny graphs,
breadth-first search for the transitive-closure grammar, the simultaneous
update's intermediate states (Algorithm 1 in numpy, itself pinned), and the
Boolean product against a float64 matrix product.  Planted mistakes in a copy
of its source must each fail one of these.
"""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

from oracle import alg1, bitset, brute, worklist
from tests.test_oracle_pins import _bfs_closure, _two_cycle_expected
from workloads import configs, grammars, graphs


def _pins_hold(lib) -> bool:
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")))
    inst = configs.worked_example()
    bits, loops, rc = bitset.closure(inst.n, inst.edges, inst.grammar, lib=lib)
    rel = worklist.relations(bits, inst.n)
    if rc != 0 or loops != 6:  # six loops in section 4.3, the sixth adding nothing
        return False
    for name in inst.grammar.nonterminals:
        if rel[inst.grammar.nt(name)] != {tuple(p) for p in gold["relations"][name]}:
            return False
    # two cycles: the closed form, and Lemma 3's loop count H_max = 8065
    c1 = configs.config1()
    bits, loops, rc = bitset.closure(c1.n, c1.edges, c1.grammar, lib=lib)
    rel = worklist.relations(bits, c1.n)
    s_min, _ = _two_cycle_expected()
    if rc != 0 or loops != 8065 or rel[c1.grammar.nt("S")] != set(s_min) or rel[c1.grammar.nt("S1")] != set(s_min):
        return False
    # multi-edges, several rules per terminal: brute force over paths
    g = grammars.CNF(("S", "X", "Y"), ("a", "b"), ((1, 0), (2, 0), (2, 1)), ((0, 1, 2), (0, 0, 0)), "mut")
    for seed in range(3):
        n, e = graphs.random_tiny(6, 12, 2, 900 + seed, acyclic=True)
        if worklist.relations(bitset.closure(n, e, g, lib=lib)[0], n) != brute.paths_up_to(n, e, g, n - 1):
            return False
    # several words per row (n = 150, ragged): transitive closure against BFS
    n, e = graphs.erdos_renyi(150, 200, 901, labels=2)
    got = worklist.relations(bitset.closure(n, e, grammars.transitive_closure(), lib=lib)[0], n)
    if got[0] != _bfs_closure(n, [(int(u), int(v)) for u, x, v in e if x == 0]):
        return False
    # the simultaneous update, loop by loop, on a grammar with unequal operands
    n, e = graphs.erdos_renyi(70, 220, 5, labels=2)
    _, _, hist = alg1.closure(n, e, grammars.anbn(), keep_history=True)
    for k in (1, 2, 3):
        bits, loops, rc = bitset.closure(n, e, grammars.anbn(), max_loops=k, lib=lib)
        want = hist[min(k, len(hist) - 1)]
        if loops != k or not np.array_equal(worklist.unpack(bits, n), want):
            return False
    return True


def test_bitset_oracle_passes_pins():
    assert _pins_hold(None)


@pytest.mark.parametrize("grammar", ["dyck", "anbn", "same_generation"])
def test_equals_worklist_and_alg1(grammar):
    g = grammars.BY_NAME[grammar]()
    for seed, (n, m) in enumerate([(1, 1), (63, 150), (64, 200), (129, 400)]):
        if grammar == "same_generation":
            n, e = graphs.hierarchy(max(n, 2), seed, roots=1, reverse=bool(seed % 2))
        else:
            n, e = graphs.erdos_renyi(n, min(m, n * (n - 1)) if n > 1 else 0, 60 + seed, labels=len(g.terminals))
        bits, loops, rc = bitset.closure(n, e, g)
        t, loops_a, _ = alg1.closure(n, e, g)
        assert rc == 0 and loops == loops_a, (grammar, n)
        assert np.array_equal(bits, worklist.closure(n, e, g)), (grammar, n)
        assert np.array_equal(worklist.unpack(bits, n), t)


def test_thread_count_does_not_change_the_result():
    inst = configs.config3(1024)
    a, la, _ = bitset.closure(inst.n, inst.edges, inst.grammar, threads=1)
    b, lb, _ = bitset.closure(inst.n, inst.edges, inst.grammar, threads=4)
    assert la == lb and np.array_equal(a, b)
    assert np.array_equal(a, worklist.closure(inst.n, inst.edges, inst.grammar))


@pytest.mark.parametrize("n", [1, 64, 65, 200])
def test_product_against_float_matmul(n):
    rng = np.random.default_rng(n)
    b = rng.random((n, n)) < 0.1
    c = rng.random((n, n)) < 0.1
    a0 = rng.random((n, n)) < 0.05
    B, C, A = (worklist.pack(x) for x in (b, c, a0))
    bitset.product(n, B, C, A)
    assert np.array_equal(worklist.unpack(A, n), a0 | alg1.bool_product(b, c))
    # a row range touches only those rows of A
    A2 = worklist.pack(a0)
    r0, r1 = n // 3, (2 * n) // 3
    bitset.product(n, B, C, A2, rows=(r0, r1))
    want = a0.copy()
    want[r0:r1] |= alg1.bool_product(b[r0:r1], c)
    assert np.array_equal(worklist.unpack(A2, n), want)


def test_empty_and_invalid():
    g = grammars.dyck()
    bits, loops, rc = bitset.closure(0, np.zeros((0, 3), np.int32), g)
    assert rc == 0 and bits.shape[1] == 0
    bits, loops, rc = bitset.closure(5, np.zeros((0, 3), np.int32), g)
    assert rc == 0 and loops == 1 and not bits.any()
    with pytest.raises(ValueError):
        bitset.closure(4, np.array([[0, 0, 4]], np.int32), g)
    with pytest.raises(ValueError):
        bitset.closure(4, np.array([[0, 7, 1]], np.int32), g)


MUTANTS = {
    "in_place_products": ("product_rows(n, W, out + (size_t)b * mat, out + (size_t)c * mat, next + (size_t)a * mat, 0, n);",
                          "product_rows(n, W, next + (size_t)b * mat, next + (size_t)c * mat, next + (size_t)a * mat, 0, n);"),
    "or_becomes_copy": ("dst[j] |= src[j];", "dst[j] = src[j];"),
    "bit_off_by_one": ("const int64_t k = kw * 64 + __builtin_ctzll(bits);",
                       "const int64_t k = kw * 64 + __builtin_ctzll(bits) + 1;"),
    "first_word_skipped": ("for (int64_t kw = 0; kw < W; ++kw) {", "for (int64_t kw = 1; kw < W; ++kw) {"),
    "operands_swapped": ("out + (size_t)b * mat, out + (size_t)c * mat, next", "out + (size_t)c * mat, out + (size_t)b * mat, next"),
    "first_rule_only": ("for (int32_t r = 0; r < n_bin; ++r) {\n            const int32_t a = bin[3 * r]",
                        "for (int32_t r = 0; r < 1 && r < n_bin; ++r) {\n            const int32_t a = bin[3 * r]"),
    "reversed_edges": ("out[(size_t)term[2 * r] * mat + (size_t)i * W + j / 64] |= 1ull << (j % 64);",
                       "out[(size_t)term[2 * r] * mat + (size_t)j * W + i / 64] |= 1ull << (i % 64);"),
    "last_loop_not_counted": ("        ++loops;\n        const int changed", "        const int changed"),
    "stops_one_loop_early": ("if (!changed) break;", "if (!changed || loops > 1) break;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(bitset._SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    lib = bitset.load_library(bitset.build(True, str(path), str(tmp_path / f"libmut_{name}.so")))
    try:
        held = _pins_hold(lib)
    except (ValueError, IndexError, AssertionError):
        held = False
    assert not held, f"mutant {name} passed every pin"
