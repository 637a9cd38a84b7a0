"""The oracle's pins must catch plausible mistakes in it.

Each case plants one mistake in a copy of the oracle's C source (a dropped
term, a wrong index, a transposed operand, a missed case), builds the copy with
gcc in a temporary directory, and checks that at least one pin fails on it:
the worked example of section 4.3, the two-cycle closed form, or brute force on
tiny graphs.  The real oracle is untouched; nothing here runs on a GPU.
"""
from __future__ import annotations

import json
import os
import subprocess

import pytest

from oracle import brute, worklist
from tests.test_oracle_pins import _bfs_closure
from workloads import configs, grammars, graphs

SRC = os.path.join(os.path.dirname(worklist.__file__), "cfpq_worklist.c")

MUTANTS = {
    "dropped_negation": ("uint64_t fresh = cj[w] & ~ai[w];", "uint64_t fresh = cj[w] & ai[w];"),
    "right_branch_missing": ("if (c == x) {", "if (0) {"),
    "left_branch_missing": ("if (b == x) {", "if (0) {"),
    "transposed_left_operand": ("const uint64_t *cj = row_of(s.fwd, &s, c, j);",
                                "const uint64_t *cj = row_of(s.bwd, &s, c, j);"),
    "wrong_rule_operand": ("const uint64_t *bi = row_of(s.bwd, &s, b, i);",
                           "const uint64_t *bi = row_of(s.bwd, &s, c, i);"),
    "swapped_result_index": ("insert(&s, a, (int32_t)(w * 64 + k), j);",
                             "insert(&s, a, j, (int32_t)(w * 64 + k));"),
    "first_terminal_rule_only": ("if (term[2 * r + 1] == t[1]) insert(&s, term[2 * r], t[0], t[2]);",
                                 "if (term[2 * r + 1] == t[1]) { insert(&s, term[2 * r], t[0], t[2]); break; }"),
    "reversed_edges": ("insert(&s, term[2 * r], t[0], t[2]);", "insert(&s, term[2 * r], t[2], t[0]);"),
    "off_by_one_word": ("for (int64_t w = 0; w < s.words; ++w) {\n                    uint64_t fresh = cj[w]",
                        "for (int64_t w = 1; w < s.words; ++w) {\n                    uint64_t fresh = cj[w]"),
}


def _pins_hold(lib) -> bool:
    """True if every pin passes for the library ``lib``."""
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")))
    inst = configs.worked_example()
    rel = worklist.relations(worklist.closure(inst.n, inst.edges, inst.grammar, lib=lib), inst.n)
    for name in inst.grammar.nonterminals:
        if rel[inst.grammar.nt(name)] != {tuple(p) for p in gold["relations"][name]}:
            return False
    c1 = configs.config1()
    rel = worklist.relations(worklist.closure(c1.n, c1.edges, c1.grammar, lib=lib), c1.n)
    want = {(i, j) for i in range(64) for j in [0] + list(range(64, 126))}
    if rel[0] != want or rel[1] != want:
        return False
    # multi-edge / several rules per terminal, large enough for several words per row
    g = grammars.CNF(("S", "X", "Y"), ("a", "b"), ((1, 0), (2, 0), (2, 1)), ((0, 1, 2), (0, 0, 0)), "mut")
    for seed in range(3):
        n, e = graphs.random_tiny(6, 12, 2, 900 + seed, acyclic=True)
        if worklist.relations(worklist.closure(n, e, g, lib=lib), n) != brute.paths_up_to(n, e, g, n - 1):
            return False
    # several words per row: transitive closure against breadth-first search
    n, e = graphs.erdos_renyi(150, 200, 901, labels=2)
    got = worklist.relations(worklist.closure(n, e, grammars.transitive_closure(), lib=lib), n)
    return got[0] == _bfs_closure(n, [(int(u), int(v)) for u, x, v in e if x == 0])


def test_real_oracle_passes_mutation_harness():
    assert _pins_hold(None)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / f"libmut_{name}.so"
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-o", str(so), str(path)])
    lib = worklist.load_library(str(so))
    try:
        caught = not _pins_hold(lib)
    except (ValueError, MemoryError):
        caught = True
    assert caught, f"mutant {name} passed every pin"
