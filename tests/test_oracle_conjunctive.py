"""Pins for the conjunctive-grammar oracle.

Conjunctive CYK against the language definition of {a^n b^n c^n}; the matrix
closure against conjunctive CYK on chains (one path between two nodes, so the
closure is exact there), against the relational oracle when every rule has
one conjunct, against the intersection of two relational closures for a
grammar whose start rules conjoin two context-free grammars, and as an upper
bound of brute-force path enumeration on tiny graphs.  A small mutation
harness checks that planted mistakes break a pin.
"""
from __future__ import annotations

import itertools
import os
import types

import numpy as np
import pytest

from oracle import alg1, brute, conjunctive, worklist
from workloads import grammars, graphs


def _is_anbncn(word):
    k = len(word) // 3
    return k >= 1 and len(word) == 3 * k and word == [0] * k + [1] * k + [2] * k


def test_conj_cyk_is_the_language_definition():
    g = grammars.anbncn()
    S = g.nt("S")
    for L in range(1, 9):
        for word in itertools.product(range(3), repeat=L):
            word = list(word)
            assert (S in brute.conj_cyk_table(word, g)[0][L]) == _is_anbncn(word), word


def test_conj_cyk_with_one_conjunct_is_cyk():
    g = grammars.dyck()
    cg = grammars.conjunctive_from_cnf(g)
    rng = np.random.default_rng(3)
    for _ in range(30):
        word = [int(x) for x in rng.integers(0, 2, int(rng.integers(1, 12)))]
        a, b = brute.cyk_table(word, g), brute.conj_cyk_table(word, cg)
        assert all(a[s][e] == b[s][e] for s in range(len(word)) for e in range(s + 1, len(word) + 1))


def _chain_matches_cyk(mod, g, word) -> bool:
    n, e = graphs.chain(word)
    t, _ = mod.closure(n, e, g)
    tab = brute.conj_cyk_table(word, g)
    for s in range(len(word)):
        for end in range(s + 1, len(word) + 1):
            got = {a for a in range(g.n_nonterminals) if t[a, s, end]}
            if got != tab[s][end]:
                return False
    return True


def _pins_hold(mod) -> bool:
    g = grammars.anbncn()
    for word in ([0, 0, 1, 1, 2, 2], [0, 1, 2, 0, 0, 1, 1, 2, 2, 2], [0, 0, 1, 2, 2, 1, 0, 1, 2]):
        if not _chain_matches_cyk(mod, g, word):
            return False
    # one conjunct per rule: Algorithm 1 exactly
    n, e = graphs.erdos_renyi(40, 100, 8, labels=2)
    t, loops = mod.closure(n, e, grammars.conjunctive_from_cnf(grammars.dyck()))
    t1, loops1, _ = alg1.closure(n, e, grammars.dyck())
    if loops != loops1 or not np.array_equal(t, t1):
        return False
    # start rules conjoining Dyck and a^n b^n: R_S = R_Dyck & R_anbn
    g2 = grammars.dyck_and_anbn()
    t, _ = mod.closure(n, e, g2)
    d = worklist.unpack(worklist.closure(n, e, grammars.dyck()), n)[0]
    ab = worklist.unpack(worklist.closure(n, e, grammars.anbn()), n)[0]
    return bool(np.array_equal(t[g2.nt("S")], d & ab))


def test_closure_on_chains_equals_conjunctive_cyk():
    g = grammars.anbncn()
    rng = np.random.default_rng(4)
    words = [[0] * k + [1] * k + [2] * k for k in (1, 2, 5)]
    words += [[int(x) for x in rng.integers(0, 3, 14)] for _ in range(6)]
    words.append([0, 0, 0, 1, 1, 1, 2, 2, 2, 0, 1, 2])
    for w in words:
        assert _chain_matches_cyk(conjunctive, g, w), w


def test_one_conjunct_rules_equal_algorithm_1():
    for seed in range(3):
        n, e = graphs.erdos_renyi(50, 130, 20 + seed, labels=2)
        for g in (grammars.dyck(), grammars.anbn()):
            t, loops = conjunctive.closure(n, e, grammars.conjunctive_from_cnf(g))
            t1, loops1, _ = alg1.closure(n, e, g)
            assert loops == loops1 and np.array_equal(t, t1)
            assert np.array_equal(t, worklist.unpack(worklist.closure(n, e, g), n))


def test_conjoined_start_rules_give_the_intersection():
    g2 = grammars.dyck_and_anbn()
    for seed in range(3):
        n, e = graphs.erdos_renyi(60, 150, 30 + seed, labels=2)
        t, _ = conjunctive.closure(n, e, g2)
        d = worklist.unpack(worklist.closure(n, e, grammars.dyck()), n)[0]
        ab = worklist.unpack(worklist.closure(n, e, grammars.anbn()), n)[0]
        assert np.array_equal(t[g2.nt("S")], d & ab)


def test_closure_bounds_every_conjunctive_path_from_above():
    """Every path whose label word the conjunctive grammar derives is in the
    closure (the over-approximation contains the exact answer)."""
    g = grammars.anbncn()
    for seed in range(4):
        n, e = graphs.random_tiny(6, 12, 3, 700 + seed)
        t, _ = conjunctive.closure(n, e, g)
        exact = brute.conj_paths_up_to(n, e, g, 6)
        for a, pairs in exact.items():
            for i, j in pairs:
                assert t[a, i, j], (seed, a, i, j)


def test_real_oracle_passes_harness():
    assert _pins_hold(conjunctive)


CJ_MUTANTS = {
    "or_across_conjuncts": ("            acc = np.ones((n, n), dtype=bool)\n            for b, c in parts:\n"
                            "                acc &= bool_product(t[b], t[c])",
                            "            acc = np.zeros((n, n), dtype=bool)\n            for b, c in parts:\n"
                            "                acc |= bool_product(t[b], t[c])"),
    "first_conjunct_only": ("            for b, c in parts:\n                acc &= bool_product(t[b], t[c])",
                            "            for b, c in parts[:1]:\n                acc &= bool_product(t[b], t[c])"),
    "transposed_product": ("acc &= bool_product(t[b], t[c])", "acc &= bool_product(t[c], t[b])"),
    "no_union_with_old": ("            new[a] |= acc", "            new[a] = acc"),
}


@pytest.mark.parametrize("name", sorted(CJ_MUTANTS))
def test_conjunctive_mutant_is_caught(name):
    old, new = CJ_MUTANTS[name]
    src = open(conjunctive.__file__).read()
    assert src.count(old) == 1, name
    mod = types.ModuleType(f"mutant_{name}")
    exec(compile(src.replace(old, new), os.path.basename(conjunctive.__file__), "exec"), mod.__dict__)
    assert not _pins_hold(mod), f"mutant {name} passed every pin"
