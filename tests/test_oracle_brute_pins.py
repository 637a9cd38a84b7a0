"""Pins for the two enumeration helpers of ``oracle.brute`` that serve as
language and path oracles: ``cfg_words`` (every short word each nonterminal
of a general context-free grammar derives, the definition of L(A) of
section 2) and ``conj_paths_up_to`` (every pair joined by a short path whose
word a conjunctive grammar derives, the set the conclusion's remark says the
conjunctive closure over-approximates).

Each is checked against results fixed by the mathematics, not by another
oracle function:

* ``cfg_words`` against languages known in closed form -- a^n b^n, balanced
  brackets, equal letter counts, palindromes, even / odd lengths through
  mutual recursion, and a unit cycle with nullable symbols whose language is
  worked out by hand ({a^k, a^k c});
* ``conj_paths_up_to`` against Boolean matrix powers: a path i -> j spells
  a^n b^n c^n iff (M_a^n M_b^n M_c^n)[i, j] for the adjacency matrices of the
  three labels, so the pairs of {a^n b^n c^n} and of Dyck AND a^n b^n (which
  is a^n b^n) up to a length bound are unions of such products; on a chain it
  must equal the conjunctive CYK table, and with one conjunct per rule the
  plain path enumeration.

A mutation harness plants plausible mistakes in copies of the two functions
(reversed concatenation, a strict length bound, a dropped empty word, a single
pass, a wrong end node, ...) and checks that a pin catches each.
"""
from __future__ import annotations

import itertools
import os
import types

import numpy as np
import pytest

from oracle import brute
from workloads import grammars, graphs

BRUTE_SRC = brute.__file__


# ---------------------------------------------------------------- cfg_words

def _all_words(alphabet, max_len):
    for L in range(0, max_len + 1):
        for w in itertools.product(alphabet, repeat=L):
            yield w


def _balanced(w, open_="a", close="b"):
    depth = 0
    for x in w:
        depth += 1 if x == open_ else -1
        if depth < 0:
            return False
    return depth == 0


# (rules, alphabet, max_len, {nonterminal: membership predicate})
CFG_CASES = {
    "anbn_nullable": (
        {"S": [("a", "S", "b"), ()]}, "ab", 8,
        {"S": lambda w: len(w) % 2 == 0 and w == ("a",) * (len(w) // 2) + ("b",) * (len(w) // 2)}),
    "dyck_nullable": (
        {"S": [("a", "S", "b", "S"), ()]}, "ab", 8,
        {"S": _balanced}),
    "dyck_nonempty": (
        {"S": [("S", "S"), ("a", "S", "b"), ("a", "b")]}, "ab", 8,
        {"S": lambda w: len(w) > 0 and _balanced(w)}),
    "equal_counts": (
        {"S": [("a", "S", "b", "S"), ("b", "S", "a", "S"), ()]}, "ab", 8,
        {"S": lambda w: w.count("a") == w.count("b")}),
    "palindromes": (
        {"S": [("a", "S", "a"), ("b", "S", "b"), ("a",), ("b",), ()]}, "ab", 7,
        {"S": lambda w: w == w[::-1]}),
    "even_odd": (
        {"E": [("a", "O"), ()], "O": [("a", "E")]}, "a", 9,
        {"E": lambda w: len(w) % 2 == 0, "O": lambda w: len(w) % 2 == 1}),
    # S -> A | c, A -> B, B -> S | a A | eps: each of S, A, B derives exactly
    # eps, c and every word a^k or a^k c (the least set holding eps and c and
    # closed under putting an a in front).
    "unit_cycle_nullable": (
        {"S": [("A",), ("c",)], "A": [("B",)], "B": [("S",), ("a", "A"), ()]}, "ac", 6,
        {x: (lambda w: "c" not in w[:-1] and all(y == "a" for y in w if y != "c") and w.count("c") <= 1)
         for x in "SAB"}),
}


def _cfg_pins_hold(cfg_words) -> bool:
    for rules, alphabet, max_len, member in CFG_CASES.values():
        got = cfg_words(rules, max_len)
        for a, pred in member.items():
            want = {w for w in _all_words(alphabet, max_len) if pred(w)}
            if got[a] != want:
                return False
    return True


@pytest.mark.parametrize("case", sorted(CFG_CASES))
def test_cfg_words_closed_form(case):
    rules, alphabet, max_len, member = CFG_CASES[case]
    got = brute.cfg_words(rules, max_len)
    for a, pred in member.items():
        want = {w for w in _all_words(alphabet, max_len) if pred(w)}
        assert got[a] == want, (case, a, sorted(got[a] ^ want)[:5])


def test_cfg_words_counts():
    """Number of balanced words of length 2m is the Catalan number C_m."""
    got = brute.cfg_words({"S": [("a", "S", "b", "S"), ()]}, 12)["S"]
    catalan = [1, 1, 2, 5, 14, 42, 132]
    for m in range(7):
        assert sum(1 for w in got if len(w) == 2 * m) == catalan[m]


# ---------------------------------------------------------------- conj_paths_up_to

def _adj(n, edges, label):
    m = np.zeros((n, n), dtype=np.int64)
    for u, x, v in edges:
        if x == label:
            m[u, v] = 1
    return m


def _bool_power(m, k):
    out = np.eye(m.shape[0], dtype=np.int64)
    for _ in range(k):
        out = ((out @ m) > 0).astype(np.int64)
    return out


def _pairs_of_power_words(n, edges, labels, max_len):
    """{(i, j)}: some path i -> j spells x1^k x2^k ... (labels in order) for a
    k >= 1 with len(labels) * k <= max_len, from Boolean matrix powers."""
    mats = [_adj(n, edges, x) for x in labels]
    out = set()
    for k in range(1, max_len // len(labels) + 1):
        prod = np.eye(n, dtype=np.int64)
        for m in mats:
            prod = ((prod @ _bool_power(m, k)) > 0).astype(np.int64)
        out |= set(zip(*(x.tolist() for x in np.nonzero(prod))))
    return out


def _conj_pins_hold(conj_paths_up_to) -> bool:
    g3 = grammars.anbncn()
    g2 = grammars.dyck_and_anbn()
    for seed in range(4):
        n, e = graphs.random_tiny(5, 15, 3, 300 + seed)
        got = conj_paths_up_to(n, e, g3, 6)
        if got[g3.nt("S")] != _pairs_of_power_words(n, e, [0, 1, 2], 6):
            return False
        n, e = graphs.random_tiny(5, 10, 2, 400 + seed)
        got = conj_paths_up_to(n, e, g2, 6)
        if got[g2.nt("S")] != _pairs_of_power_words(n, e, [0, 1], 6):
            return False
    # chains: the pairs are the conjunctive CYK table of the word
    for word in ([0, 0, 1, 1, 2, 2], [0, 1, 2, 0, 0, 1, 1, 2, 2], [2, 0, 1, 2, 1, 0]):
        n, e = graphs.chain(word)
        got = conj_paths_up_to(n, e, g3, len(word))
        tab = brute.conj_cyk_table(word, g3)
        for a in range(g3.n_nonterminals):
            want = {(s, t) for s in range(len(word)) for t in range(s + 1, len(word) + 1) if a in tab[s][t]}
            if got[a] != want:
                return False
    # one conjunct per rule: the plain path enumeration
    for seed in range(3):
        n, e = graphs.random_tiny(5, 9, 2, 500 + seed)
        g = grammars.dyck()
        if conj_paths_up_to(n, e, grammars.conjunctive_from_cnf(g), 5) != brute.paths_up_to(n, e, g, 5):
            return False
    return True


def test_conj_paths_anbncn_matches_matrix_powers():
    g = grammars.anbncn()
    for seed in range(6):
        n, e = graphs.random_tiny(5, 15, 3, 300 + seed)
        got = brute.conj_paths_up_to(n, e, g, 6)[g.nt("S")]
        assert got == _pairs_of_power_words(n, e, [0, 1, 2], 6), seed


def test_conj_paths_dyck_and_anbn_matches_matrix_powers():
    g = grammars.dyck_and_anbn()
    for seed in range(6):
        n, e = graphs.random_tiny(5, 10, 2, 400 + seed)
        got = brute.conj_paths_up_to(n, e, g, 6)[g.nt("S")]
        assert got == _pairs_of_power_words(n, e, [0, 1], 6), seed


def test_conj_paths_harness_on_real_functions():
    assert _conj_pins_hold(brute.conj_paths_up_to)
    assert _cfg_pins_hold(brute.cfg_words)


# ---------------------------------------------------------------- mutation harness

CFG_MUTANTS = {
    "reversed_concatenation": ("partial = {p + q for p in partial", "partial = {q + p for p in partial"),
    "strict_length_bound": ("if len(p) + len(q) <= max_len}", "if len(p) + len(q) < max_len}"),
    "empty_word_dropped": ("                partial = {()}\n", "                partial = {()} if alt else set()\n"),
    "single_pass": ("                    changed = True\n", "                    changed = False\n"),
    "first_alternative_only": ("            for alt in alts:\n                partial = {()}",
                               "            for alt in alts[:1]:\n                partial = {()}"),
    "symbols_all_terminal": ("opts = words[x] if x in rules else {(x,)}", "opts = {(x,)}"),
}

CONJ_MUTANTS = {
    "length_bound_off_by_one": ("        if len(word) == max_len:\n            return\n        for x, v in out_edges",
                                "        if len(word) == max_len - 1:\n            return\n        for x, v in out_edges"),
    "records_current_node": ("            for a in conj_cyk_table(word, grammar)[0][len(word)]:\n"
                             "                result[a].add((start, v))",
                             "            for a in conj_cyk_table(word, grammar)[0][len(word)]:\n"
                             "                result[a].add((start, node))"),
    "last_letter_only": ("conj_cyk_table(word, grammar)[0][len(word)]",
                         "conj_cyk_table(word, grammar)[len(word) - 1][len(word)]"),
    "start_not_recorded": ("        walk(start, start, [])", "        walk(0, start, [])"),
}


def _mutant_module(old: str, new: str):
    src = open(BRUTE_SRC).read()
    assert src.count(old) == 1, f"mutation site not found exactly once: {old!r}"
    mod = types.ModuleType("brute_mutant")
    exec(compile(src.replace(old, new), os.path.basename(BRUTE_SRC), "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name", sorted(CFG_MUTANTS))
def test_cfg_words_mutant_is_caught(name):
    mod = _mutant_module(*CFG_MUTANTS[name])
    assert not _cfg_pins_hold(mod.cfg_words), f"mutant {name} passed every pin"


@pytest.mark.parametrize("name", sorted(CONJ_MUTANTS))
def test_conj_paths_mutant_is_caught(name):
    mod = _mutant_module(*CONJ_MUTANTS[name])
    try:
        caught = not _conj_pins_hold(mod.conj_paths_up_to)
    except (RecursionError, IndexError):
        caught = True
    assert caught, f"mutant {name} passed every pin"
