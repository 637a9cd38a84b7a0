"""Pins of the CPU oracle against values and facts fixed by the paper and by
plain mathematics (no GPU).  Each test names what it pins."""
from __future__ import annotations

import json
import os
from collections import deque

import numpy as np
import pytest

from oracle import alg1, brute, worklist
from workloads import configs, grammars, graphs
from tests.helpers import closed_under_rules, contains_init, rel_from_dense

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def _dense_from_rows(rows, g):
    n = len(rows)
    t = np.zeros((g.n_nonterminals, n, n), dtype=bool)
    for i, r in enumerate(rows):
        for j, cell in enumerate(r):
            for name in cell:
                t[g.nt(name), i, j] = True
    return t


# ---------------------------------------------------------------- worked example

def test_worked_example_relations_worklist():
    """All seven R_A printed in section 4.3 (context-free relations figure)."""
    gold = _golden()["relations"]
    inst = configs.worked_example()
    bits = worklist.closure(inst.n, inst.edges, inst.grammar)
    rel = worklist.relations(bits, inst.n)
    for name in inst.grammar.nonterminals:
        assert rel[inst.grammar.nt(name)] == {tuple(p) for p in gold[name]}, name


def test_worked_example_every_state_alg1():
    """T0, T0 x T0, T1..T5 and the loop count k = 6 printed in section 4.3."""
    gold = _golden()
    inst = configs.worked_example()
    g = inst.grammar
    t, loops, hist = alg1.closure(inst.n, inst.edges, g, keep_history=True)
    assert np.array_equal(hist[0], _dense_from_rows(gold["T0"]["rows"], g))
    assert np.array_equal(alg1.matrix_product(hist[0], g), _dense_from_rows(gold["T0xT0"]["rows"], g))
    for st in gold["T"]:
        assert np.array_equal(hist[st["k"]], _dense_from_rows(st["rows"], g)), st["k"]
    assert loops == gold["loops"]["k"] == 6
    assert np.array_equal(hist[6], hist[5])
    rel = rel_from_dense(t)
    for name in g.nonterminals:
        assert rel[g.nt(name)] == {tuple(p) for p in gold["relations"][name]}


def test_worked_example_graph_recovery_is_unique():
    """The graph used for the example is the only one (over the example's four
    labels) whose initial matrix is the printed T0: with one-to-one terminal
    rules, each set bit of T0 names exactly one edge."""
    gold = _golden()
    inst = configs.worked_example()
    g = inst.grammar
    t0 = _dense_from_rows(gold["T0"]["rows"], g)
    term_of = {a: x for a, x in g.term}
    rebuilt = sorted((i, term_of[a], j) for a, i, j in zip(*np.nonzero(t0)))
    assert rebuilt == sorted(tuple(int(v) for v in e) for e in inst.edges)


# ---------------------------------------------------------------- two cycles (closed form)

def _two_cycle_expected():
    """Closed form for a^n b^n on an a-cycle of 64 and a b-cycle of 63 nodes
    sharing node 0.  The b-edges only leave nodes of the b-cycle, so an a^n b^n
    path from i must reach node 0 after its n a-steps: n = -i (mod 64); the n
    b-steps then end at b-cycle position n mod 63.  gcd(64, 63) = 1, so by the
    Chinese remainder theorem every (a-node, b-node) pair has such an n >= 1.
    S1 derives a^n b^(n+1): the same argument with n + 1 b-steps."""
    a_nodes = list(range(64))
    b_cycle = [0] + list(range(64, 126))
    pos = {v: p for p, v in enumerate(b_cycle)}
    s_min, s1_min = {}, {}
    for i in a_nodes:
        for j in b_cycle:
            s_min[(i, j)] = next(n for n in range(1, 4033) if (i + n) % 64 == 0 and n % 63 == pos[j])
            s1_min[(i, j)] = next(n for n in range(1, 4033) if (i + n) % 64 == 0 and (n + 1) % 63 == pos[j])
    return s_min, s1_min


def test_two_cycles_closed_form():
    inst = configs.config1()
    g = inst.grammar
    s_min, s1_min = _two_cycle_expected()
    rel = worklist.relations(worklist.closure(inst.n, inst.edges, g), inst.n)
    pairs = set(s_min)
    assert len(pairs) == 4032
    assert rel[g.nt("S")] == pairs
    assert rel[g.nt("S1")] == pairs
    assert rel[g.nt("A")] == {(i, (i + 1) % 64) for i in range(64)}
    assert len(rel[g.nt("B")]) == 63


@pytest.mark.slow
def test_two_cycles_jacobi_loop_count():
    """Lemma 3: after loop k, T holds exactly the triples whose minimal
    derivation tree has height <= k + 1.  With S -> A S1 | A B, S1 -> S B,
    a^n b^n needs height 2n and a^n b^(n+1) (S1) height 2n + 1, so the last
    triple appears in loop H_max - 1 and one more loop confirms the fixpoint:
    H_max loops in total.  H_max comes from the closed form above (8065)."""
    inst = configs.config1()
    s_min, s1_min = _two_cycle_expected()
    h_max = max(max(2 * v for v in s_min.values()), max(2 * v + 1 for v in s1_min.values()), 1)
    assert h_max == 8065
    t, loops, _ = alg1.closure(inst.n, inst.edges, inst.grammar)
    assert loops == h_max
    bits = worklist.closure(inst.n, inst.edges, inst.grammar)
    assert np.array_equal(worklist.unpack(bits, inst.n), t)


# ---------------------------------------------------------------- textbook special cases

def _bfs_closure(n, pairs):
    adj = [[] for _ in range(n)]
    for u, v in pairs:
        adj[u].append(v)
    out = set()
    for s in range(n):
        seen = set()
        dq = deque(adj[s])
        while dq:
            v = dq.popleft()
            if v in seen:
                continue
            seen.add(v)
            dq.extend(adj[v])
        out |= {(s, v) for v in seen}
    return out


@pytest.mark.parametrize("seed", range(6))
def test_transitive_closure_grammar_is_bfs(seed):
    """S -> S S | a: R_S is the set of pairs joined by a non-empty a-path,
    computed here by breadth-first search."""
    n = 40
    _, e = graphs.erdos_renyi(n, 60, seed, labels=2)
    g = grammars.transitive_closure()
    rel = worklist.relations(worklist.closure(n, e, g), n)
    want = _bfs_closure(n, [(int(u), int(v)) for u, x, v in e if x == 0])
    assert rel[0] == want


@pytest.mark.parametrize("name,seed", [(nm, s) for nm in ("dyck", "anbn", "same_generation", "adjacent_layers") for s in range(3)])
def test_chain_graph_is_cyk_table(name, seed):
    """On a chain labelled w, (i, j) in R_A iff A =>* w[i:j]: the CYK table
    (the setting of Valiant's algorithm, section 2)."""
    g = grammars.BY_NAME[name]()
    rng = np.random.default_rng(100 + seed)
    word = [int(x) for x in rng.integers(0, g.n_terminals, size=14)]
    n, e = graphs.chain(word)
    rel = worklist.relations(worklist.closure(n, e, g), n)
    tab = brute.cyk_table(word, g)
    for a in range(g.n_nonterminals):
        want = {(s, t) for s in range(n) for t in range(s + 1, n) if a in tab[s][t]}
        assert rel[a] == want


@pytest.mark.parametrize("seed", range(4))
def test_dyck_on_chain_is_bracket_matching(seed):
    """Dyck on a chain: w[i:j] is a non-empty balanced bracket word iff the
    running balance never drops below zero and ends at zero."""
    rng = np.random.default_rng(200 + seed)
    word = [int(x) for x in rng.integers(0, 2, size=40)]
    n, e = graphs.chain(word)
    g = grammars.dyck()
    rel = worklist.relations(worklist.closure(n, e, g), n)
    want = set()
    for i in range(n):
        bal = 0
        for j in range(i, n - 1):
            bal += 1 if word[j] == 0 else -1
            if bal < 0:
                break
            if bal == 0:
                want.add((i, j + 1))
    assert rel[g.nt("S")] == want


def test_terminal_only_grammar_is_edge_set():
    n, e = graphs.erdos_renyi(50, 200, 7, labels=3)
    from workloads.grammars import CNF
    g = CNF(("X", "Y", "Z"), ("p", "q", "r"), ((0, 0), (0, 1), (1, 2)), (), "terminal_only")
    rel = worklist.relations(worklist.closure(n, e, g), n)
    assert rel[0] == {(int(u), int(v)) for u, x, v in e if x in (0, 1)}
    assert rel[1] == {(int(u), int(v)) for u, x, v in e if x == 2}
    assert rel[2] == set()


def test_empty_inputs():
    g = grammars.dyck()
    assert worklist.closure(0, np.zeros((0, 3), np.int32), g).shape == (4, 0, 1)
    bits = worklist.closure(5, np.zeros((0, 3), np.int32), g)
    assert not bits.any()


# ---------------------------------------------------------------- brute force on tiny graphs

TINY_GRAMMARS = ["dyck", "anbn", "same_generation", "adjacent_layers", "transitive_closure"]


@pytest.mark.parametrize("name,seed", [(nm, s) for nm in TINY_GRAMMARS for s in range(4)])
def test_tiny_dag_equals_path_enumeration(name, seed):
    """On a DAG every path has at most n - 1 edges, so enumerating all paths
    and testing each label word by CYK gives R_A exactly."""
    g = grammars.BY_NAME[name]()
    n, e = graphs.random_tiny(7, 14, g.n_terminals, 300 + seed, acyclic=True)
    want = brute.paths_up_to(n, e, g, n - 1)
    got = worklist.relations(worklist.closure(n, e, g), n)
    assert got == want


@pytest.mark.parametrize("name,seed", [(nm, s) for nm in TINY_GRAMMARS for s in range(4)])
def test_tiny_cyclic_graphs(name, seed):
    """Cyclic tiny graphs (self-loops and multi-edges included).  Paths of at
    most L edges give a subset of R_A for every L; the oracle result contains
    the initial matrix and is closed under every rule, so it contains the least
    such set, R_A.  With all witness paths short the two meet: equality at
    L = 10 on these cases."""
    g = grammars.BY_NAME[name]()
    n, e = graphs.random_tiny(4, 7, g.n_terminals, 400 + seed)
    bits = worklist.closure(n, e, g)
    dense = worklist.unpack(bits, n)
    assert contains_init(dense, n, e, g)
    assert closed_under_rules(dense, g)
    got = rel_from_dense(dense)
    for L in (1, 3, 6):
        low = brute.paths_up_to(n, e, g, L)
        assert all(low[a] <= got[a] for a in got)
    assert brute.paths_up_to(n, e, g, 10) == got


# ---------------------------------------------------------------- invariants

@pytest.mark.parametrize("name", ["dyck", "same_generation", "anbn"])
def test_worklist_equals_algorithm1(name):
    """Two independent routes to the same least fixpoint (Theorem 2)."""
    g = grammars.BY_NAME[name]()
    if g.terminals == grammars.HIERARCHY_TERMINALS:
        n, e = graphs.erdos_renyi_hier_labels(90, 150, 11)
    else:
        n, e = graphs.erdos_renyi(90, 200, 11)
    t, _, _ = alg1.closure(n, e, g)
    assert np.array_equal(worklist.unpack(worklist.closure(n, e, g), n), t)


def test_monotone_in_edges():
    """Adding edges never removes a pair (each loop only adds, Theorem 3)."""
    g = grammars.dyck()
    n, e = graphs.erdos_renyi(60, 150, 12)
    small = worklist.unpack(worklist.closure(n, e[:100], g), n)
    big = worklist.unpack(worklist.closure(n, e, g), n)
    assert not (small & ~big).any()


def test_node_permutation_equivariance():
    g = grammars.dyck()
    n, e = graphs.erdos_renyi(70, 160, 13)
    perm = np.random.default_rng(5).permutation(n)
    e2 = e.copy()
    e2[:, 0] = perm[e[:, 0]]
    e2[:, 2] = perm[e[:, 2]]
    a = worklist.unpack(worklist.closure(n, e, g), n)
    b = worklist.unpack(worklist.closure(n, e2, g), n)
    # node u of the first graph is node perm[u] of the second
    assert np.array_equal(b[:, perm][:, :, perm], a)
    assert a.any()


def test_disjoint_union_is_block_diagonal():
    """Two graphs side by side: the result is the two results on the diagonal
    blocks and nothing across them."""
    g = grammars.dyck()
    n1, e1 = graphs.erdos_renyi(50, 120, 14)
    n2, e2 = graphs.erdos_renyi(37, 90, 15)
    e2s = e2.copy()
    e2s[:, 0] += n1
    e2s[:, 2] += n1
    both = worklist.unpack(worklist.closure(n1 + n2, np.concatenate([e1, e2s]), g), n1 + n2)
    r1 = worklist.unpack(worklist.closure(n1, e1, g), n1)
    r2 = worklist.unpack(worklist.closure(n2, e2, g), n2)
    assert np.array_equal(both[:, :n1, :n1], r1)
    assert np.array_equal(both[:, n1:, n1:], r2)
    assert not both[:, :n1, n1:].any() and not both[:, n1:, :n1].any()


@pytest.mark.parametrize("seed", range(3))
def test_valiant_closure_matches(seed):
    """Theorem 1: a^+ = a^cf.  Valiant's union over path lengths, cut at 12,
    is inside a^cf and equal to it on these tiny graphs."""
    g = grammars.dyck()
    n, e = graphs.random_tiny(4, 7, 2, 500 + seed)
    cf, _, _ = alg1.closure(n, e, g)
    plus = alg1.valiant_plus(n, e, g, 12)
    assert not (plus & ~cf).any()
    assert np.array_equal(plus, cf)


def test_pack_unpack_roundtrip():
    rng = np.random.default_rng(0)
    d = rng.random((3, 70, 70)) < 0.3
    assert np.array_equal(worklist.unpack(worklist.pack(d), 70), d)
