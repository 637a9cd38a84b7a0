"""Pins for the single-path oracle (section 5 lengths and witnesses).

Pinned against: Algorithm 1 (the relation and the loop count are those of the
relational closure), breadth-first search (S -> S S | a gives shortest path
lengths), a chain (every path i -> j has j - i edges), the two-cycle closed
form (a^m b^m with m fixed by the Chinese remainder theorem), a hand-built
graph where the first length found is not the shortest one (the section's
"never changed afterwards"), and CYK on every witness path.  A small mutation
harness checks that each planted mistake in the oracle breaks one of them.
"""
from __future__ import annotations

import collections
import os
import types

import numpy as np
import pytest

from oracle import alg1, brute, single_path
from workloads import configs, grammars, graphs


def _bfs_lengths(n, pairs):
    """d[i][j] = fewest edges (>= 1) on a path i -> j, 0 if none."""
    adj = collections.defaultdict(list)
    for u, v in pairs:
        adj[u].append(v)
    d = np.zeros((n, n), dtype=np.int64)
    for s in range(n):
        frontier, seen, depth = list(adj[s]), set(), 1
        while frontier:
            nxt = []
            for v in frontier:
                if v in seen:
                    continue
                seen.add(v)
                d[s, v] = depth
                nxt.extend(adj[v])
            frontier, depth = nxt, depth + 1
    return d


def _first_found_graph():
    """0 -a-> 1 ... -a-> 8 (8 edges) and 0 -b-> 9 -b-> 10 -b-> 11 -b-> 12 -b-> 8
    (5 edges).  S derives a^8 with a balanced tree of height 4 and b^5 only
    with a tree of height 5, so (S, 0, 8) is first added (at the fourth step)
    with length 8, and the shorter b-path found one step later must not
    replace it."""
    e = [(i, 0, i + 1) for i in range(8)] + [(0, 1, 9), (9, 1, 10), (10, 1, 11), (11, 1, 12), (12, 1, 8)]
    g = grammars._mk("first_found", ["S", "T", "U", "A", "B", "X1", "X2", "X3"], ["a", "b"],
                     [("A", "a"), ("B", "b")],
                     [("S", "T", "T"), ("T", "U", "U"), ("U", "A", "A"),
                      ("S", "B", "X1"), ("X1", "B", "X2"), ("X2", "B", "X3"), ("X3", "B", "B")])
    return 13, np.array(e, dtype=np.int32), g


def _check_witnesses(mod, n, e, g, L, cells=None):
    """Every (sampled) cell's witness is a path of exactly L edges from i to j
    in the graph whose label word the nonterminal derives (CYK)."""
    edge_set = {tuple(int(v) for v in x) for x in e}
    idx = np.argwhere(L > 0)
    if cells is not None and len(idx) > cells:
        idx = idx[np.random.default_rng(0).choice(len(idx), cells, replace=False)]
    for a, i, j in idx:
        path = mod.witness(n, e, g, L, int(a), int(i), int(j))
        if len(path) != L[a, i, j] or path[0][0] != i or path[-1][2] != j:
            return False
        if any(p[2] != q[0] for p, q in zip(path, path[1:])) or any(p not in edge_set for p in path):
            return False
        word = [p[1] for p in path]
        if len(word) <= 24 and int(a) not in brute.cyk_table(word, g)[0][len(word)]:
            return False
    return True


def _pins_hold(mod) -> bool:
    # relation and loop count of Algorithm 1
    for n, e, g in [(*graphs.erdos_renyi(40, 90, 5, labels=2), grammars.dyck()),
                    (*graphs.hierarchy(120, 6, roots=2, reverse=True), grammars.same_generation()),
                    (configs.worked_example().n, configs.worked_example().edges, configs.worked_example().grammar)]:
        L, loops = mod.lengths(n, e, g)
        t, loops1, _ = alg1.closure(n, e, g)
        if loops != loops1 or not np.array_equal(L > 0, t):
            return False
        if not _check_witnesses(mod, n, e, g, L, cells=25):
            return False
    # breadth-first search
    n, e = graphs.erdos_renyi(60, 110, 7, labels=2)
    L, _ = mod.lengths(n, e, grammars.transitive_closure())
    if not np.array_equal(L[0], _bfs_lengths(n, [(int(u), int(v)) for u, x, v in e if x == 0])):
        return False
    # chain: every length is j - i
    word = [0, 0, 1, 0, 1, 1, 0, 0, 1, 1, 1, 0, 1]
    n, e = graphs.chain(word)
    L, _ = mod.lengths(n, e, grammars.dyck())
    ii, jj = np.nonzero(L[0])
    if len(ii) == 0 or not np.array_equal(L[0][ii, jj], jj - ii):
        return False
    # first length found is kept
    n, e, g = _first_found_graph()
    L, _ = mod.lengths(n, e, g)
    if L[g.nt("S"), 0, 8] != 8:
        return False
    return True


def test_relation_and_loops_match_algorithm_1():
    for seed in range(3):
        n, e = graphs.random_tiny(7, 14, 2, 300 + seed)
        for g in (grammars.dyck(), grammars.anbn()):
            L, loops = single_path.lengths(n, e, g)
            t, loops1, _ = alg1.closure(n, e, g)
            assert loops == loops1
            assert np.array_equal(L > 0, t)
            assert (L[L > 0] >= 1).all()


def test_transitive_closure_gives_bfs_distances():
    n, e = graphs.erdos_renyi(80, 160, 11, labels=2)
    L, _ = single_path.lengths(n, e, grammars.transitive_closure())
    assert np.array_equal(L[0], _bfs_lengths(n, [(int(u), int(v)) for u, x, v in e if x == 0]))


@pytest.mark.parametrize("grammar", ["dyck", "anbn", "same_generation"])
def test_chain_lengths_are_distances(grammar):
    g = grammars.BY_NAME[grammar]()
    rng = np.random.default_rng(5)
    word = [int(x) for x in rng.integers(0, len(g.terminals), 24)]
    n, e = graphs.chain(word)
    L, _ = single_path.lengths(n, e, g)
    a, i, j = np.nonzero(L)
    assert len(a) > 0
    assert np.array_equal(L[a, i, j], j - i)


def two_cycle_lengths(na, nb):
    """Closed form for a^n b^n on two cycles of coprime lengths na, nb sharing
    node 0: (S, u, v) for u in the a-cycle and v at position p of the b-cycle.
    The label a^m b^m leaves u, reaches node 0 after m a-edges (m = -u mod na)
    and walks m b-edges (m = p mod nb); the smallest such m >= 1 has the lowest
    derivation tree (height 2m), so the first length found is 2m."""
    bcyc = [0] + list(range(na, na + nb - 1))
    out = {}
    for u in range(na):
        for pos, v in enumerate(bcyc):
            m = next(m for m in range(1, na * nb + 1) if (u + m) % na == 0 and m % nb == pos)
            out[(u, v)] = 2 * m
    return out


def test_two_cycles_closed_form():
    n, e = graphs.two_cycles(8, 7)
    g = grammars.anbn()
    L, loops = single_path.lengths(n, e, g)
    assert loops == 2 * 8 * 7 + 1
    S = g.nt("S")
    want = two_cycle_lengths(8, 7)
    for (u, v), l in want.items():
        assert L[S, u, v] == l, (u, v)
    assert int((L[S] > 0).sum()) == len(want) == 56


def test_first_length_found_is_kept():
    n, e, g = _first_found_graph()
    L, _ = single_path.lengths(n, e, g)
    assert L[g.nt("S"), 0, 8] == 8
    t, _, _ = alg1.closure(n, e, g)
    assert np.array_equal(L > 0, t)


def test_witnesses_on_tiny_graphs():
    g = grammars.CNF(("S", "X", "Y"), ("a", "b"), ((1, 0), (2, 0), (2, 1)), ((0, 1, 2), (0, 0, 0), (1, 0, 2)),
                     "tiny")
    for seed in range(4):
        n, e = graphs.random_tiny(6, 11, 2, 500 + seed)
        L, _ = single_path.lengths(n, e, g)
        assert _check_witnesses(single_path, n, e, g, L)
    n, e = graphs.two_cycles(8, 7)
    L, _ = single_path.lengths(n, e, grammars.anbn())
    assert _check_witnesses(single_path, n, e, grammars.anbn(), L)


def test_real_oracle_passes_harness():
    assert _pins_hold(single_path)


SP_MUTANTS = {
    "last_split_wins": ("np.minimum(out, lb[:, k:k + 1] + lc[k:k + 1, :], out=out)",
                        "out = np.where(lb[:, k:k + 1] + lc[k:k + 1, :] < INF, lb[:, k:k + 1] + lc[k:k + 1, :], out)"),
    "length_plus_one": ("np.minimum(out, lb[:, k:k + 1] + lc[k:k + 1, :], out=out)",
                        "np.minimum(out, lb[:, k:k + 1] + lc[k:k + 1, :] + 1, out=out)"),
    "later_shorter_replaces": ("new = (L == INF) & (cand < INF)", "new = cand < L"),
    "reads_current_step": ("            cand[a] = np.minimum(cand[a], min_plus(L[b], L[c]))",
                           "            cand[a] = np.minimum(cand[a], min_plus(L[b], L[c]))\n"
                           "            L[a] = np.where(L[a] == INF, cand[a], L[a])"),
    "witness_ignores_length": ("(lb > 0) & (lc > 0) & (lb + lc == l)", "(lb > 0) & (lc > 0)"),
}


@pytest.mark.parametrize("name", sorted(SP_MUTANTS))
def test_single_path_mutant_is_caught(name):
    old, new = SP_MUTANTS[name]
    src = open(single_path.__file__).read()
    assert src.count(old) == 1, name
    mod = types.ModuleType(f"mutant_{name}")
    mod.__file__ = single_path.__file__
    exec(compile(src.replace(old, new), os.path.basename(single_path.__file__), "exec"), mod.__dict__)
    try:
        held = _pins_hold(mod)
    except (ValueError, IndexError):
        held = False
    assert not held, f"mutant {name} passed every pin"


# ---- the C transcription (cfpq_single_path.c), used for the larger digests ----

def _native_module(lib=None):
    """``lengths`` of the C transcription with the numpy ``witness``, in the
    shape the pin harness takes."""
    def lengths(n, e, g, max_loops=None):
        L, loops, rc = single_path.lengths_native(n, e, g, max_loops, lib=lib)
        assert rc in (0, 3), rc
        return L.astype(np.int64), loops
    return types.SimpleNamespace(lengths=lengths, witness=single_path.witness)


def test_native_oracle_passes_harness():
    assert _pins_hold(_native_module())


@pytest.mark.parametrize("grammar", ["dyck", "anbn", "same_generation", "transitive_closure"])
def test_native_equals_numpy(grammar):
    g = grammars.BY_NAME[grammar]()
    for seed, (n, m) in enumerate([(1, 1), (13, 30), (64, 150), (97, 260)]):
        if grammar == "same_generation":
            n, e = graphs.hierarchy(max(n, 2), seed, roots=1, reverse=bool(seed % 2))
        else:
            n, e = graphs.erdos_renyi(n, min(m, n * (n - 1)) if n > 1 else 0, 40 + seed, labels=len(g.terminals))
        L, loops = single_path.lengths(n, e, g)
        Lc, loops_c, rc = single_path.lengths_native(n, e, g)
        assert rc == 0 and loops_c == loops
        assert np.array_equal(Lc.astype(np.int64), L), (grammar, n)
    # a cap on the loop count stops both at the same state
    n, e = graphs.erdos_renyi(50, 140, 3, labels=len(g.terminals))
    L, loops = single_path.lengths(n, e, g, max_loops=2)
    Lc, loops_c, rc = single_path.lengths_native(n, e, g, max_loops=2)
    assert loops_c == loops == 2 and np.array_equal(Lc.astype(np.int64), L)


def doubling_grammar(k_max: int):
    """A0 -> a, A_k -> A_(k-1) A_(k-1): on one node with an a-loop, A_k has the
    single length 2^k (its only derivation tree is complete of height k)."""
    names = [f"A{k}" for k in range(k_max + 1)]
    return grammars._mk(f"doubling{k_max}", names, ["a"], [("A0", "a")],
                        [(names[k], names[k - 1], names[k - 1]) for k in range(1, k_max + 1)])


def test_native_doubling_lengths_and_overflow():
    e = np.array([[0, 0, 0]], dtype=np.int32)
    L, loops, rc = single_path.lengths_native(1, e, doubling_grammar(30))
    assert rc == 0 and loops == 31
    assert [int(L[k, 0, 0]) for k in range(31)] == [2 ** k for k in range(31)]
    # 2^31 does not fit the GPU path's lengths: the oracle says so
    _, _, rc = single_path.lengths_native(1, e, doubling_grammar(31))
    assert rc == 1


SP_C_MUTANTS = {
    "length_plus_one": ("ABSENT : b + crk[j];", "ABSENT : b + crk[j] + 1;"),
    "largest_split_wins": ("crow[j] = s < crow[j] ? s : crow[j];",
                           "crow[j] = (crow[j] == ABSENT || (s != ABSENT && s > crow[j])) ? s : crow[j];"),
    "later_shorter_replaces": ("if (L[x] == ABSENT && cand[x] != ABSENT) {", "if (cand[x] < L[x]) {"),
    "transposed_right_operand": ("const uint32_t *crk = lc + (size_t)k * n;\n                    for (int32_t j = 0; j < n; ++j) {\n                        /* both lengths are below 2^31, so the sum fits */\n                        const uint32_t s = crk[j] == ABSENT ? ABSENT : b + crk[j];",
                                 "const uint32_t *crk = lc + (size_t)k;\n                    for (int32_t j = 0; j < n; ++j) {\n                        /* both lengths are below 2^31, so the sum fits */\n                        const uint32_t s = crk[(size_t)j * n] == ABSENT ? ABSENT : b + crk[(size_t)j * n];"),
    "first_rule_only": ("for (int32_t r = 0; r < n_bin; ++r) {\n            const uint32_t *lb", "for (int32_t r = 0; r < 1 && r < n_bin; ++r) {\n            const uint32_t *lb"),
    "last_step_not_counted": ("        if (added == 0) {\n            capped = 0;", "        if (added == 0) {\n            --loops;\n            capped = 0;"),
    "reversed_edges": ("L[(size_t)term[2 * r] * cells + (size_t)t[0] * n + t[2]] = 1;",
                       "L[(size_t)term[2 * r] * cells + (size_t)t[2] * n + t[0]] = 1;"),
}


@pytest.mark.parametrize("name", sorted(SP_C_MUTANTS))
def test_native_mutant_is_caught(name, tmp_path):
    old, new = SP_C_MUTANTS[name]
    src = open(single_path._C_SRC).read()
    assert src.count(old) == 1, name
    msrc = tmp_path / "mutant.c"
    msrc.write_text(src.replace(old, new))
    lib = single_path.load_native(single_path.build_native(True, str(msrc), str(tmp_path / "libmutant.so")))
    try:
        held = _pins_hold(_native_module(lib))
    except (ValueError, IndexError, AssertionError):
        held = False
    assert not held, f"mutant {name} passed every pin"
