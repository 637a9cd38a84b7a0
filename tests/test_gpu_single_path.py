"""GPU parity of the single-path lengths (section 5) against the oracle, the
two-cycle closed form and breadth-first search, plus witness paths checked
edge by edge and by CYK."""
from __future__ import annotations

import hashlib
import json
import os
import sys

import numpy as np
import pytest

from oracle import brute, single_path as sp
from tests.test_oracle_single_path import _bfs_lengths, _first_found_graph, doubling_grammar, two_cycle_lengths
from workloads import configs, grammars, graphs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cfpq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_01007_amd as m
    m.lib()
    return m


def _say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def _lengths(cfpq, n, e, g, **kw):
    _say("single_path", n, g.name, kw)
    res, L = cfpq.single_path(n, e, g, **kw)
    return res, L[:, :n, :n].cpu().numpy().astype(np.int64)


def _check_paths(cfpq, n, e, g, L, count=40, seed=0):
    edge_set = {tuple(int(v) for v in x) for x in np.asarray(e).reshape(-1, 3)}
    idx = np.argwhere(L > 0)
    if len(idx) > count:
        idx = idx[np.random.default_rng(seed).choice(len(idx), count, replace=False)]
    full = np.zeros((L.shape[0], cfpq.padded_rows(n), cfpq.padded_rows(n)), dtype=np.uint32)
    full[:, :n, :n] = L
    for a, i, j in idx:
        path = cfpq.witness(n, e, g, full, int(a), int(i), int(j))
        assert len(path) == L[a, i, j]
        assert path[0][0] == i and path[-1][2] == j
        assert all(p[2] == q[0] for p, q in zip(path, path[1:]))
        assert all(tuple(p) in edge_set for p in path)
        word = [p[1] for p in path]
        if len(word) <= 30:
            assert int(a) in brute.cyk_table(word, g)[0][len(word)]


def _dense_nested_dyck():
    """Two components: the nested chain a^40 b^40 (its outermost pair found only
    after about 80 steps) and a dense G(90, 4200), together more than npad^2 /
    16 edges.  The dense part's full matrices make the tile min-plus kernel the
    cheaper choice for S -> S S in every step where S gains cells, so it runs
    past the first 14 steps (narrow, 16-bit) on the 32-bit kernel."""
    n1, chain = graphs.chain([0] * 40 + [1] * 40)
    n2, dense = graphs.erdos_renyi(90, 4200, 8, labels=2)
    dense = np.asarray(dense, np.int32).reshape(-1, 3) + np.array([n1, 0, n1], np.int32)
    return n1 + n2, np.concatenate([np.asarray(chain, np.int32).reshape(-1, 3), dense]), grammars.dyck()


CASES = {
    "worked_example": lambda: (configs.worked_example().n, configs.worked_example().edges,
                               configs.worked_example().grammar),
    "er40_dyck": lambda: (*graphs.erdos_renyi(40, 100, 3, labels=2), grammars.dyck()),
    "er65_anbn": lambda: (*graphs.erdos_renyi(65, 200, 4, labels=2), grammars.anbn()),
    "er200_dyck": lambda: (*graphs.erdos_renyi(200, 600, 5, labels=2), grammars.dyck()),
    "er257_dyck": lambda: (*graphs.erdos_renyi(257, 700, 6, labels=2), grammars.dyck()),
    "hier300_rev_samegen": lambda: (*graphs.hierarchy(300, 7, roots=2, reverse=True), grammars.same_generation()),
    "first_found": lambda: _first_found_graph(),
    # more than npad^2 / 16 edges: every rule on the tile min-plus kernel
    "er90_dense_dyck": lambda: (*graphs.erdos_renyi(90, 4200, 8, labels=2), grammars.dyck()),
    # 15 k-chunks of 32: S -> S S on tiles split along k in its later loops
    "er450_dyck": lambda: (*graphs.erdos_renyi(450, 1350, 14, labels=2), grammars.dyck()),
    # tile kernel past the narrow steps
    "dense_nested_dyck": _dense_nested_dyck,
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_lengths_match_oracle(cfpq, name):
    n, e, g = CASES[name]()
    want, loops = sp.lengths(n, e, g)
    res, got = _lengths(cfpq, n, e, g)
    assert res.stats["iterations"] == loops
    assert np.array_equal(got, want)
    if name in ("er450_dyck", "er90_dense_dyck", "dense_nested_dyck"):
        assert res.stats["minplus_terms"] > 0  # the tile kernel ran
    if name == "dense_nested_dyck":
        assert res.stats["iterations"] > 14 and int(got[0, 0, 80]) == 80  # S over the whole chain: 80 edges
    bits = cfpq.result_bits(res)
    from oracle import worklist
    assert np.array_equal(bits, worklist.closure(n, e, g))
    _check_paths(cfpq, n, e, g, got)


def test_two_cycles_closed_form(cfpq):
    inst = configs.config1()
    res, got = _lengths(cfpq, inst.n, inst.edges, inst.grammar)
    assert res.stats["iterations"] == 8065
    S = inst.grammar.nt("S")
    want = two_cycle_lengths(64, 63)
    assert int((got[S] > 0).sum()) == len(want) == 4032
    for (u, v), l in want.items():
        assert got[S, u, v] == l, (u, v)
    _check_paths(cfpq, inst.n, inst.edges, inst.grammar, got, count=10)


def test_transitive_closure_is_bfs(cfpq):
    n, e = graphs.erdos_renyi(600, 1400, 12, labels=2)
    res, got = _lengths(cfpq, n, e, grammars.transitive_closure())
    assert np.array_equal(got[0], _bfs_lengths(n, [(int(u), int(v)) for u, x, v in e if x == 0]))


def test_chain_lengths(cfpq):
    rng = np.random.default_rng(9)
    word = [int(x) for x in rng.integers(0, 2, 300)]
    n, e = graphs.chain(word)
    res, got = _lengths(cfpq, n, e, grammars.dyck())
    a, i, j = np.nonzero(got)
    assert len(a) > 0 and np.array_equal(got[a, i, j], j - i)


def test_partial_result_is_a_prefix(cfpq):
    n, e, g = CASES["er200_dyck"]()
    full, _ = sp.lengths(n, e, g)
    res, got = _lengths(cfpq, n, e, g, max_iters=3, allow_partial=True)
    assert res.status == -4
    want, _ = sp.lengths(n, e, g, max_loops=3)
    assert np.array_equal(got, want)
    assert np.array_equal(got[got > 0], full[got > 0])


def test_device_edges_and_larger_graph(cfpq):
    """ER 2048 Dyck from device edges: the lengths' support is the relational
    closure, and sampled witnesses are valid paths."""
    import torch
    inst = configs.config3(2048)
    res, got = _lengths(cfpq, inst.n, torch.from_numpy(inst.edges).cuda(), inst.grammar)
    rel = cfpq.closure(inst.n, inst.edges, inst.grammar)
    bits = cfpq.result_bits(rel)
    from oracle import worklist
    assert np.array_equal(worklist.unpack(bits, inst.n), got > 0)
    assert np.array_equal(cfpq.result_bits(res), bits)
    _check_paths(cfpq, inst.n, inst.edges, inst.grammar, got, count=25)


def _shortest_lengths(n, e):
    """Fewest edges (>= 1) on a path i -> j, 0 if none, for every pair: scipy's
    unweighted shortest paths, with d[i][i] = the shortest cycle through i."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path
    src, dst = e[:, 0].astype(np.int64), e[:, 2].astype(np.int64)
    A = csr_matrix((np.ones(len(src)), (src, dst)), shape=(n, n))
    d = shortest_path(A, method="D", unweighted=True)
    diag = np.full(n, np.inf)
    np.minimum.at(diag, src, 1.0 + d[dst, src])  # leave i by one edge, come back
    np.fill_diagonal(d, diag)
    d[~np.isfinite(d)] = 0
    return d.astype(np.int64)


@pytest.mark.parametrize("side", ["right_linear", "left_linear"])
def test_linear_closure_lengths_are_shortest_paths(cfpq, side):
    """S -> a | A S (or S A), A -> a: each loop extends paths by one edge, so a
    cell's length is its shortest path length.  The fixed sparse operand A
    sends the rule through the row gather (A S) or the column index (S A)
    min-plus; n = 4500 makes rows longer than 64 words."""
    g = grammars.CNF(("S", "A"), ("a",), ((0, 0), (1, 0)), ((0, 1, 0) if side == "right_linear" else (0, 0, 1),),
                     name=side)
    n, e = graphs.erdos_renyi(4500, 6500, 13, labels=1)
    res, got = _lengths(cfpq, n, e, g)
    assert np.array_equal(got[0], _shortest_lengths(n, e))
    assert np.array_equal(got[1] > 0, _shortest_lengths(n, e) == 1)


def test_degenerate_inputs(cfpq):
    """No edges; edges whose label no rule reads; one node with a self-loop;
    a grammar without binary rules (lengths are the edge cells only)."""
    empty = np.zeros((0, 3), dtype=np.int32)
    res, got = _lengths(cfpq, 50, empty, grammars.dyck())
    assert not got.any() and not cfpq.result_bits(res).any()
    tc = grammars.transitive_closure()  # reads label a (0) only
    res, got = _lengths(cfpq, 30, np.array([[0, 1, 1], [1, 1, 2]], dtype=np.int32), tc)
    assert not got.any()
    res, got = _lengths(cfpq, 1, np.array([[0, 0, 0]], dtype=np.int32), tc)
    assert got.shape == (1, 1, 1) and got[0, 0, 0] == 1
    only_terms = grammars.CNF(("S",), ("a", "b"), ((0, 0),), (), name="only_terms")
    n, e = graphs.erdos_renyi(70, 300, 21, labels=2)
    res, got = _lengths(cfpq, n, e, only_terms)
    want = np.zeros((n, n), dtype=np.int64)
    a_edges = e[e[:, 1] == 0]
    want[a_edges[:, 0], a_edges[:, 2]] = 1
    assert np.array_equal(got[0], want)


DIGESTS = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "digests.json")))


@pytest.mark.parametrize("name", ["sp_er2048_dyck", "sp_er4096_dyck"])
def test_er_dyck_lengths_match_oracle_digest(cfpq, name):
    """The ER Dyck recipe at n = 2048 and at the benchmark's n = 4096, edges in
    device memory as the benchmark passes them: every length equals the C
    single-path oracle's (per-nonterminal counts and sums, and a SHA-256 of
    all n x n lengths of every nonterminal), with the same loop count."""
    import torch
    gold = DIGESTS[name]
    inst = configs.config3(gold["n"])
    res, got = _lengths(cfpq, inst.n, torch.from_numpy(inst.edges).cuda(), inst.grammar)
    assert res.stats["iterations"] == gold["jacobi_loops"]
    got = got.astype(np.uint32)
    assert [int((x > 0).sum()) for x in got] == gold["counts"]
    assert [int(x.astype(np.int64).sum()) for x in got] == gold["length_sums"]
    assert hashlib.sha256(np.ascontiguousarray(got).astype("<u4").tobytes()).hexdigest() == gold["sha256"]


def test_length_overflow_is_reported(cfpq):
    """One node with an a-loop and A0 -> a, A_k -> A_(k-1) A_(k-1): A_k has the
    single length 2^k.  Up to k = 30 every length is exact (and equal to the
    oracle's); at k = 31 the length 2^31 does not fit, and the call reports
    CFPQ_ERANGE, as the oracle does."""
    from paper_1707_01007_amd import _abi
    e = np.array([[0, 0, 0]], dtype=np.int32)
    g30 = doubling_grammar(30)
    res, got = _lengths(cfpq, 1, e, g30)
    want, loops, rc = sp.lengths_native(1, e, g30)
    assert rc == 0 and res.stats["iterations"] == loops == 31
    assert np.array_equal(got.astype(np.uint32), want)
    assert [int(got[k, 0, 0]) for k in range(31)] == [2 ** k for k in range(31)]
    g31 = doubling_grammar(31)
    assert sp.lengths_native(1, e, g31)[2] == 1
    _say("single_path", 1, g31.name, "expect CFPQ_ERANGE")
    with pytest.raises(_abi.CfpqError) as err:
        cfpq.single_path(1, e, g31)
    assert err.value.status == _abi.CFPQ_ERANGE
