"""GPU parity of the conjunctive-grammar closure against the oracle
(Algorithm 1 with the AND of conjunct products), bit for bit, for both dense
product kernels and both schedules."""
from __future__ import annotations

import hashlib
import json
import os
import sys

import numpy as np
import pytest

from oracle import conjunctive, worklist
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


def _run(cfpq, n, e, g, **kw):
    print("[gpu-case] conjunctive", n, g.name, kw, file=sys.stderr, flush=True)
    res = cfpq.conjunctive_closure(n, e, g, **kw)
    return worklist.unpack(cfpq.result_bits(res), n), res


def _anbncn_chain(k_list, noise_seed):
    rng = np.random.default_rng(noise_seed)
    word = []
    for k in k_list:
        word += [0] * k + [1] * k + [2] * k
        word += [int(x) for x in rng.integers(0, 3, 3)]
    return graphs.chain(word)


CASES = {
    "chain_anbncn": lambda: (*_anbncn_chain([1, 3, 2, 5], 1), grammars.anbncn()),
    "er90_anbncn": lambda: (*graphs.erdos_renyi(90, 400, 2, labels=3), grammars.anbncn()),
    "er300_anbncn": lambda: (*graphs.erdos_renyi(300, 1500, 3, labels=3), grammars.anbncn()),
    "er257_dyck_and_anbn": lambda: (*graphs.erdos_renyi(257, 800, 4, labels=2), grammars.dyck_and_anbn()),
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("path", ["bits", "mfma", "fp4"])
@pytest.mark.parametrize("schedule", ["inplace", "jacobi"])
@pytest.mark.parametrize("hybrid", [0, 1])
def test_conjunctive_matches_oracle(cfpq, name, path, schedule, hybrid):
    """Every dense kernel, both schedules, and with (hybrid 1) or without the
    ROWS products of conjuncts whose left operand is an edge matrix."""
    n, e, g = CASES[name]()
    want, loops = conjunctive.closure(n, e, g)
    got, res = _run(cfpq, n, e, g, path=path, schedule=schedule, dirty=(schedule == "inplace"), hybrid=hybrid)
    assert np.array_equal(got, want)
    if schedule == "jacobi":
        assert res.stats["iterations"] == loops
    if not hybrid:
        assert res.stats["sparse_products"] == 0
    elif name == "er257_dyck_and_anbn":  # conjuncts A D1, A E1, A B: left operand A -> a
        assert 0 < res.stats["sparse_products"] < res.stats["products"]


def test_one_conjunct_rules_equal_plain_closure(cfpq):
    n, e = graphs.erdos_renyi(700, 2800, 5, labels=2)
    got, _ = _run(cfpq, n, e, grammars.conjunctive_from_cnf(grammars.dyck()))
    plain = cfpq.closure(n, e, grammars.dyck())
    assert np.array_equal(got, worklist.unpack(cfpq.result_bits(plain), n))


def test_conjoined_start_rules_are_the_intersection(cfpq):
    """R_S = R_Dyck & R_anbn on a 1500-node graph (oracle: two relational
    closures of the C worklist)."""
    n, e = graphs.erdos_renyi(1500, 4500, 6, labels=2)
    g = grammars.dyck_and_anbn()
    got, _ = _run(cfpq, n, e, g, path="mfma")
    d = worklist.unpack(worklist.closure(n, e, grammars.dyck()), n)[0]
    ab = worklist.unpack(worklist.closure(n, e, grammars.anbn()), n)[0]
    assert np.array_equal(got[g.nt("S")], d & ab)


def test_partial_and_device_edges(cfpq):
    import torch
    n, e, g = CASES["er90_anbncn"]()
    want, _ = conjunctive.closure(n, e, g, max_loops=2)
    got, res = _run(cfpq, n, torch.from_numpy(e).cuda(), g, schedule="jacobi", dirty=False, max_iters=2,
                    allow_partial=True)
    assert res.status in (0, -4)
    assert np.array_equal(got, want)


def _anbncn_three_conjuncts():
    """S -> P Cp & Ap Q & Ap X with X => (b|c)^+: the same language as
    anbncn (the third conjunct is implied), through a rule of three conjuncts
    (Q &= R for the middle one, the last folded into the union)."""
    return grammars._mk_conj(
        "anbncn3", ["S", "P", "P1", "Q", "Q1", "Ap", "Cp", "A", "B", "C", "X"], ["a", "b", "c"],
        [("A", "a"), ("B", "b"), ("C", "c"), ("Ap", "a"), ("Cp", "c"), ("X", "b"), ("X", "c")],
        [("S", [("P", "Cp"), ("Ap", "Q"), ("Ap", "X")]),
         ("P", [("A", "B")]), ("P", [("A", "P1")]), ("P1", [("P", "B")]),
         ("Q", [("B", "C")]), ("Q", [("B", "Q1")]), ("Q1", [("Q", "C")]),
         ("Ap", [("A", "Ap")]), ("Cp", [("C", "Cp")]), ("X", [("B", "X")]), ("X", [("C", "X")])])


@pytest.mark.parametrize("graph", ["chain", "er120"])
@pytest.mark.parametrize("path", ["bits", "fp4"])
@pytest.mark.parametrize("hybrid", [0, 1])
def test_three_conjunct_rule_matches_oracle(cfpq, graph, path, hybrid):
    g = _anbncn_three_conjuncts()
    n, e = _anbncn_chain([2, 4, 1], 7) if graph == "chain" else graphs.erdos_renyi(120, 600, 8, labels=3)
    want, _ = conjunctive.closure(n, e, g)
    got, _ = _run(cfpq, n, e, g, path=path, hybrid=hybrid)
    assert np.array_equal(got, want)
    if graph == "chain":  # exactly a^n b^n c^n on a chain
        plain, _ = conjunctive.closure(n, e, grammars.anbncn())
        assert np.array_equal(got[g.nt("S")], plain[grammars.anbncn().nt("S")])


def test_er8192_benchmark_matches_oracle_digest(cfpq):
    """The benchmark's conjunctive workload (Dyck conjoined with a^n b^n, ER
    recipe at n = 8192), edges in device memory and the library's default
    products as the benchmark runs it: every bit equals the conjunctive
    oracle's (per-nonterminal counts and a SHA-256 of the packed result)."""
    import torch
    gold = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                       "digests.json")))["er8192_dyck_and_anbn"]
    inst = configs.config3(gold["n"])
    g = grammars.dyck_and_anbn()
    print("[gpu-case] conjunctive", inst.n, g.name, "benchmark", file=sys.stderr, flush=True)
    res = cfpq.conjunctive_closure(inst.n, torch.from_numpy(inst.edges).cuda(), g)
    bits = cfpq.result_bits(res)
    assert [int(np.unpackbits(b.view(np.uint8)).sum()) for b in bits] == gold["counts"]
    assert hashlib.sha256(np.ascontiguousarray(bits).astype("<u8").tobytes()).hexdigest() == gold["sha256"]
    assert res.stats["sparse_products"] > 0  # conjuncts with an edge-matrix operand ran as ROWS / COLS
