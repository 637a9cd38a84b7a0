"""GPU parity of the batched engine (cfpq_batch_closure) against the oracle:
every instance bit-exact, alone or in the mix."""
from __future__ import annotations

import hashlib
import json
import os
import sys

import numpy as np
import pytest

from oracle import worklist
from workloads import configs, grammars, graphs

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


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


def _digest(bits):
    return hashlib.sha256(np.ascontiguousarray(bits).astype("<u8").tobytes()).hexdigest()


def _mixed_instances():
    insts = [configs.worked_example(), configs.config1()]
    insts += configs.config4(count=40)
    n, e = graphs.erdos_renyi(0, 0, 1)
    insts.append(configs.Instance(0, e, grammars.dyck(), "empty"))
    n, e = graphs.erdos_renyi(300, 600, 2)
    insts.append(configs.Instance(n, e, grammars.CNF(("X",), ("a", "b"), ((0, 0),), (), "terminal_only"), "term_only"))
    n, e = graphs.erdos_renyi(1500, 6000, 3)
    insts.append(configs.Instance(n, e, grammars.dyck(), "er1500"))
    n, e = graphs.hierarchy(3000, 4, roots=3, reverse=True)
    insts.append(configs.Instance(n, e, grammars.same_generation(), "hier3000_rev"))
    return insts


@pytest.mark.parametrize("hybrid", [0, 1])
def test_mixed_batch_matches_oracle(cfpq, hybrid):
    insts = _mixed_instances()
    _say("mixed batch", len(insts), "instances, sizes", sorted(i.n for i in insts)[-5:], "hybrid", hybrid)
    res = cfpq.batch_closure([(i.n, i.edges, i.grammar) for i in insts], hybrid=hybrid)
    for inst, r in zip(insts, res):
        want = worklist.closure(inst.n, inst.edges, inst.grammar)
        assert np.array_equal(cfpq.result_bits(r), want), inst.tag
        assert r.stats["converged"] == 1


def test_batch_alone_equals_in_mix(cfpq):
    """Disjoint-union invariant: the same query gives the same bits alone and
    inside a batch."""
    insts = _mixed_instances()
    mix = cfpq.batch_closure([(i.n, i.edges, i.grammar) for i in insts])
    for k in (0, 1, 5, len(insts) - 1, len(insts) - 2):
        inst = insts[k]
        alone = cfpq.closure(inst.n, inst.edges, inst.grammar)
        alone_b = cfpq.batch_closure([(inst.n, inst.edges, inst.grammar)])[0]
        a = cfpq.result_bits(alone)
        assert np.array_equal(a, cfpq.result_bits(mix[k])), inst.tag
        assert np.array_equal(a, cfpq.result_bits(alone_b)), inst.tag


# route tables of the batched engine: padded side -> (route, tile); missing
# sides take the default (resident up to 512, 256 tiles above)
ROUTE_TABLES = {
    "default": {},
    "tiles256_everywhere": {256: ("tiles", 256), 512: ("tiles", 256)},
    "tiles128_everywhere": {p: ("tiles", 128) for p in range(256, 2049, 256)},
    "resident_then_tiles128": {256: ("resident", 0), 512: ("resident", 0),
                               **{p: ("tiles", 128) for p in range(768, 2049, 256)}},
}


def _set_routes(cfpq, table):
    cfpq.tune_clear()
    for npad, (route, tile) in table.items():
        cfpq.batch_tune_set(npad, route, tile)


@pytest.mark.parametrize("table", sorted(ROUTE_TABLES))
def test_full_batch_workload_digests(cfpq, table):
    """All 512 instances of the batch workload, each against its stored
    oracle digest, under several route tables of the batched engine (every
    route gives the same bits)."""
    gold = json.load(open(os.path.join(GOLD, "batch_digests.json")))["batch512"]
    insts = configs.config4()
    _say("batch512", table)
    _set_routes(cfpq, ROUTE_TABLES[table])
    try:
        res = cfpq.batch_closure([(i.n, i.edges, i.grammar) for i in insts])
    finally:
        cfpq.tune_clear()
    for k, (inst, r) in enumerate(zip(insts, res)):
        bits = cfpq.result_bits(r)
        assert [int(np.unpackbits(b.view(np.uint8)).sum()) for b in bits] == gold[k]["counts"], (k, inst.tag)
        assert _digest(bits) == gold[k]["sha256"], (k, inst.tag)
        assert r.stats["converged"] == 1


def test_batch_autotune_records_routes_and_keeps_bits(cfpq):
    """The batch autotuner on a sample of the batch workload: one entry per
    padded side present, with every candidate timed (the resident route
    offered only up to 512); a side leaves its default route only for a
    candidate more than 2% faster; the entries are recorded in the table, and
    the batch closure that follows uses them and matches the oracle digests."""
    gold = json.load(open(os.path.join(GOLD, "batch_digests.json")))["batch512"]
    insts = configs.config4()
    items = [(i.n, i.edges, i.grammar) for i in insts]
    cfpq.tune_clear()
    try:
        _say("batch autotune")
        entries = cfpq.batch_autotune(items, max_per_bucket=8, reps=1)
        sides = sorted({cfpq.padded_rows(i.n) for i in insts if i.n > 0})
        assert [e["npad"] for e in entries] == sides
        for e in entries:
            c = e["candidates_ms"]
            assert {"tiles256", "tiles128"} <= set(c)
            assert ("resident" in c) == (e["npad"] <= 512)
            chosen = "resident" if e["route"] == "resident" else f"tiles{e['tile']}"
            default = "resident" if e["npad"] <= 512 else "tiles256"
            assert e["ms"] == pytest.approx(c[chosen])
            assert chosen == default or c[chosen] < 0.98 * c[default]
            assert cfpq.batch_tune_get(e["npad"])["route"] == e["route"]
            assert 0 < e["instances"] <= 8
        res = cfpq.batch_closure(items)
    finally:
        cfpq.tune_clear()
    for k, (inst, r) in enumerate(zip(insts, res)):
        assert _digest(cfpq.result_bits(r)) == gold[k]["sha256"], (k, inst.tag)


@pytest.mark.parametrize("table", ["tiles128_everywhere", "tiles256_everywhere"])
def test_server_follows_route_table(cfpq, table):
    """Servers created after the table is set take its routes: the same bits
    as the oracle for a mixed stream with every route forced."""
    insts = configs.config4(count=30)
    _set_routes(cfpq, ROUTE_TABLES[table])
    try:
        with cfpq.Server(hbm_budget=2 << 30, max_slots=64, hybrid_lanes=0) as srv:
            tickets = [srv.submit(i.n, i.edges, i.grammar) for i in insts]
            infos = [srv.wait(t) for t in tickets]
    finally:
        cfpq.tune_clear()
    for inst, info in zip(insts, infos):
        assert info["status"] == 0
        assert np.array_equal(cfpq.result_bits(info["result"]), worklist.closure(inst.n, inst.edges, inst.grammar))


def test_batch_device_edges_and_errors(cfpq):
    import torch
    insts = configs.config4(count=6)
    items = [(i.n, torch.from_numpy(i.edges).cuda(), i.grammar) for i in insts]
    res = cfpq.batch_closure(items)
    for inst, r in zip(insts, res):
        assert np.array_equal(cfpq.result_bits(r), worklist.closure(inst.n, inst.edges, inst.grammar))
    bad = insts[3].edges.copy()
    bad[0, 0] = insts[3].n + 1
    items[3] = (insts[3].n, torch.from_numpy(bad).cuda(), insts[3].grammar)
    with pytest.raises(cfpq.CfpqError) as ei:
        cfpq.batch_closure(items)
    assert ei.value.status == -1 and "instance 3" in str(ei.value)


@pytest.mark.parametrize("size", [300, 1500])
def test_batch_bad_device_edge_on_each_route(cfpq, size):
    """An out-of-range device edge in a resident-route instance (padded side
    <= 512) or a tile-route one fails the batch with CFPQ_EINVAL naming it;
    the same batch without it matches the oracle."""
    import torch
    g = grammars.dyck()
    insts = [graphs.erdos_renyi(sz, 3 * sz, 20 + k) for k, sz in enumerate((200, size, 900))]
    items = [(n, torch.from_numpy(e).cuda(), g) for n, e in insts]
    res = cfpq.batch_closure(items)
    for (n, e), r in zip(insts, res):
        assert np.array_equal(cfpq.result_bits(r), worklist.closure(n, e, g))
    n, e = insts[1]
    bad = e.copy()
    bad[-1, 2] = n
    items[1] = (n, torch.from_numpy(bad).cuda(), g)
    with pytest.raises(cfpq.CfpqError) as ei:
        cfpq.batch_closure(items)
    assert ei.value.status == -1 and "instance 1" in str(ei.value)


def test_batch_max_iters_partial_is_sound(cfpq):
    insts = [configs.config1(), configs.config3(1024)]
    res = cfpq.batch_closure([(i.n, i.edges, i.grammar) for i in insts], max_iters=3, allow_partial=True)
    assert res[0].status == -4
    for inst, r in zip(insts, res):
        part = worklist.unpack(cfpq.result_bits(r), inst.n)
        full = worklist.unpack(worklist.closure(inst.n, inst.edges, inst.grammar), inst.n)
        assert not (part & ~full).any()
        assert r.stats["iterations"] == 3 and r.stats["converged"] == 0


@pytest.mark.parametrize("capture", [1, 3, 16])
def test_batch_capture_depths(cfpq, capture):
    insts = configs.config4(count=12)
    res = cfpq.batch_closure([(i.n, i.edges, i.grammar) for i in insts], capture=capture)
    for inst, r in zip(insts, res):
        assert np.array_equal(cfpq.result_bits(r), worklist.closure(inst.n, inst.edges, inst.grammar)), inst.tag


@pytest.mark.parametrize("dirty", [True, False])
def test_batch_row_gather_rules(cfpq, dirty):
    """Larger instances whose edge-matrix rules run as row gathers (hybrid on)
    against the oracle: ragged sizes past several 256-row tiles, a node with
    hundreds of out-edges (one long row of B, and every row of C pushed into
    it), two rules with one head, and a graph too dense for the gather (tiles
    only); the same bits with hybrid off.  With and without the dirty-rule
    worklist (the rows pushed after the first loops are those that changed
    since the rule last read them, in either case)."""
    insts = []
    n, e = graphs.erdos_renyi(1000, 3000, 41, labels=2)
    insts.append(configs.Instance(n, e, grammars.dyck(), "er1000"))
    n, e = graphs.erdos_renyi(777, 2500, 42, labels=2)
    star = np.array([[5, 0, j] for j in range(0, 777, 1)], dtype=np.int32)
    insts.append(configs.Instance(n, np.concatenate([e, star]), grammars.dyck(), "er777_star"))
    n, e = graphs.hierarchy(2100, 3, roots=2, reverse=False)
    insts.append(configs.Instance(n, e, grammars.same_generation(), "hier2100"))
    n, e = graphs.erdos_renyi(600, 40000, 43, labels=2)
    insts.append(configs.Instance(n, e, grammars.dyck(), "er600_dense"))
    _say("row-gather batch", [i.tag for i in insts])
    on = cfpq.batch_closure([(i.n, i.edges, i.grammar) for i in insts], hybrid=1, dirty=dirty)
    off = cfpq.batch_closure([(i.n, i.edges, i.grammar) for i in insts], hybrid=0, dirty=dirty)
    for inst, a, b in zip(insts, on, off):
        want = worklist.closure(inst.n, inst.edges, inst.grammar)
        assert np.array_equal(cfpq.result_bits(a), want), inst.tag
        assert np.array_equal(cfpq.result_bits(b), want), inst.tag
        assert a.stats["converged"] == 1
        assert a.stats["iterations"] > 2 or inst.tag == "er600_dense"  # the push loops ran


def test_batch_grammar_with_many_rules(cfpq):
    """A grammar with more binary rules than the resident kernel keeps in LDS
    (300 rules over 24 nonterminals), on small graphs (one workgroup each,
    the rule table read in place) and on one that takes the tiles, against the
    oracle."""
    rng = np.random.default_rng(71)
    n_nt = 24
    rules = set()
    while len(rules) < 300:
        rules.add(tuple(int(x) for x in rng.integers(0, n_nt, 3)))
    g = grammars.CNF(tuple(f"N{i}" for i in range(n_nt)), ("a", "b"),
                     tuple((i, i % 2) for i in range(0, n_nt, 3)), tuple(sorted(rules)), "many_rules")
    insts = []
    for k, (n, m) in enumerate(((60, 90), (200, 250), (700, 900))):
        n, e = graphs.erdos_renyi(n, m, 72 + k, labels=2)
        insts.append(configs.Instance(n, e, g, f"many_rules_er{n}"))
    _say("many rules", [i.tag for i in insts])
    res = cfpq.batch_closure([(i.n, i.edges, i.grammar) for i in insts])
    for inst, r in zip(insts, res):
        assert np.array_equal(cfpq.result_bits(r), worklist.closure(inst.n, inst.edges, inst.grammar)), inst.tag
