"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bit-exact everywhere (the whole computation is Boolean).  Cases span the
paper's worked example, the five workload recipes at oracle-friendly sizes,
ragged sizes around the 64/256 tile edges, degenerate inputs, and every
product kernel (dense VALU, dense MFMA, sparse rows, sparse columns, and the
hybrid per-product choice) under both schedules.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys

import numpy as np
import pytest

from oracle import alg1, worklist
from workloads import configs, grammars, graphs

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")
PATHS = ["bits", "mfma", "fp4", "rows", "cols"]
SCHEDULES = ["inplace", "jacobi"]


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


def _run(cfpq, inst, **kw):
    _say(inst.tag, inst.n, kw)
    res = cfpq.closure(inst.n, inst.edges, inst.grammar, **kw)
    return cfpq.result_bits(res), res


def _digest(bits):
    return hashlib.sha256(np.ascontiguousarray(bits).astype("<u8").tobytes()).hexdigest()


# ---------------------------------------------------------------- paper example

@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("capture", [0, 1, 8])
def test_worked_example(cfpq, path, schedule, capture):
    gold = json.load(open(os.path.join(GOLD, "worked_example.json")))
    inst = configs.worked_example()
    bits, res = _run(cfpq, inst, path=path, schedule=schedule, dirty=(schedule == "inplace"), capture=capture)
    rel = worklist.relations(bits, inst.n)
    for name in inst.grammar.nonterminals:
        assert rel[inst.grammar.nt(name)] == {tuple(p) for p in gold["relations"][name]}, name
    if schedule == "jacobi":
        assert res.stats["iterations"] == gold["loops"]["k"] == 6
    assert res.stats["converged"] == 1


@pytest.mark.parametrize("path", PATHS)
def test_two_cycles(cfpq, path):
    inst = configs.config1()
    want = worklist.closure(inst.n, inst.edges, inst.grammar)
    bits, res = _run(cfpq, inst, path=path, schedule="inplace")
    assert np.array_equal(bits, want)


@pytest.mark.parametrize("capture", [0, 64])
def test_two_cycles_jacobi_loop_count(cfpq, capture):
    """8065 loops (Lemma 3 with the closed form; the oracle tests pin it),
    host-driven and with 64 captured loops per graph."""
    inst = configs.config1()
    bits, res = _run(cfpq, inst, path="bits", schedule="jacobi", dirty=True, capture=capture)
    assert res.stats["iterations"] == 8065
    assert np.array_equal(bits, worklist.closure(inst.n, inst.edges, inst.grammar))


# ---------------------------------------------------------------- digests of larger workloads

DIGESTS = json.load(open(os.path.join(GOLD, "digests.json")))
MAKERS = {
    "hierarchy4096_samegen": lambda: configs.config2(),
    "hierarchy4096_rev_samegen": lambda: configs.config2(reverse=True),
    "er16384_induced1024_dyck": lambda: configs.config3_induced(1024),
    "er1024_dyck": lambda: configs.config3(1024),
    "er2048_dyck": lambda: configs.config3(2048),
    "er4096_dyck": lambda: configs.config3(4096),
}


@pytest.mark.parametrize("name", sorted(MAKERS))
@pytest.mark.parametrize("path,hybrid", [("bits", 0), ("mfma", 0), ("fp4", 0), ("rows", 0), ("cols", 0),
                                         ("bits", 1), ("mfma", 1), ("fp4", 1)])
def test_workload_digest(cfpq, name, path, hybrid):
    inst = MAKERS[name]()
    bits, res = _run(cfpq, inst, path=path, hybrid=hybrid)
    d = DIGESTS[name]
    got = [int(np.unpackbits(b.view(np.uint8)).sum()) for b in bits]
    assert got == d["counts"]
    assert _digest(bits) == d["sha256"]


def test_host_loop_equals_captured_loop(cfpq):
    """Same loop counts and products with and without device-side loop control."""
    inst = configs.config3(1024)
    for schedule in SCHEDULES:
        a, ra = _run(cfpq, inst, path="bits", schedule=schedule, capture=0)
        b, rb = _run(cfpq, inst, path="bits", schedule=schedule, capture=3)
        assert np.array_equal(a, b)
        if schedule == "jacobi":
            assert ra.stats["iterations"] == rb.stats["iterations"]
            assert ra.stats["products"] == rb.stats["products"]


def test_jacobi_equals_inplace_er(cfpq):
    inst = configs.config3(1024)
    a, ra = _run(cfpq, inst, path="mfma", schedule="jacobi", dirty=False)
    b, rb = _run(cfpq, inst, path="bits", schedule="inplace", dirty=True)
    assert np.array_equal(a, b)
    assert rb.stats["iterations"] <= ra.stats["iterations"]


# ---------------------------------------------------------------- ragged sizes, random grammars

RAGGED = [1, 2, 63, 64, 65, 127, 200, 255, 256, 257, 300, 511, 513, 700]


@pytest.mark.parametrize("n", RAGGED)
@pytest.mark.parametrize("path", PATHS)
def test_ragged_sizes(cfpq, n, path):
    g = grammars.dyck()
    _, e = graphs.erdos_renyi(n, max(1, 2 * n), 1000 + n, labels=2)
    inst = configs.Instance(n, e, g, f"er{n}")
    want = worklist.closure(n, e, g)
    bits, _ = _run(cfpq, inst, path=path, schedule="inplace")
    assert np.array_equal(bits, want)


@pytest.mark.parametrize("name", ["same_generation", "adjacent_layers", "anbn", "transitive_closure"])
@pytest.mark.parametrize("path", PATHS)
def test_grammars_on_hierarchy_and_er(cfpq, name, path):
    g = grammars.BY_NAME[name]()
    if g.terminals == grammars.HIERARCHY_TERMINALS:
        n, e = graphs.hierarchy(600, 21, roots=3, reverse=True)
    else:
        n, e = graphs.erdos_renyi(600, 1500, 22, labels=2)
    want = worklist.closure(n, e, g)
    bits, _ = _run(cfpq, configs.Instance(n, e, g, name), path=path, schedule="jacobi")
    assert np.array_equal(bits, want)


# ---------------------------------------------------------------- small closures on the resident kernel

def test_small_default_closure_runs_resident(cfpq):
    """A default closure of at most 512 padded rows runs as a one-instance
    batch (one resident workgroup): the oracle's bits, the same as with a
    forced product path, and a sound subset when max_iters cuts it short."""
    cases = [configs.config1(), configs.worked_example()]
    n, e = graphs.erdos_renyi(500, 1500, 61, labels=2)
    cases.append(configs.Instance(n, e, grammars.dyck(), "er500"))
    n, e = graphs.hierarchy(450, 62, roots=3, reverse=True)
    cases.append(configs.Instance(n, e, grammars.same_generation(), "hier450_rev"))
    for inst in cases:
        _say("resident", inst.tag, inst.n)
        want = worklist.closure(inst.n, inst.edges, inst.grammar)
        res = cfpq.closure(inst.n, inst.edges, inst.grammar)
        assert res.stats["path_used"] == 1 and res.stats["converged"] == 1, inst.tag  # BITS, the resident product
        assert np.array_equal(cfpq.result_bits(res), want), inst.tag
        forced = cfpq.closure(inst.n, inst.edges, inst.grammar, path="fp4")
        assert forced.stats["path_used"] == 5
        assert np.array_equal(cfpq.result_bits(forced), want), inst.tag
    inst = configs.config1()
    part = cfpq.closure(inst.n, inst.edges, inst.grammar, max_iters=50, allow_partial=True)
    assert part.status == -4 and part.stats["iterations"] == 50
    full = worklist.unpack(worklist.closure(inst.n, inst.edges, inst.grammar), inst.n)
    got = worklist.unpack(cfpq.result_bits(part), inst.n)
    assert not (got & ~full).any() and got.any()


def test_small_jacobi_closure_runs_resident(cfpq):
    """Tiny graphs run the Jacobi schedule in the resident kernel (both buffers
    in LDS): Algorithm 1's loop counts (6 on the worked example, 8065 on the
    two cycles) and bits, equal to a forced-path Jacobi closure; a graph whose
    two buffers do not fit takes the ordinary loop with the same results."""
    gold = json.load(open(os.path.join(GOLD, "worked_example.json")))
    for inst, loops in ((configs.worked_example(), gold["loops"]["k"]), (configs.config1(), 8065)):
        _say("resident jacobi", inst.tag)
        res = cfpq.closure(inst.n, inst.edges, inst.grammar, schedule="jacobi", dirty=False)
        assert res.stats["path_used"] == 1 and res.stats["iterations"] == loops, inst.tag
        forced = cfpq.closure(inst.n, inst.edges, inst.grammar, schedule="jacobi", dirty=False, path="bits")
        assert forced.stats["iterations"] == loops
        assert np.array_equal(cfpq.result_bits(res), cfpq.result_bits(forced))
        assert np.array_equal(cfpq.result_bits(res), worklist.closure(inst.n, inst.edges, inst.grammar))
        dirty = cfpq.closure(inst.n, inst.edges, inst.grammar, schedule="jacobi")
        assert dirty.stats["iterations"] == loops and np.array_equal(cfpq.result_bits(dirty), cfpq.result_bits(res))
    # 7 nonterminals at 250 nodes: 2 x 7 x 256 rows x 8 words > 48 KiB, the ordinary loop
    n, e = graphs.hierarchy(250, 63, roots=3, reverse=True)
    g = grammars.same_generation()
    res = cfpq.closure(n, e, g, schedule="jacobi")
    assert np.array_equal(cfpq.result_bits(res), worklist.closure(n, e, g))
    t, loops, _ = alg1.closure(n, e, g)
    assert res.stats["iterations"] == loops


# ---------------------------------------------------------------- degenerate inputs

def test_empty_graph_and_no_edges(cfpq):
    g = grammars.dyck()
    for n in (0, 5):
        res = cfpq.closure(n, np.zeros((0, 3), np.int32), g)
        assert not cfpq.result_bits(res).any()
        assert res.stats["converged"] == 1


def test_no_binary_rules_gives_edge_set(cfpq):
    g = grammars.CNF(("X", "Y"), ("a", "b"), ((0, 0), (1, 0), (1, 1)), (), "terminal_only")
    n, e = graphs.erdos_renyi(100, 300, 5, labels=2)
    res = cfpq.closure(n, e, g)
    assert np.array_equal(cfpq.result_bits(res), worklist.closure(n, e, g))


def test_multi_edges_and_self_loops(cfpq):
    g = grammars.dyck()
    e = np.array([[0, 0, 0], [0, 1, 0], [0, 0, 1], [0, 0, 1], [1, 1, 0], [1, 1, 1]], np.int32)
    res = cfpq.closure(2, e, g)
    assert np.array_equal(cfpq.result_bits(res), worklist.closure(2, e, g))


def test_device_edges_and_invalid_device_edges(cfpq):
    import torch
    g = grammars.dyck()
    n, e = graphs.erdos_renyi(300, 900, 6, labels=2)
    res = cfpq.closure(n, torch.from_numpy(e).cuda(), g)
    assert np.array_equal(cfpq.result_bits(res), worklist.closure(n, e, g))
    bad = e.copy()
    bad[7, 2] = n + 3
    with pytest.raises(cfpq.CfpqError) as ei:
        cfpq.closure(n, torch.from_numpy(bad).cuda(), g)
    assert ei.value.status == -1


@pytest.mark.parametrize("capture", [0, 8])
def test_max_iters_partial_is_sound(cfpq, capture):
    inst = configs.config1()
    res = cfpq.closure(inst.n, inst.edges, inst.grammar, schedule="jacobi", max_iters=100, allow_partial=True,
                       capture=capture)
    assert res.stats["iterations"] == 100
    assert res.status == -4 and res.stats["converged"] == 0
    part = worklist.unpack(cfpq.result_bits(res), inst.n)
    full = worklist.unpack(worklist.closure(inst.n, inst.edges, inst.grammar), inst.n)
    assert not (part & ~full).any()
    # Jacobi after 100 loops holds exactly the triples of derivation height <= 101 (Lemma 3)
    t, _, _ = alg1.closure(inst.n, inst.edges, inst.grammar, max_loops=100)
    assert np.array_equal(part, t)


# ---------------------------------------------------------------- single products

@pytest.mark.parametrize("n", [64, 256, 300, 1000, 2048])
@pytest.mark.parametrize("density", [0.002, 0.05, 0.5])
@pytest.mark.parametrize("path", PATHS)
def test_product_against_boolean_matmul(cfpq, n, density, path):
    import torch
    rng = np.random.default_rng(n + int(density * 1000))
    b = rng.random((n, n)) < density
    c = rng.random((n, n)) < density
    a0 = rng.random((n, n)) < 0.01
    want = a0 | alg1.bool_product(b, c)
    dev = cfpq.upload_bits(n, worklist.pack(np.stack([b, c, a0])))
    _say("product", n, density, path)
    changed = cfpq.product(n, dev[0], dev[1], dev[2], path=path)
    torch.cuda.synchronize()
    got = worklist.unpack(dev[2, :n, : (n + 63) // 64].cpu().numpy().view(np.uint64), n)
    assert np.array_equal(got, want)
    assert int(changed.item()) == int((want != a0).any())
    # repeating the product changes nothing and leaves the flag clear
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    cfpq.product(n, dev[0], dev[1], dev[2], path=path, changed=flag)
    assert int(flag.item()) == 0


def test_popcount(cfpq):
    n = 777
    rng = np.random.default_rng(3)
    d = rng.random((3, n, n)) < 0.2
    dev = cfpq.upload_bits(n, worklist.pack(d))
    assert cfpq.popcount(n, dev, 3) == [int(x.sum()) for x in d]


@pytest.mark.parametrize("n", [1000, 2048])
@pytest.mark.parametrize("tile", [8, 16, 32])
def test_bits_strip_variants(cfpq, n, tile):
    """Every output strip width of the VALU kernel gives the same product."""
    import torch
    rng = np.random.default_rng(40 + tile)
    b = rng.random((n, n)) < 0.03
    c = rng.random((n, n)) < 0.03
    want = alg1.bool_product(b, c)
    dev = cfpq.upload_bits(n, worklist.pack(np.stack([b, c, np.zeros_like(b)])))
    _say("bits strip", n, tile)
    cfpq.product(n, dev[0], dev[1], dev[2], path="bits", tile=tile)
    torch.cuda.synchronize()
    got = worklist.unpack(dev[2, :n, : (n + 63) // 64].cpu().numpy().view(np.uint64), n)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("n", [1, 200, 256, 257, 600, 777, 1024, 1500])
@pytest.mark.parametrize("stages", [2, 3, 5])
def test_fp4_pipeline_depths(cfpq, n, stages):
    """Every fp4 kernel variant (register pipelines of 2 or 3 chunk buffers,
    and the persistent kernel, tile 5) gives the Boolean product, at sizes
    whose 256-k chunk counts leave every remainder of the loop (1, 2, 3, 4
    and 6 chunks) and ragged edges; below 8 x 256 tiles some persistent
    workgroups have no tile at all."""
    import torch
    rng = np.random.default_rng(70 + n + stages)
    b = rng.random((n, n)) < 0.02
    c = rng.random((n, n)) < 0.3
    a0 = rng.random((n, n)) < 0.01
    want = a0 | alg1.bool_product(b, c)
    dev = cfpq.upload_bits(n, worklist.pack(np.stack([b, c, a0])))
    _say("fp4 stages", n, stages)
    changed = cfpq.product(n, dev[0], dev[1], dev[2], path="fp4", tile=stages)
    torch.cuda.synchronize()
    got = worklist.unpack(dev[2, :n, : (n + 63) // 64].cpu().numpy().view(np.uint64), n)
    assert np.array_equal(got, want)
    assert int(changed.item()) == int((want != a0).any())


def test_closure_with_each_fp4_depth(cfpq):
    inst = configs.config3(1024)
    want = worklist.closure(inst.n, inst.edges, inst.grammar)
    for tile in (2, 3, 5):
        for sched in SCHEDULES:
            bits, res = _run(cfpq, inst, path="fp4", tile=tile, schedule=sched)
            assert np.array_equal(bits, want), (tile, sched)


def test_closure_with_each_bits_tile(cfpq):
    inst = configs.config3(1024)
    want = worklist.closure(inst.n, inst.edges, inst.grammar)
    for tile in (8, 16, 32):
        bits, _ = _run(cfpq, inst, path="bits", tile=tile)
        assert np.array_equal(bits, want), tile


@pytest.mark.parametrize("path,hybrid", [("auto", 0), ("auto", 1), ("bits", 1), ("mfma", 0), ("fp4", 0)])
def test_full_size_er16384(cfpq, path, hybrid):
    """The benchmark workload at full size (n = 16384, device-resident edges,
    the benchmark's launch configurations: the dense autotuned kernel, and the
    hybrid choice), bit-exact against the oracle's stored digest."""
    import torch
    inst = configs.config3(16384)
    d = DIGESTS.get("er16384_dyck")
    if d is None:
        pytest.skip("digest for the 16384-node workload not generated")
    _say(inst.tag, path, hybrid)
    res = cfpq.closure(inst.n, torch.from_numpy(inst.edges).cuda(), inst.grammar, path=path, hybrid=hybrid)
    bits = cfpq.result_bits(res)
    assert [int(np.unpackbits(b.view(np.uint8)).sum()) for b in bits] == d["counts"]
    assert _digest(bits) == d["sha256"]
    if hybrid:
        # the three rules with a terminal operand run sparse, S -> S S dense;
        # the last loop, with few new bits, runs S -> S S on its deltas
        assert 0 < res.stats["sparse_products"] < res.stats["products"]
        assert res.stats["delta_products"] > 0
    else:
        assert res.stats["sparse_products"] == 0 and res.stats["delta_products"] == 0


# ---------------------------------------------------------------- hybrid choice

@pytest.mark.parametrize("schedule", SCHEDULES)
def test_hybrid_equals_dense_and_oracle(cfpq, schedule):
    """At a padded size where the hybrid choice is in effect: identical bits
    with and without it, equal to the oracle; loop counts agree (the choice
    changes only how a product is computed, never what it adds)."""
    inst = configs.config3(4096)
    want = worklist.closure(inst.n, inst.edges, inst.grammar)
    a, ra = _run(cfpq, inst, path="mfma", schedule=schedule, hybrid=0, capture=0)
    b, rb = _run(cfpq, inst, path="mfma", schedule=schedule, hybrid=1)
    assert np.array_equal(a, want) and np.array_equal(b, want)
    assert rb.stats["sparse_products"] > 0
    assert ra.stats["sparse_products"] == 0
    if schedule == "jacobi":
        assert ra.stats["iterations"] == rb.stats["iterations"]
    # the dense products are the only ones counted as bit-operations
    npad = cfpq.padded_rows(inst.n)
    dense = rb.stats["products"] - rb.stats["sparse_products"]
    assert rb.stats["bitops"] == 2.0 * npad ** 3 * dense


@pytest.mark.parametrize("schedule", SCHEDULES)
def test_hybrid_without_dirty_worklist(cfpq, schedule):
    """Hybrid choice with the dirty-rule worklist off: a rule whose operands
    gained nothing in the last loop has empty delta halves, so it launches
    nothing and is not counted -- the same rules the worklist skips, so the
    loop, product and bit-op counts equal those with the worklist on."""
    inst = configs.config3(4096)
    want = worklist.closure(inst.n, inst.edges, inst.grammar)
    a, ra = _run(cfpq, inst, path="fp4", schedule=schedule, hybrid=1, dirty=True)
    b, rb = _run(cfpq, inst, path="fp4", schedule=schedule, hybrid=1, dirty=False)
    assert np.array_equal(a, want) and np.array_equal(b, want)
    for k in ("iterations", "products", "sparse_products", "delta_products", "bitops"):
        assert ra.stats[k] == rb.stats[k], k


@pytest.mark.parametrize("path", ["rows", "cols"])
def test_sparse_paths_under_jacobi_give_algorithm_1_loops(cfpq, path):
    """Jacobi with the sparse products reproduces Algorithm 1's loop count on
    the two-cycle graph (8065, pinned by the oracle tests)."""
    inst = configs.config1()
    bits, res = _run(cfpq, inst, path=path, schedule="jacobi", dirty=True)
    assert res.stats["iterations"] == 8065
    assert res.stats["sparse_products"] == res.stats["products"]
    assert np.array_equal(bits, worklist.closure(inst.n, inst.edges, inst.grammar))


# ---------------------------------------------------------------- warm start

@pytest.mark.parametrize("path", PATHS)
def test_warm_start_resumes_a_partial_result(cfpq, path):
    """A result cut short by max_iters (a sound subset of R) continues to R."""
    inst = configs.config3(1024)
    want = worklist.closure(inst.n, inst.edges, inst.grammar)
    _say("warm start partial", path)
    part = cfpq.closure(inst.n, inst.edges, inst.grammar, path=path, max_iters=2, allow_partial=True)
    assert part.status == -4
    assert not np.array_equal(cfpq.result_bits(part), want)
    res = cfpq.closure(inst.n, inst.edges, inst.grammar, path=path, out=part.bits.view(-1), warm_start=True)
    assert np.array_equal(cfpq.result_bits(res), want)


@pytest.mark.parametrize("schedule", SCHEDULES)
def test_warm_start_after_adding_edges(cfpq, schedule):
    """R of a graph is a subset of R of the graph with more edges
    (monotonicity), so it is a valid starting point for the larger graph."""
    inst = configs.config3(2048)
    half = inst.edges[: len(inst.edges) // 2]
    _say("warm start edges", schedule)
    first = cfpq.closure(inst.n, half, inst.grammar, schedule=schedule)
    assert np.array_equal(cfpq.result_bits(first), worklist.closure(inst.n, half, inst.grammar))
    res = cfpq.closure(inst.n, inst.edges, inst.grammar, schedule=schedule, out=first.bits.view(-1),
                       warm_start=True)
    assert np.array_equal(cfpq.result_bits(res), worklist.closure(inst.n, inst.edges, inst.grammar))


@pytest.mark.parametrize("path", ["rows", "cols"])
@pytest.mark.parametrize("n", [300, 2048, 4100])
def test_sparse_products_with_skewed_rows(cfpq, path, n):
    """A few rows (and columns) far denser than the rest: the row product
    splits long rows over several wavefronts and ORs their parts atomically."""
    import torch
    rng = np.random.default_rng(n + 7)
    b = rng.random((n, n)) < 0.001
    c = rng.random((n, n)) < 0.001
    b[[0, n // 2, n - 1], :] = rng.random((3, n)) < 0.7
    c[:, [1, n // 3]] = rng.random((n, 2)) < 0.7
    c[[2, n - 2], :] = rng.random((2, n)) < 0.6
    a0 = rng.random((n, n)) < 0.002
    want = a0 | alg1.bool_product(b, c)
    dev = cfpq.upload_bits(n, worklist.pack(np.stack([b, c, a0])))
    _say("skewed product", n, path)
    changed = cfpq.product(n, dev[0], dev[1], dev[2], path=path)
    torch.cuda.synchronize()
    got = worklist.unpack(dev[2, :n, : (n + 63) // 64].cpu().numpy().view(np.uint64), n)
    assert np.array_equal(got, want)
    assert int(changed.item()) == 1
