"""GPU parity of the continuous-batching server: every query bit-exact
against the oracle, identical alone and in the mix, under admission pressure
and with queries arriving while others run."""
from __future__ import annotations

import hashlib
import json
import os
import sys
import threading
import time

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


def _queries():
    qs = [configs.worked_example(), configs.config1()]
    insts, _ = configs.config5(count=24)
    qs += [i for i in insts if i.n <= 3000]
    n, e = graphs.erdos_renyi(2500, 10000, 9)
    qs.append(configs.Instance(n, e, grammars.dyck(), "er2500"))
    return qs


def test_server_results_match_oracle(cfpq):
    qs = _queries()
    _say("server", len(qs), "queries")
    with cfpq.Server(hbm_budget=4 << 30, max_slots=64) as srv:
        tickets = [srv.submit(q.n, q.edges, q.grammar) for q in qs]
        infos = [srv.wait(t) for t in tickets]
    for q, info in zip(qs, infos):
        assert info["status"] == 0 and info["done"] == 1, q.tag
        assert np.array_equal(cfpq.result_bits(info["result"]), worklist.closure(q.n, q.edges, q.grammar)), q.tag
        assert info["latency_ms"] >= info["run_ms"] >= 0


def test_server_alone_equals_in_mix(cfpq):
    qs = _queries()
    with cfpq.Server(hbm_budget=4 << 30, max_slots=64) as srv:
        mix = [srv.wait(t) for t in [srv.submit(q.n, q.edges, q.grammar) for q in qs]]
        for k in (0, 1, 3, len(qs) - 1):
            alone = srv.wait(srv.submit(qs[k].n, qs[k].edges, qs[k].grammar))
            a = cfpq.result_bits(alone["result"])
            assert np.array_equal(a, cfpq.result_bits(mix[k]["result"])), qs[k].tag
            plain = cfpq.closure(qs[k].n, qs[k].edges, qs[k].grammar)
            assert np.array_equal(a, cfpq.result_bits(plain)), qs[k].tag


def test_server_admission_by_footprint(cfpq):
    """A budget that holds only a couple of large queries at once: later ones
    wait in the queue (queue_ms > 0) and still come out exact."""
    big = []
    for s in range(6):
        n, e = graphs.erdos_renyi(2048, 8192, 50 + s)
        big.append(configs.Instance(n, e, grammars.dyck(), f"er2048_{s}"))
    # each: 4 matrices + 3 transposes of 512 KiB plus edges, about 3.7 MiB
    with cfpq.Server(hbm_budget=12 << 20, max_slots=16) as srv:
        tickets = [srv.submit(q.n, q.edges, q.grammar) for q in big]
        infos = [srv.wait(t) for t in tickets]
    assert max(i["queue_ms"] for i in infos) > 0.0
    for q, info in zip(big, infos):
        assert np.array_equal(cfpq.result_bits(info["result"]), worklist.closure(q.n, q.edges, q.grammar)), q.tag


def test_server_arrivals_while_running(cfpq):
    """Queries submitted from two threads while earlier ones run."""
    qs = _queries()
    out = {}
    with cfpq.Server(hbm_budget=4 << 30, max_slots=32) as srv:
        def client(idx):
            for k in idx:
                out[k] = srv.submit(qs[k].n, qs[k].edges, qs[k].grammar)
                time.sleep(0.0005)
        th = [threading.Thread(target=client, args=(list(range(j, len(qs), 2)),)) for j in range(2)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        infos = {k: srv.wait(t) for k, t in out.items()}
    for k, info in infos.items():
        assert np.array_equal(cfpq.result_bits(info["result"]), worklist.closure(qs[k].n, qs[k].edges, qs[k].grammar))


def test_server_stream_digests(cfpq):
    """All 600 requests the benchmark submits (100 warm-up and 500 measured of
    the seed-5 stream), through a server configured as the benchmark's, against
    stored oracle digests."""
    path = os.path.join(GOLD, "batch_digests.json")
    gold = json.load(open(path))["serve600"]
    insts, _ = configs.config5(count=len(gold))
    with cfpq.Server(hbm_budget=32 << 30, max_slots=512, capture=4) as srv:
        tickets = [srv.submit(i.n, i.edges, i.grammar) for i in insts]
        infos = [srv.wait(t) for t in tickets]
    for k, (inst, info) in enumerate(zip(insts, infos)):
        assert info["status"] == 0, (k, inst.tag)
        bits = cfpq.result_bits(info["result"])
        assert [int(np.unpackbits(b.view(np.uint8)).sum()) for b in bits] == gold[k]["counts"], (k, inst.tag)
        assert _digest(bits) == gold[k]["sha256"], (k, inst.tag)


def test_server_errors(cfpq):
    import torch
    g = grammars.dyck()
    with cfpq.Server(hbm_budget=64 << 20, max_slots=4) as srv:
        with pytest.raises(cfpq.CfpqError) as ei:
            srv.submit(10, np.array([[0, 5, 1]], np.int32), g)
        assert ei.value.status == -1
        n, e = graphs.erdos_renyi(16384, 100, 1)
        with pytest.raises(cfpq.CfpqError) as ei:
            srv.submit(n, e, g)  # 4 matrices of 32 MiB: never fits a 64 MiB budget
        assert ei.value.status == -2
        n, e = graphs.erdos_renyi(300, 900, 2)
        bad = e.copy()
        bad[3, 2] = 301
        t = srv.submit(n, torch.from_numpy(bad).cuda(), g)
        info = srv.wait(t)
        assert info["status"] == -1
        ok = srv.wait(srv.submit(n, e, g))
        assert ok["status"] == 0
        assert np.array_equal(cfpq.result_bits(ok["result"]), worklist.closure(n, e, g))


def test_server_bad_device_edges_on_every_route(cfpq):
    """A request whose device edges hold an id out of range completes with
    CFPQ_EINVAL whichever route runs it -- a resident workgroup (padded side
    <= 512), the engine's tile list (up to 2048) or a hybrid lane (4096 and up)
    -- while the good requests submitted with it are served exactly."""
    import torch
    g = grammars.dyck()
    with cfpq.Server(hbm_budget=2 << 30, max_slots=16) as srv:
        jobs = []
        for size, seed in ((300, 11), (1500, 12), (4500, 13)):
            n, e = graphs.erdos_renyi(size, 3 * size, seed)
            bad = e.copy()
            bad[len(e) // 2, 0] = -1 if size == 1500 else size
            jobs.append((srv.submit(n, torch.from_numpy(bad).cuda(), g), None, None))
            jobs.append((srv.submit(n, torch.from_numpy(e).cuda(), g), n, e))
        for t, n, e in jobs:
            info = srv.wait(t)
            if n is None:
                assert info["status"] == -1
            else:
                assert info["status"] == 0
                assert np.array_equal(cfpq.result_bits(info["result"]), worklist.closure(n, e, g))


def test_server_lanes_equal_engine(cfpq):
    """Large queries (padded side >= 4096) go to the hybrid lanes; the same
    mix served with no lanes (everything in the batched engine) gives the same
    bits, and both equal the plain closure."""
    qs = []
    for s, n in enumerate((4096, 5000, 6000)):
        n_, e = graphs.erdos_renyi(n, 4 * n, 70 + s)
        qs.append(configs.Instance(n_, e, grammars.dyck(), f"er{n}"))
    n_, e = graphs.hierarchy(4500, 71, roots=9, reverse=True)
    qs.append(configs.Instance(n_, e, grammars.same_generation(), "hier4500_rev"))
    qs += [q for q in _queries() if q.n <= 1000][:6]
    results = {}
    for lanes in (0, 2):
        _say("server lanes", lanes)
        with cfpq.Server(hbm_budget=8 << 30, max_slots=32, hybrid_lanes=lanes) as srv:
            infos = [srv.wait(t) for t in [srv.submit(q.n, q.edges, q.grammar) for q in qs]]
        assert all(i["status"] == 0 for i in infos)
        results[lanes] = [cfpq.result_bits(i["result"]) for i in infos]
        if lanes:
            big = [i for q, i in zip(qs, infos) if q.n >= 4096]
            assert all(i["stats"]["sparse_products"] > 0 for i in big)
    for q, a, b in zip(qs, results[0], results[2]):
        assert np.array_equal(a, b), q.tag
        assert np.array_equal(a, cfpq.result_bits(cfpq.closure(q.n, q.edges, q.grammar))), q.tag
    for q, a in zip(qs[:2], results[2][:2]):
        assert np.array_equal(a, worklist.closure(q.n, q.edges, q.grammar)), q.tag


def test_worker_fault_waits_for_the_lane(cfpq):
    """A worker failure (forced from the host: no device work fails) while a
    lane runs a large query.  Queued queries complete with CFPQ_EDEVICE; the
    lane's query completes only after its closure has finished, so the bits
    it reports are whole (equal to the oracle's digest); later submits fail,
    and closing the server reports the failure."""
    from paper_1707_01007_amd import _abi
    gold = json.load(open(os.path.join(GOLD, "digests.json")))["er4096_dyck"]
    big = configs.config3(4096)
    small = [configs.Instance(*graphs.erdos_renyi(n, 3 * n, 60 + n, labels=2), grammars.dyck(), f"er{n}")
             for n in (90, 200, 300, 700, 1100)]
    srv = cfpq.Server(hbm_budget=4 << 30, max_slots=16, hybrid_lanes=1)
    _say("server fault while a lane runs")
    t_big = srv.submit(big.n, big.edges, big.grammar)
    tickets = [srv.submit(i.n, i.edges, i.grammar) for i in small * 4]
    srv.inject_fault()
    info = srv.wait(t_big)
    assert info["status"] in (0, _abi.CFPQ_EDEVICE)
    if info["status"] == 0:  # the lane had started: its result is complete
        bits = cfpq.result_bits(info["result"])
        assert hashlib.sha256(np.ascontiguousarray(bits).astype("<u8").tobytes()).hexdigest() == gold["sha256"]
    _say("lane query status", info["status"])
    for k, t in enumerate(tickets):
        x = srv.wait(t)
        assert x["status"] in (0, _abi.CFPQ_EDEVICE)
        if x["status"] == 0:
            inst = (small * 4)[k]
            assert np.array_equal(cfpq.result_bits(x["result"]), worklist.closure(inst.n, inst.edges, inst.grammar))
    with pytest.raises(cfpq.CfpqError) as err:
        srv.submit(small[0].n, small[0].edges, small[0].grammar)
    assert err.value.status == _abi.CFPQ_EDEVICE
    with pytest.raises(cfpq.CfpqError) as err:
        srv.close()
    assert err.value.status == _abi.CFPQ_EDEVICE
