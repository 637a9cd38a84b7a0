"""The environment switches of cfpq_closure: CFPQ_PATH replaces the AUTO
product choice (same bits as the oracle, the named kernel used), and CFPQ_LOG
receives one JSON line per host-driven loop, per captured replay and per call,
consistent with the call's own statistics."""
from __future__ import annotations

import json

import numpy as np
import pytest

from oracle import worklist
from workloads import configs, graphs, grammars

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cfpq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_01007_amd as m
    m.lib()
    return m


def _events(path):
    with open(path) as f:
        return [json.loads(line) for line in f if line.strip()]


def test_log_lines_follow_the_loops(cfpq, tmp_path, monkeypatch):
    log = tmp_path / "cfpq.jsonl"
    monkeypatch.setenv("CFPQ_LOG", str(log))
    inst = configs.worked_example()
    res = cfpq.closure(inst.n, inst.edges, inst.grammar, path="bits", schedule="jacobi", capture=0)
    ev = _events(log)
    loops = [e for e in ev if e["event"] == "loop"]
    calls = [e for e in ev if e["event"] == "closure"]
    assert [e["loop"] for e in loops] == list(range(1, res.stats["iterations"] + 1))
    assert res.stats["iterations"] == 6  # the section 4.3 example (simultaneous update)
    assert all(e["changed"] > 0 for e in loops[:-1]) and loops[-1]["changed"] == 0
    assert loops[-1]["products"] == res.stats["products"]
    assert len(calls) == 1 and calls[0]["iterations"] == 6 and calls[0]["path"] == "bits"
    assert calls[0]["products"] == res.stats["products"] and calls[0]["captured"] == 0
    assert calls[0]["n"] == inst.n and calls[0]["converged"] == 1
    # captured loops: one line per replay, then the call's line
    log.unlink()
    res = cfpq.closure(inst.n, inst.edges, inst.grammar, path="bits", schedule="jacobi", capture=4)
    ev = _events(log)
    reps = [e for e in ev if e["event"] == "replay"]
    assert [e["replay"] for e in reps] == list(range(1, len(reps) + 1)) and reps[-1]["done"] == 1
    assert reps[-1]["loops"] == res.stats["iterations"] == 6
    assert ev[-1]["event"] == "closure" and ev[-1]["captured"] == 4 and ev[-1]["iterations"] == 6
    # a small graph on the resident route logs its call too
    log.unlink()
    res = cfpq.closure(inst.n, inst.edges, inst.grammar)
    ev = _events(log)
    assert len(ev) == 1 and ev[0]["path"] == "resident" and ev[0]["iterations"] == res.stats["iterations"]


def test_log_of_a_hybrid_closure(cfpq, tmp_path, monkeypatch):
    """The hybrid closure (padded side 4608: dense, row-gather and delta
    products chosen per loop) logs every loop; its running counts end at the
    call's statistics."""
    log = tmp_path / "hybrid.jsonl"
    monkeypatch.setenv("CFPQ_LOG", str(log))
    n, e = graphs.erdos_renyi(4500, 13500, 43, labels=2)
    g = grammars.anbn()
    res = cfpq.closure(n, e, g)
    assert np.array_equal(cfpq.result_bits(res), worklist.closure(n, e, g))
    ev = _events(log)
    loops = [x for x in ev if x["event"] == "loop"]
    call = ev[-1]
    assert call["event"] == "closure" and call["hybrid"] == 1 and call["iterations"] == res.stats["iterations"]
    assert [x["loop"] for x in loops] == list(range(1, res.stats["iterations"] + 1))
    assert loops[-1]["changed"] == 0 and all(x["changed"] > 0 for x in loops[:-1])
    assert loops[-1]["products"] == res.stats["products"] == call["products"]
    assert loops[-1]["sparse_products"] == res.stats["sparse_products"] == call["sparse_products"]
    assert loops[-1]["delta_products"] == res.stats["delta_products"] == call["delta_products"]
    assert res.stats["sparse_products"] > 0
    counts = [x["products"] for x in loops]
    assert counts == sorted(counts)


@pytest.mark.parametrize("name,code", [("rows", 3), ("cols", 4), ("bits", 1), ("fp4", 5)])
def test_path_variable_replaces_auto(cfpq, monkeypatch, name, code):
    n, e = graphs.erdos_renyi(700, 2100, 41, labels=2)
    g = grammars.dyck()
    want = worklist.closure(n, e, g)
    monkeypatch.setenv("CFPQ_PATH", name)
    res = cfpq.closure(n, e, g)
    assert res.stats["path_used"] == code
    assert np.array_equal(cfpq.result_bits(res), want)
    # an explicit path is left alone
    res = cfpq.closure(n, e, g, path="mfma")
    assert res.stats["path_used"] == 2
    assert np.array_equal(cfpq.result_bits(res), want)


def test_unknown_path_value_is_ignored(cfpq, monkeypatch):
    n, e = graphs.erdos_renyi(700, 2100, 42, labels=2)
    g = grammars.dyck()
    monkeypatch.setenv("CFPQ_PATH", "nonsense")
    res = cfpq.closure(n, e, g)
    monkeypatch.delenv("CFPQ_PATH")
    ref = cfpq.closure(n, e, g)
    assert res.stats["path_used"] == ref.stats["path_used"]
    assert np.array_equal(cfpq.result_bits(res), worklist.closure(n, e, g))
