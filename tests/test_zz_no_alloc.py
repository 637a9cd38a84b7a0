"""cfpq_closure_static: the closure with the library's static device workspace
(no allocation in the call) against cfpq_closure with a caller workspace, bit
for bit, on two calls in a row -- the second on a smaller graph, so it runs on
what the first left in the shared array -- plus concurrent calls from two
threads and the size limit."""
from __future__ import annotations

import sys
import threading

import numpy as np
import pytest

from oracle import worklist
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


def test_static_workspace_equals_caller_workspace(cfpq):
    big = configs.config3(4096)  # hybrid choice on: dense and sparse products, delta snapshots
    n, e = graphs.erdos_renyi(700, 2100, 31, labels=2)
    small = configs.Instance(n, e, grammars.anbn(), "er700_anbn")
    for inst, kw in ((big, {}), (small, {"schedule": "jacobi"})):
        _say("closure_static", inst.tag, inst.n, kw)
        want = cfpq.closure(inst.n, inst.edges, inst.grammar, **kw)
        got = cfpq.closure_static(inst.n, inst.edges, inst.grammar, **kw)
        assert got.status == 0 and got.stats["converged"] == 1
        assert np.array_equal(cfpq.result_bits(got), cfpq.result_bits(want)), inst.tag
        if kw.get("schedule") == "jacobi":  # Algorithm 1's loop count on either path
            assert got.stats["iterations"] == want.stats["iterations"]
    assert np.array_equal(cfpq.result_bits(got), worklist.closure(small.n, small.edges, small.grammar))


def test_static_workspace_two_threads(cfpq):
    """Calls on one GPU from two host threads take turns on the array."""
    import torch
    insts = [configs.config3(2048), configs.config2()]
    want = [cfpq.result_bits(cfpq.closure(i.n, i.edges, i.grammar)) for i in insts]
    got = [None, None]
    dev = torch.cuda.current_device()

    def run(k):
        torch.cuda.set_device(dev)
        s = torch.cuda.Stream()
        r = cfpq.closure_static(insts[k].n, insts[k].edges, insts[k].grammar, stream=s)
        got[k] = cfpq.result_bits(r)

    _say("closure_static from two threads")
    th = [threading.Thread(target=run, args=(k,)) for k in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for k in range(2):
        assert got[k] is not None and np.array_equal(got[k], want[k])


def test_static_workspace_limit(cfpq):
    """A closure whose workspace exceeds the static array is refused before
    any device work, with the sizes in the message."""
    inst = configs.config3(8192)
    with pytest.raises(cfpq.CfpqError) as err:
        cfpq.closure_static(inst.n, inst.edges, inst.grammar)
    assert err.value.status == -2 and "static workspace" in str(err.value)
