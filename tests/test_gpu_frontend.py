"""The front end feeding the GPU closure: grammar text converted to normal
form and a generated RDF-style hierarchy written as N-Triples and loaded back
give the same R_S on the GPU as the hand-converted grammar in the oracle."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from oracle import worklist
from paper_1707_01007_amd import frontend
from tests.test_frontend import QUERY1, QUERY2
from workloads import grammars, graphs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cfpq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_01007_amd as m
    m.lib()
    return m


def _as_ntriples(n, edges, labels):
    """Forward edges of a generated hierarchy as N-Triples text (made-up IRIs)."""
    lines = []
    for u, x, v in edges:
        if labels[x].endswith("_r"):
            continue
        lines.append(f"<http://example.org/n{u}> <http://example.org/{labels[x]}> <http://example.org/n{v}> .")
    return "\n".join(lines)


@pytest.mark.parametrize("text,hand", [(QUERY1, grammars.same_generation), (QUERY2, grammars.adjacent_layers)])
def test_text_grammar_and_ntriples_on_gpu(cfpq, text, hand):
    h = hand()
    n, e = graphs.hierarchy(3000, 17, roots=6, reverse=True)
    doc = _as_ntriples(n, e, list(h.terminals))
    names = {f"<http://example.org/{x}>": x for x in ("sc", "ty")}
    rdf = frontend.load_ntriples(doc, predicate_names=names)
    g = frontend.grammar_from_text(text, terminals=h.terminals)
    edges = frontend.relabel_edges(rdf.edges, rdf.labels, g.terminals)
    print("[gpu-case] frontend", hand.__name__, rdf.n, len(edges), file=sys.stderr, flush=True)
    res = cfpq.closure(rdf.n, edges, g)
    got = worklist.unpack(cfpq.result_bits(res), rdf.n)[g.nt("S")]
    want = worklist.unpack(worklist.closure(rdf.n, edges, h), rdf.n)[h.nt("S")]
    assert np.array_equal(got, want)
    assert got.sum() > 0
