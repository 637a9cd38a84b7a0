"""Front end: grammar text -> normal form, N-Triples -> labelled graph.

The conversion is pinned against the definition of the languages (every
word up to a length bound that each input nonterminal derives, computed by
``oracle.brute.cfg_words`` straight from the rules) through CYK on the
converted grammar, and against the hand-converted query grammars of the
paper's evaluation (section 6) through the relational oracle."""
from __future__ import annotations

import itertools

import numpy as np
import pytest

from oracle import brute, worklist
from paper_1707_01007_amd import frontend
from workloads import grammars, graphs

QUERY1 = """
# same-generation query: S -> sc^-1 S sc | ty^-1 S ty | sc^-1 sc | ty^-1 ty
S -> sc_r S sc | ty_r S ty | sc_r sc | ty_r ty
"""
QUERY2 = """
# adjacent layers: S -> B sc | sc ; B -> sc^-1 B sc | sc^-1 sc
S -> B sc | sc
B -> sc_r B sc | sc_r sc
"""


def _check_language(text, alphabet, max_len):
    cfg = frontend.parse_grammar(text)
    cnf = frontend.to_cnf(cfg, terminals=alphabet)
    want = brute.cfg_words(cfg.rules, max_len)
    for L in range(1, max_len + 1):
        for word in itertools.product(range(len(alphabet)), repeat=L):
            tab = brute.cyk_table(list(word), cnf)[0][L]
            for a in cfg.nonterminals:
                derived = tuple(alphabet[x] for x in word) in want[a]
                assert (cnf.nt(a) in tab) == derived, (text, a, word)


@pytest.mark.parametrize("text", [
    "S -> a S b | eps",                                   # nullable start
    "S -> a S b S | b S a S |",                            # empty alternative, long rules
    "S -> A B\nA -> a | eps\nB -> b | A",                  # unit rules through nullable
    "S -> A | b S\nA -> B\nB -> a B | a | S a",            # unit cycle S -> A -> B -> ... S
    "E -> E p T | T\nT -> T m F | F\nF -> l E r | x",      # arithmetic expressions
])
def test_conversion_preserves_nonempty_languages(text):
    alphabet = sorted(set(frontend.parse_grammar(text).terminals()))
    _check_language(text, alphabet, 6 if len(alphabet) <= 2 else 5)


def test_random_grammars():
    rng = np.random.default_rng(1)
    for case in range(12):
        nts = ["S", "X", "Y"]
        lines = []
        for a in nts:
            alts = []
            for _ in range(int(rng.integers(1, 4))):
                k = int(rng.integers(0, 4))
                alts.append(" ".join(str(rng.choice(nts + ["a", "b"])) for _ in range(k)) or "eps")
            lines.append(f"{a} -> " + " | ".join(alts))
        _check_language("\n".join(lines), ["a", "b"], 6)


@pytest.mark.parametrize("text,hand", [(QUERY1, grammars.same_generation), (QUERY2, grammars.adjacent_layers)])
def test_query_grammars_match_the_hand_conversions(text, hand):
    h = hand()
    g = frontend.grammar_from_text(text, terminals=h.terminals)
    for reverse in (False, True):
        n, e = graphs.hierarchy(500, 3, roots=4, reverse=reverse)
        a = worklist.unpack(worklist.closure(n, e, g), n)[g.nt("S")]
        b = worklist.unpack(worklist.closure(n, e, h), n)[h.nt("S")]
        assert np.array_equal(a, b)


def test_normal_form_shape():
    g = frontend.grammar_from_text("S -> a S b c | S S | eps | d", name="t")
    assert all(0 <= x < g.n_terminals for _, x in g.term)
    assert all(max(r) < g.n_nonterminals for r in g.bin)
    assert g.nonterminals[0] == "S" and g.name == "t"


NT_DOC = """
# a small made-up ontology
<http://example.org/Cat> <http://www.w3.org/2000/01/rdf-schema#subClassOf> <http://example.org/Mammal> .
<http://example.org/Dog> <http://www.w3.org/2000/01/rdf-schema#subClassOf> <http://example.org/Mammal> .
<http://example.org/Mammal> <http://www.w3.org/2000/01/rdf-schema#subClassOf> <http://example.org/Animal> .
<http://example.org/rex> <http://www.w3.org/1999/02/22-rdf-syntax-ns#type> <http://example.org/Dog> .
<http://example.org/rex> <http://example.org/name> "Rex \\"the dog\\""@en .
_:b0 <http://www.w3.org/1999/02/22-rdf-syntax-ns#type> <http://example.org/Cat> .
"""
NAMES = {"<http://www.w3.org/2000/01/rdf-schema#subClassOf>": "sc",
         "<http://www.w3.org/1999/02/22-rdf-syntax-ns#type>": "ty"}


def test_ntriples_loader():
    rdf = frontend.load_ntriples(NT_DOC, predicate_names=NAMES)
    assert rdf.n == 7
    assert rdf.labels[:4] == ["sc", "sc_r", "ty", "ty_r"]
    node = {t: k for k, t in enumerate(rdf.nodes)}
    lab = {x: k for k, x in enumerate(rdf.labels)}
    e = {tuple(int(v) for v in x) for x in rdf.edges}
    assert len(rdf.edges) == 12
    cat, mammal = node["<http://example.org/Cat>"], node["<http://example.org/Mammal>"]
    assert (cat, lab["sc"], mammal) in e and (mammal, lab["sc_r"], cat) in e
    assert '"Rex \\"the dog\\""@en' in node
    with pytest.raises(ValueError):
        frontend.load_ntriples("<a> <b> .")


def test_same_generation_on_rdf():
    """Query 1 on the made-up ontology.  With edges subject -> object (sc goes
    from a class up to its superclass) the query's sc_r ... sc relates a node
    to itself through a child; with the other direction it relates siblings
    (Cat and Dog, both below Mammal)."""
    g = frontend.grammar_from_text(QUERY1, terminals=["sc", "sc_r", "ty", "ty_r"])
    for flip in (False, True):
        rdf = frontend.load_ntriples(NT_DOC, predicate_names=NAMES, object_to_subject=flip)
        e = frontend.relabel_edges(rdf.edges, rdf.labels, g.terminals)
        assert len(e) == 10  # the name triple's two edges are not query terminals
        rel = worklist.relations(worklist.closure(rdf.n, e, g), rdf.n)[g.nt("S")]
        node = {t: k for k, t in enumerate(rdf.nodes)}
        cat, dog = node["<http://example.org/Cat>"], node["<http://example.org/Dog>"]
        mammal, animal = node["<http://example.org/Mammal>"], node["<http://example.org/Animal>"]
        rex, b0 = node["<http://example.org/rex>"], node["_:b0"]
        if flip:
            assert {(cat, dog), (dog, cat), (cat, cat), (dog, dog), (rex, b0), (mammal, mammal)} <= rel
        else:
            assert {(mammal, mammal), (animal, animal), (dog, dog), (cat, cat)} <= rel
            assert (cat, dog) not in rel and (rex, b0) not in rel
