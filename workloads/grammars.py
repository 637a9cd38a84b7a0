"""CNF grammars used as query inputs.

A grammar is data only: nonterminal and terminal names plus two rule lists,
``term`` = [(A, x)] for A -> x and ``bin`` = [(A, B, C)] for A -> B C, all as
dense 0-based ids.  The grammar form (no start symbol, no epsilon rules) is the
one fixed in the paper's preliminaries (section 2).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple


@dataclass(frozen=True)
class CNF:
    nonterminals: Tuple[str, ...]
    terminals: Tuple[str, ...]
    term: Tuple[Tuple[int, int], ...]          # (A, x): A -> x
    bin: Tuple[Tuple[int, int, int], ...]      # (A, B, C): A -> B C
    name: str = field(default="")

    @property
    def n_nonterminals(self) -> int:
        return len(self.nonterminals)

    @property
    def n_terminals(self) -> int:
        return len(self.terminals)

    def nt(self, name: str) -> int:
        return self.nonterminals.index(name)

    def t(self, name: str) -> int:
        return self.terminals.index(name)

    def relabel_terminals(self, terminals: Sequence[str], mapping: dict) -> "CNF":
        """Same rules over another terminal alphabet; ``mapping`` maps each old
        terminal name to a new one.  Used to pair a grammar with a graph whose
        labels have other names (e.g. a := sc_r, b := sc on a hierarchy)."""
        terminals = tuple(terminals)
        term = tuple((a, terminals.index(mapping[self.terminals[x]])) for a, x in self.term)
        return CNF(self.nonterminals, terminals, term, self.bin, self.name)


def _mk(name: str, nts: List[str], ts: List[str], term, bin_) -> CNF:
    nt = {s: i for i, s in enumerate(nts)}
    t = {s: i for i, s in enumerate(ts)}
    return CNF(
        tuple(nts),
        tuple(ts),
        tuple((nt[a], t[x]) for a, x in term),
        tuple((nt[a], nt[b], nt[c]) for a, b, c in bin_),
        name,
    )


def same_generation() -> CNF:
    """The paper's example query in normal form (section 4.3, the normal-form
    production figure): S -> S1 S5 | S3 S6 | S1 S2 | S3 S4, S5 -> S S2,
    S6 -> S S4, S1 -> sc_r, S2 -> sc, S3 -> ty_r, S4 -> ty.  ``sc`` stands for
    subClassOf, ``ty`` for type and the ``_r`` suffix for the inverse label.
    The same grammar is Query 1 of the evaluation (section 6)."""
    return _mk(
        "same_generation",
        ["S", "S1", "S2", "S3", "S4", "S5", "S6"],
        ["sc", "sc_r", "ty", "ty_r"],
        [("S1", "sc_r"), ("S2", "sc"), ("S3", "ty_r"), ("S4", "ty")],
        [("S", "S1", "S5"), ("S", "S3", "S6"), ("S", "S1", "S2"), ("S", "S3", "S4"),
         ("S5", "S", "S2"), ("S6", "S", "S4")],
    )


def adjacent_layers() -> CNF:
    """Query 2 of the evaluation (section 6): S -> B sc | sc,
    B -> sc_r B sc | sc_r sc, put in normal form by hand:
    S -> B SC, B -> SCR B1 | SCR SC, B1 -> B SC, plus S -> sc, SC -> sc,
    SCR -> sc_r."""
    return _mk(
        "adjacent_layers",
        ["S", "B", "B1", "SC", "SCR"],
        ["sc", "sc_r", "ty", "ty_r"],
        [("S", "sc"), ("SC", "sc"), ("SCR", "sc_r")],
        [("S", "B", "SC"), ("B", "SCR", "B1"), ("B", "SCR", "SC"), ("B1", "B", "SC")],
    )


def anbn() -> CNF:
    """a^n b^n (n >= 1): S -> A S1 | A B, S1 -> S B, A -> a, B -> b."""
    return _mk(
        "anbn",
        ["S", "S1", "A", "B"],
        ["a", "b"],
        [("A", "a"), ("B", "b")],
        [("S", "A", "S1"), ("S", "A", "B"), ("S1", "S", "B")],
    )


def dyck() -> CNF:
    """Dyck-like language S -> S S | a S b | a b in normal form:
    S -> S S | A S1 | A B, S1 -> S B, A -> a, B -> b."""
    return _mk(
        "dyck",
        ["S", "S1", "A", "B"],
        ["a", "b"],
        [("A", "a"), ("B", "b")],
        [("S", "S", "S"), ("S", "A", "S1"), ("S", "A", "B"), ("S1", "S", "B")],
    )


def transitive_closure() -> CNF:
    """S -> S S | a: R_S is the transitive closure of the a-labelled edges
    (b-labelled edges are inert)."""
    return _mk("transitive_closure", ["S"], ["a", "b"], [("S", "a")], [("S", "S", "S")])


HIERARCHY_TERMINALS = ("sc", "sc_r", "ty", "ty_r")


def for_hierarchy(g: CNF) -> CNF:
    """Pair a grammar with a hierarchy graph (labels sc, sc_r, ty, ty_r).
    a^n b^n and Dyck read a := sc_r and b := sc, so ty edges are inert."""
    if g.terminals == HIERARCHY_TERMINALS:
        return g
    return g.relabel_terminals(HIERARCHY_TERMINALS, {"a": "sc_r", "b": "sc"})


BY_NAME = {
    "same_generation": same_generation,
    "adjacent_layers": adjacent_layers,
    "anbn": anbn,
    "dyck": dyck,
    "transitive_closure": transitive_closure,
}


# ---------------------------------------------------------------- conjunctive grammars

@dataclass(frozen=True)
class ConjCNF:
    """Conjunctive grammar in binary normal form (the generalisation named in
    the paper's conclusion): rules A -> x and A -> B1 C1 & ... & Bk Ck (k >= 1;
    k = 1 is an ordinary CNF rule).  Data only."""
    nonterminals: Tuple[str, ...]
    terminals: Tuple[str, ...]
    term: Tuple[Tuple[int, int], ...]                              # (A, x)
    conj: Tuple[Tuple[int, Tuple[Tuple[int, int], ...]], ...]     # (A, ((B1, C1), ..., (Bk, Ck)))
    name: str = field(default="")

    @property
    def n_nonterminals(self) -> int:
        return len(self.nonterminals)

    @property
    def n_terminals(self) -> int:
        return len(self.terminals)

    def nt(self, name: str) -> int:
        return self.nonterminals.index(name)


def conjunctive_from_cnf(g: CNF) -> ConjCNF:
    """The same grammar with every binary rule as a one-conjunct rule."""
    return ConjCNF(g.nonterminals, g.terminals, g.term, tuple((a, ((b, c),)) for a, b, c in g.bin), g.name)


def _mk_conj(name: str, nts: List[str], ts: List[str], term, conj) -> ConjCNF:
    nt = {s: i for i, s in enumerate(nts)}
    t = {s: i for i, s in enumerate(ts)}
    return ConjCNF(tuple(nts), tuple(ts), tuple((nt[a], t[x]) for a, x in term),
                   tuple((nt[a], tuple((nt[b], nt[c]) for b, c in parts)) for a, parts in conj), name)


def anbncn() -> ConjCNF:
    """{a^n b^n c^n : n >= 1} as the intersection of a^n b^n c^+ and a^+ b^n c^n:
    S -> P Cp & Ap Q with P => a^n b^n, Cp => c^+, Ap => a^+, Q => b^n c^n."""
    return _mk_conj("anbncn", ["S", "P", "P1", "Q", "Q1", "Ap", "Cp", "A", "B", "C"], ["a", "b", "c"],
                    [("A", "a"), ("B", "b"), ("C", "c"), ("Ap", "a"), ("Cp", "c")],
                    [("S", [("P", "Cp"), ("Ap", "Q")]),
                     ("P", [("A", "B")]), ("P", [("A", "P1")]), ("P1", [("P", "B")]),
                     ("Q", [("B", "C")]), ("Q", [("B", "Q1")]), ("Q1", [("Q", "C")]),
                     ("Ap", [("A", "Ap")]), ("Cp", [("C", "Cp")])])


def dyck_and_anbn() -> ConjCNF:
    """Words in both Dyck(a, b) and a^n b^n (which is all of a^n b^n): the
    start rules of both grammars, conjoined pairwise; used to check that a
    conjunction never adds what either conjunct lacks."""
    return _mk_conj("dyck_and_anbn", ["S", "D", "D1", "E", "E1", "A", "B"], ["a", "b"],
                    [("A", "a"), ("B", "b")],
                    [("S", [("D", "D"), ("A", "E1")]), ("S", [("D", "D"), ("A", "B")]),
                     ("S", [("A", "D1"), ("A", "E1")]), ("S", [("A", "D1"), ("A", "B")]),
                     ("S", [("A", "B"), ("A", "E1")]), ("S", [("A", "B"), ("A", "B")]),
                     ("D", [("D", "D")]), ("D", [("A", "D1")]), ("D", [("A", "B")]), ("D1", [("D", "B")]),
                     ("E", [("A", "E1")]), ("E", [("A", "B")]), ("E1", [("E", "B")])])
