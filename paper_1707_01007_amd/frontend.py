"""Front end: grammars as text, conversion to the normal form the closure
takes, and RDF triples as labelled graphs (host-side preparation; the query
itself runs in the HIP library).

* ``parse_grammar(text)``: rules ``A -> alpha | beta`` one nonterminal per
  line; a symbol is a nonterminal iff it heads some rule, every other symbol
  is a terminal; ``eps`` (or an empty alternative) is the empty word.
* ``to_cnf(cfg)``: the normal form of section 2 (rules ``A -> B C`` and
  ``A -> x``, no start symbol, no empty word).  Classical steps: terminals in
  long rules get their own nonterminal, long rules are split into binary
  ones, empty-word rules are removed by adding the variants without nullable
  symbols, unit rules ``A -> B`` are replaced by the rules of B.  Every
  nonterminal of the input keeps its name and derives the same non-empty
  words (the closure never relates a node to itself by the empty path, so
  the empty word has no meaning there).
* ``load_ntriples(text)``: an N-Triples document as a graph: subjects and
  objects become nodes, each triple ``(s, p, o)`` gives the edges
  ``s -p-> o`` and ``o -p_r-> s`` (the inverse label the paper adds when it
  converts RDF graphs, section 6).
"""
from __future__ import annotations

import re
from dataclasses import dataclass, field
from typing import Dict, List, Sequence, Tuple

import numpy as np

EPS_NAMES = ("eps", "epsilon", "ε")


@dataclass
class CFG:
    """A context-free grammar: rules[A] = list of alternatives, each a tuple
    of symbols (empty tuple = the empty word)."""
    rules: Dict[str, List[Tuple[str, ...]]] = field(default_factory=dict)
    order: List[str] = field(default_factory=list)  # nonterminals in first-seen order

    @property
    def nonterminals(self) -> List[str]:
        return list(self.order)

    def terminals(self) -> List[str]:
        seen: List[str] = []
        for a in self.order:
            for alt in self.rules[a]:
                for x in alt:
                    if x not in self.rules and x not in seen:
                        seen.append(x)
        return seen


def parse_grammar(text: str) -> CFG:
    g = CFG()
    lines = []
    for raw in text.splitlines():
        line = raw.split("#", 1)[0].strip()
        if not line:
            continue
        if "->" not in line:
            raise ValueError(f"not a rule: {raw!r}")
        head, body = line.split("->", 1)
        head = head.strip()
        if not re.fullmatch(r"\S+", head):
            raise ValueError(f"bad rule head: {raw!r}")
        lines.append((head, body))
        if head not in g.rules:
            g.rules[head] = []
            g.order.append(head)
    for head, body in lines:
        for alt in body.split("|"):
            syms = tuple(s for s in alt.split() if s not in EPS_NAMES)
            if syms not in g.rules[head]:
                g.rules[head].append(syms)
    return g


@dataclass(frozen=True)
class CNFGrammar:
    """Normal-form grammar with dense ids, the shape the binding takes."""
    nonterminals: Tuple[str, ...]
    terminals: Tuple[str, ...]
    term: Tuple[Tuple[int, int], ...]
    bin: Tuple[Tuple[int, int, int], ...]
    name: str = ""

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


def to_cnf(cfg: CFG, terminals: Sequence[str] | None = None, name: str = "") -> CNFGrammar:
    """Normal form preserving every input nonterminal's non-empty words.
    ``terminals`` fixes the terminal ids (default: first-seen order)."""
    rules: Dict[str, List[Tuple[str, ...]]] = {a: list(alts) for a, alts in cfg.rules.items()}
    order = list(cfg.order)
    is_nt = set(order)
    terms = list(terminals) if terminals is not None else cfg.terminals()
    for x in cfg.terminals():
        if x not in terms:
            raise ValueError(f"terminal {x!r} is not in the given alphabet")

    def fresh(base: str) -> str:
        k, cand = 0, base
        while cand in is_nt or cand in terms:
            k += 1
            cand = f"{base}_{k}"
        is_nt.add(cand)
        order.append(cand)
        rules[cand] = []
        return cand

    # 1. a terminal inside a rule of length >= 2 gets a nonterminal of its own
    term_nt: Dict[str, str] = {}
    for a in list(order):
        new_alts = []
        for alt in rules[a]:
            if len(alt) >= 2:
                alt2 = []
                for x in alt:
                    if x in is_nt:
                        alt2.append(x)
                    else:
                        if x not in term_nt:
                            t = fresh(f"T_{x}")
                            rules[t] = [(x,)]
                            term_nt[x] = t
                        alt2.append(term_nt[x])
                alt = tuple(alt2)
            new_alts.append(alt)
        rules[a] = new_alts
    # 2. split rules longer than two symbols
    for a in list(order):
        new_alts = []
        for alt in rules[a]:
            head = a
            while len(alt) > 2:
                rest = fresh(f"{a}_r")
                if head == a:
                    new_alts.append((alt[0], rest))
                else:
                    rules[head].append((alt[0], rest))
                head, alt = rest, alt[1:]
            if head == a:
                new_alts.append(alt)
            else:
                rules[head].append(alt)
        rules[a] = new_alts
    # 3. remove the empty word: nullable symbols may be dropped from binary rules
    nullable = set()
    changed = True
    while changed:
        changed = False
        for a in order:
            if a in nullable:
                continue
            if any(all(x in nullable for x in alt) for alt in rules[a]):
                nullable.add(a)
                changed = True
    for a in order:
        new_alts = []
        for alt in rules[a]:
            variants = [alt]
            if len(alt) == 2:
                if alt[0] in nullable:
                    variants.append((alt[1],))
                if alt[1] in nullable:
                    variants.append((alt[0],))
            for v in variants:
                if v and v not in new_alts:
                    new_alts.append(v)
        rules[a] = new_alts
    # 4. replace unit rules A -> B by B's other rules (over the unit closure)
    unit: Dict[str, set] = {a: {a} for a in order}
    changed = True
    while changed:
        changed = False
        for a in order:
            for alt in rules[a]:
                if len(alt) == 1 and alt[0] in is_nt:
                    for c in list(unit[alt[0]]):
                        if c not in unit[a]:
                            unit[a].add(c)
                            changed = True
    final: Dict[str, List[Tuple[str, ...]]] = {}
    for a in order:
        alts = []
        for b in sorted(unit[a], key=order.index):
            for alt in rules[b]:
                if len(alt) == 1 and alt[0] in is_nt:
                    continue
                if alt not in alts:
                    alts.append(alt)
        final[a] = alts
    nt_id = {a: k for k, a in enumerate(order)}
    t_id = {x: k for k, x in enumerate(terms)}
    term, binr = [], []
    for a in order:
        for alt in final[a]:
            if len(alt) == 1:
                term.append((nt_id[a], t_id[alt[0]]))
            else:
                binr.append((nt_id[a], nt_id[alt[0]], nt_id[alt[1]]))
    return CNFGrammar(tuple(order), tuple(terms), tuple(term), tuple(binr), name)


def grammar_from_text(text: str, terminals: Sequence[str] | None = None, name: str = "") -> CNFGrammar:
    return to_cnf(parse_grammar(text), terminals, name)


# ---------------------------------------------------------------- RDF

_TERM = r'(<[^>]*>|_:\S+|"(?:[^"\\]|\\.)*"(?:@[A-Za-z0-9-]+|\^\^<[^>]*>)?)'
_TRIPLE = re.compile(r"^\s*" + _TERM + r"\s+" + _TERM + r"\s+" + _TERM + r"\s*\.\s*$")


@dataclass
class RdfGraph:
    n: int
    edges: np.ndarray          # int32 [m, 3] (src, label, dst)
    nodes: List[str]           # node id -> RDF term
    labels: List[str]          # label id -> predicate (and predicate + "_r" for the inverse)


def load_ntriples(text: str, inverse_suffix: str = "_r", predicate_names: Dict[str, str] | None = None,
                  object_to_subject: bool = False) -> RdfGraph:
    """Parse N-Triples; predicates are named by ``predicate_names[iri]`` when
    given (e.g. {"<...#subClassOf>": "sc"}), else by their IRI text.  A
    triple (s, p, o) gives s -p-> o and o -p_r-> s; with ``object_to_subject``
    the directions swap (o -p-> s and s -p_r-> o).  Section 6 does not fix
    which of the two its conversion means, and the answers of a query like
    same-generation depend on it."""
    nodes: Dict[str, int] = {}
    labels: Dict[str, int] = {}
    node_list: List[str] = []
    label_list: List[str] = []

    def node(t: str) -> int:
        if t not in nodes:
            nodes[t] = len(node_list)
            node_list.append(t)
        return nodes[t]

    def label(name: str) -> int:
        if name not in labels:
            labels[name] = len(label_list)
            label_list.append(name)
        return labels[name]

    edges = []
    for k, raw in enumerate(text.splitlines()):
        line = raw.strip()
        if not line or line.startswith("#"):
            continue
        m = _TRIPLE.match(line)
        if not m:
            raise ValueError(f"line {k + 1}: not an N-Triples statement: {raw!r}")
        s, p, o = m.groups()
        name = (predicate_names or {}).get(p, p)
        fwd, inv = label(name), label(name + inverse_suffix)
        u, v = node(s), node(o)
        if object_to_subject:
            u, v = v, u
        edges.append((u, fwd, v))
        edges.append((v, inv, u))
    e = np.array(edges, dtype=np.int32).reshape(-1, 3)
    return RdfGraph(len(node_list), e, node_list, label_list)


def relabel_edges(edges: np.ndarray, graph_labels: Sequence[str], grammar_terminals: Sequence[str]) -> np.ndarray:
    """Map the graph's label ids onto a grammar's terminal ids; edges whose
    label is not a terminal of the grammar are dropped (they can never be
    part of a derivation)."""
    index = {x: k for k, x in enumerate(grammar_terminals)}
    lut = np.array([index.get(x, -1) for x in graph_labels], dtype=np.int64)
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 3)
    lab = lut[e[:, 1]] if len(e) else np.zeros(0, dtype=np.int64)
    keep = lab >= 0
    out = e[keep].copy()
    out[:, 1] = lab[keep]
    return out.astype(np.int32)
