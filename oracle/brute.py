"""Brute force straight from the definitions of section 2 (test infrastructure).

``cyk_table`` decides A =>* w for every substring of a word (CYK over a CNF
grammar).  ``paths_up_to`` enumerates every path of at most ``max_len`` edges
and records, for each nonterminal A, the pairs (i, j) joined by a path whose
label word A derives: that is R_A of section 2 restricted to paths of bounded
length, so it is a subset of R_A for any bound and equals R_A on a DAG once the
bound reaches n - 1.
"""
from __future__ import annotations

from typing import Dict, List, Set, Tuple


def _by_term(grammar) -> Dict[int, Set[int]]:
    by_term: Dict[int, Set[int]] = {}
    for a, x in grammar.term:
        by_term.setdefault(x, set()).add(a)
    return by_term


def _combine(left: Set[int], right: Set[int], rules) -> Set[int]:
    """N1 . N2 of section 2: {A : B in N1, C in N2, A -> B C}."""
    if not left or not right:
        return set()
    return {a for a, b, c in rules if b in left and c in right}


def cyk_table(word: List[int], grammar) -> List[List[Set[int]]]:
    """table[s][e] = {A : A =>* word[s:e]} for 0 <= s < e <= len(word)."""
    by_term = _by_term(grammar)
    rules = list(grammar.bin)
    L = len(word)
    tab = [[set() for _ in range(L + 1)] for _ in range(L + 1)]
    for s in range(L):
        tab[s][s + 1] = set(by_term.get(word[s], ()))
    for width in range(2, L + 1):
        for s in range(0, L - width + 1):
            e = s + width
            for m in range(s + 1, e):
                tab[s][e] |= _combine(tab[s][m], tab[m][e], rules)
    return tab


def derives(word: List[int], grammar) -> Set[int]:
    if not word:
        return set()
    return cyk_table(word, grammar)[0][len(word)]


def paths_up_to(n: int, edges, grammar, max_len: int) -> Dict[int, Set[Tuple[int, int]]]:
    """{A: {(i, j)}} over all paths of 1..max_len edges (multi-edges and
    self-loops are followed like any other edge).  Along a path the CYK table
    grows by one column per edge: col[e][s] = {A : A =>* labels[s:e]}."""
    by_term = _by_term(grammar)
    rules = list(grammar.bin)
    out_edges: Dict[int, List[Tuple[int, int]]] = {}
    for u, x, v in (tuple(int(t) for t in e) for e in edges):
        out_edges.setdefault(u, []).append((x, v))
    result: Dict[int, Set[Tuple[int, int]]] = {a: set() for a in range(grammar.n_nonterminals)}

    def walk(start: int, node: int, cols: List[List[Set[int]]]):
        depth = len(cols) - 1          # edges on the path so far
        if depth == max_len:
            return
        for x, v in out_edges.get(node, ()):
            e = depth + 1
            new: List[Set[int]] = [set() for _ in range(e)]
            new[e - 1] = set(by_term.get(x, ()))
            for s in range(e - 2, -1, -1):
                for m in range(s + 1, e):
                    new[s] |= _combine(cols[m][s], new[m], rules)
            for a in new[0]:
                result[a].add((start, v))
            cols.append(new)
            walk(start, v, cols)
            cols.pop()

    for start in range(n):
        walk(start, start, [[]])
    return result


def conj_cyk_table(word: List[int], grammar) -> List[List[Set[int]]]:
    """CYK for a conjunctive grammar in binary normal form: A =>* word[s:e]
    through A -> B1 C1 & ... & Bk Ck iff every conjunct m has its own split
    point p with Bm =>* word[s:p] and Cm =>* word[p:e]."""
    by_term = _by_term(grammar)
    L = len(word)
    tab = [[set() for _ in range(L + 1)] for _ in range(L + 1)]
    for s in range(L):
        tab[s][s + 1] = set(by_term.get(word[s], ()))
    for width in range(2, L + 1):
        for s in range(0, L - width + 1):
            e = s + width
            for a, parts in grammar.conj:
                if all(any(b in tab[s][p] and c in tab[p][e] for p in range(s + 1, e)) for b, c in parts):
                    tab[s][e].add(a)
    return tab


def conj_paths_up_to(n: int, edges, grammar, max_len: int) -> Dict[int, Set[Tuple[int, int]]]:
    """{A: {(i, j)}} for every path of 1..max_len edges whose label word A
    derives in the conjunctive grammar (each word checked by conj_cyk_table)."""
    out_edges: Dict[int, List[Tuple[int, int]]] = {}
    for u, x, v in (tuple(int(t) for t in e) for e in edges):
        out_edges.setdefault(u, []).append((x, v))
    result: Dict[int, Set[Tuple[int, int]]] = {a: set() for a in range(grammar.n_nonterminals)}

    def walk(start: int, node: int, word: List[int]):
        if len(word) == max_len:
            return
        for x, v in out_edges.get(node, ()):
            word.append(x)
            for a in conj_cyk_table(word, grammar)[0][len(word)]:
                result[a].add((start, v))
            walk(start, v, word)
            word.pop()

    for start in range(n):
        walk(start, start, [])
    return result


def cfg_words(rules, max_len: int) -> Dict[str, Set[Tuple]]:
    """Every word of length <= max_len that each nonterminal of a general
    context-free grammar derives (the empty word included when derivable).
    ``rules``: {A: [alternative, ...]}, an alternative a tuple of symbols,
    nonterminal iff it is a key.  The least solution of the grammar's
    language equations, restricted to short words (a derivation of a word of
    length <= max_len only uses sub-words of length <= max_len)."""
    words: Dict[str, Set[Tuple]] = {a: set() for a in rules}
    changed = True
    while changed:
        changed = False
        for a, alts in rules.items():
            for alt in alts:
                partial = {()}
                for x in alt:
                    opts = words[x] if x in rules else {(x,)}
                    partial = {p + q for p in partial for q in opts if len(p) + len(q) <= max_len}
                    if not partial:
                        break
                fresh = partial - words[a]
                if fresh:
                    words[a] |= fresh
                    changed = True
    return words
