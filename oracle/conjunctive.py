"""Algorithm 1 generalised to conjunctive grammars (test infrastructure only).

The paper's conclusion notes that the algorithm carries over to conjunctive
grammars, because their parsing is also expressible with matrix products,
and expects the result to over-approximate the conjunctive path query.  For a
rule A -> B1 C1 & ... & Bk Ck the step adds to T_A the cells where every
conjunct's product is set:

    T_A <- T_A | AND over m of (T_Bm x T_Cm)

(each conjunct may be witnessed by a different path between the same two
nodes, hence the over-approximation; on a graph with a single path between
any two nodes, a chain, it is exact).  ``closure`` iterates that step
simultaneously for every rule, as Algorithm 1 does, until nothing changes.
"""
from __future__ import annotations

from typing import Tuple

import numpy as np

from oracle.alg1 import bool_product


def initial_matrix(n: int, edges: np.ndarray, grammar) -> np.ndarray:
    t = np.zeros((grammar.n_nonterminals, n, n), dtype=bool)
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 3)
    for a, x in grammar.term:
        sel = e[e[:, 1] == x]
        t[a, sel[:, 0], sel[:, 2]] = True
    return t


def closure(n: int, edges: np.ndarray, grammar, max_loops: int | None = None) -> Tuple[np.ndarray, int]:
    """Return (T, loop count) for a ConjCNF grammar."""
    t = initial_matrix(n, edges, grammar)
    loops = 0
    while max_loops is None or loops < max_loops:
        new = t.copy()
        for a, parts in grammar.conj:
            acc = np.ones((n, n), dtype=bool)
            for b, c in parts:
                acc &= bool_product(t[b], t[c])
            new[a] |= acc
        loops += 1
        changed = bool((new != t).any())
        t = new
        if not changed:
            break
    return t, loops
