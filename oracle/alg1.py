"""Algorithm 1 of the paper, written out with numpy (test infrastructure only).

The matrix T of section 4 has subsets of N as elements; here it is held as one
Boolean n x n matrix per nonterminal, T[A][i, j] = (A in T_ij).  The product of
section 2, c_ij = union_k a_ik . b_kj with N1 . N2 = {A : B in N1, C in N2,
A -> B C}, becomes one Boolean matrix product per binary rule:
(T x T)[A] = OR over rules A -> B C of (T[B] @ T[C]).

``closure`` computes the least fixpoint of Algorithm 1 (section 4.2) by
simultaneous (Jacobi) updates: T starts as the edge matrix, and each loop
forms the union of T with T x T computed entirely from the previous loop's T,
stopping after the first loop that adds no entry.  The returned count includes
that last loop; the section 4.3 example pins it (six loops, the sixth adding
nothing).
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np


def initial_matrix(n: int, edges: np.ndarray, grammar) -> np.ndarray:
    """T_ij = {A : (i, x, j) in E and A -> x}; multi-edges contribute the union."""
    t = np.zeros((grammar.n_nonterminals, n, n), dtype=bool)
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 3)
    for a, x in grammar.term:
        sel = e[e[:, 1] == x]
        t[a, sel[:, 0], sel[:, 2]] = True
    return t


def bool_product(b: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Boolean matrix product; float64 sums of 0/1 terms are exact below 2**53."""
    return (b.astype(np.float64) @ c.astype(np.float64)) > 0.5


def matrix_product(t: np.ndarray, grammar) -> np.ndarray:
    """(T x T) of section 2: the subset product, one Boolean product per rule."""
    out = np.zeros_like(t)
    for a, b, c in grammar.bin:
        out[a] |= bool_product(t[b], t[c])
    return out


def closure(n: int, edges: np.ndarray, grammar, max_loops: int | None = None,
            keep_history: bool = False) -> Tuple[np.ndarray, int, List[np.ndarray]]:
    """Return (T^cf, loop count, [T_0, T_1, ...] if ``keep_history``)."""
    t = initial_matrix(n, edges, grammar)
    history = [t.copy()] if keep_history else []
    loops = 0
    while True:
        if max_loops is not None and loops >= max_loops:
            break
        new = t | matrix_product(t, grammar)
        loops += 1
        changed = bool((new != t).any())
        t = new
        if keep_history:
            history.append(t.copy())
        if not changed:
            break
    return t, loops, history


def valiant_plus(n: int, edges: np.ndarray, grammar, max_len: int) -> np.ndarray:
    """Valiant's closure of section 2 truncated at ``max_len``:
    union over i <= max_len of a_+^(i), a_+^(1) = a,
    a_+^(i) = union_{j < i} a_+^(j) x a_+^(i-j).  Entry (A, i, j) of a_+^(l)
    means a path of exactly l edges from i to j derives from A."""
    parts = [None, initial_matrix(n, edges, grammar)]
    for i in range(2, max_len + 1):
        acc = np.zeros_like(parts[1])
        for j in range(1, i):
            acc |= matrix_product_pair(parts[j], parts[i - j], grammar)
        parts.append(acc)
    out = np.zeros_like(parts[1])
    for p in parts[1:]:
        out |= p
    return out


def matrix_product_pair(x: np.ndarray, y: np.ndarray, grammar) -> np.ndarray:
    """x x y for two different matrices (same product as ``matrix_product``)."""
    out = np.zeros_like(x)
    for a, b, c in grammar.bin:
        out[a] |= bool_product(x[b], y[c])
    return out
