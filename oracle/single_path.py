"""Single-path semantics of section 5, written out with numpy (test
infrastructure only).

Section 5 attaches a path length to every nonterminal of the closure of
section 4.  The initial matrix holds (A, 1) in cell (i, j) for every edge
(i, x, j) with A -> x.  When a step of the closure,
a^(p) = a^(p-1) u (a^(p-1) x a^(p-1)), first puts A into cell (i, j) through a
rule A -> B C and a middle node k with (B, l_B) in a^(p-1)_{i,k} and
(C, l_C) in a^(p-1)_{k,j}, the pair gets the length l_B + l_C; a pair already
present keeps its length for good.  The section's lemma and theorem: every
stored length is the length of some path i -> j whose label word A derives.

The section does not say which length a cell keeps when one step can add A
through several (rule, k) choices with different sums; this oracle (like the
GPU path) keeps the smallest, which makes the result unique.

``lengths`` evaluates that definition one simultaneous step at a time (the
step of Algorithm 1): L[A][i, j] = 0 for an absent pair.  ``witness``
recovers one such path: a stored length l > 1 was set as l_B(i, k) + l_C(k, j)
with both stored earlier, each shorter than l, so splitting any cell into two
stored cells whose lengths add up to l recurses down to single edges.
``lengths_native`` runs the same definition in plain C (cfpq_single_path.c)
for graphs of thousands of nodes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Tuple

import numpy as np

INF = np.iinfo(np.int64).max // 4  # absent; INF + INF still fits in int64


def initial_lengths(n: int, edges: np.ndarray, grammar) -> np.ndarray:
    """Length 1 for (A, i, j) with an edge (i, x, j) and A -> x; INF elsewhere."""
    L = np.full((grammar.n_nonterminals, n, n), INF, dtype=np.int64)
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 3)
    for a, x in grammar.term:
        sel = e[e[:, 1] == x]
        L[a, sel[:, 0], sel[:, 2]] = 1
    return L


def min_plus(lb: np.ndarray, lc: np.ndarray) -> np.ndarray:
    """out[i, j] = min over k of lb[i, k] + lc[k, j]; INF where no k has both."""
    n = lb.shape[0]
    out = np.full((n, lc.shape[1]), INF, dtype=np.int64)
    for k in range(n):
        np.minimum(out, lb[:, k:k + 1] + lc[k:k + 1, :], out=out)
    out[out >= INF] = INF
    return out


def lengths(n: int, edges: np.ndarray, grammar, max_loops: int | None = None) -> Tuple[np.ndarray, int]:
    """Return (L, loop count): L[A][i, j] is the section-5 length of (A, i, j),
    0 when (i, j) is not in R_A; the loop count is that of Algorithm 1
    (including the last step, which adds nothing)."""
    L = initial_lengths(n, edges, grammar)
    loops = 0
    while max_loops is None or loops < max_loops:
        cand = np.full_like(L, INF)
        for a, b, c in grammar.bin:
            cand[a] = np.minimum(cand[a], min_plus(L[b], L[c]))
        new = (L == INF) & (cand < INF)
        loops += 1
        if not new.any():
            break
        L = np.where(new, cand, L)
    return np.where(L >= INF, 0, L), loops


def witness(n: int, edges: np.ndarray, grammar, L: np.ndarray, a: int, i: int, j: int) -> List[Tuple[int, int, int]]:
    """A path i -> j of exactly L[a][i, j] edges, as (src, label, dst) triples,
    whose label word ``a`` derives."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 3)
    term_of = {}
    for lhs, x in grammar.term:
        term_of.setdefault(lhs, set()).add(x)
    out: List[Tuple[int, int, int]] = []
    stack = [(a, i, j)]  # cells still to expand, leftmost on top
    budget = 2 * int(L[a, i, j])  # a derivation tree with l leaves has 2l - 1 nodes
    while stack:
        budget -= 1
        if budget < 0:
            raise ValueError("the splits do not add up to the stored length")
        A, s, t = stack.pop()
        l = int(L[A, s, t])
        if l <= 0:
            raise ValueError(f"({A}, {s}, {t}) is not in R_A")
        if l == 1:
            hit = [tuple(int(v) for v in ed) for ed in e
                   if ed[0] == s and ed[2] == t and int(ed[1]) in term_of.get(A, ())]
            if not hit:
                raise ValueError(f"length 1 without an edge for ({A}, {s}, {t})")
            out.append(hit[0])
            continue
        for lhs, b, c in grammar.bin:
            if lhs != A:
                continue
            lb, lc = L[b, s, :], L[c, :, t]
            ks = np.nonzero((lb > 0) & (lc > 0) & (lb + lc == l))[0]
            if len(ks):
                k = int(ks[0])
                stack.append((c, k, t))
                stack.append((b, s, k))
                break
        else:
            raise ValueError(f"no split of length {l} for ({A}, {s}, {t})")
    return out


# ---- the same definition in plain C (cfpq_single_path.c), for larger graphs ----

_C_SRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfpq_single_path.c")
_C_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcfpq_single_path_oracle.so")
_c_lib = None


def build_native(force: bool = False, src: str = _C_SRC, lib: str = _C_LIB) -> str:
    """Compile the C transcription with gcc -O3 (integer code only)."""
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
        tmp = lib + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-o", tmp, src])
        os.replace(tmp, lib)
    return lib


def load_native(path: str):
    lib = ctypes.CDLL(path)
    i32, i64, p = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    lib.cfpq_single_path_oracle.argtypes = [i32, i64, p, i32, i32, i32, p, i32, p, i64, p, p]
    lib.cfpq_single_path_oracle.restype = ctypes.c_int
    return lib


def lengths_native(n: int, edges: np.ndarray, grammar, max_loops: int | None = None, lib=None):
    """``lengths`` computed by the C transcription: returns (L as uint32
    [|N|, n, n], loop count, status) with status 0 (fixpoint reached), 1 (some
    length reached 2^31 - 1) or 3 (stopped by max_loops)."""
    global _c_lib
    if lib is None:
        if _c_lib is None:
            _c_lib = load_native(build_native())
        lib = _c_lib
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 3))
    term = np.ascontiguousarray(np.asarray(grammar.term, dtype=np.int32).reshape(-1, 2))
    binr = np.ascontiguousarray(np.asarray(grammar.bin, dtype=np.int32).reshape(-1, 3))
    out = np.zeros((grammar.n_nonterminals, n, n), dtype=np.uint32)
    loops = ctypes.c_int64(0)
    rc = lib.cfpq_single_path_oracle(n, len(e), e.ctypes.data, grammar.n_nonterminals, grammar.n_terminals,
                                     len(term), term.ctypes.data, len(binr), binr.ctypes.data,
                                     int(max_loops or 0), out.ctypes.data, ctypes.byref(loops))
    if rc == -1:
        raise ValueError("single-path oracle: invalid graph or grammar")
    if rc == -2:
        raise MemoryError("single-path oracle: out of memory")
    return out, int(loops.value), rc
