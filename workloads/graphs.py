"""Seeded synthetic edge-labelled graphs.

A graph is ``(n, edges)`` with ``edges`` an int32 array of shape [m, 3] holding
(src, label, dst) triples, nodes numbered 0..n-1 as in the paper's reduction
(section 4.1).  Every generator draws from ``numpy.random.Generator(PCG64(seed))``
so the same seed gives the same graph on every machine.  Nothing here computes
any part of the query: these are inputs only.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

from .grammars import HIERARCHY_TERMINALS

SC, SC_R, TY, TY_R = (HIERARCHY_TERMINALS.index(s) for s in ("sc", "sc_r", "ty", "ty_r"))
A_LABEL, B_LABEL = 0, 1


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _edges(triples) -> np.ndarray:
    e = np.asarray(triples, dtype=np.int32)
    return e.reshape(-1, 3) if e.size else np.zeros((0, 3), dtype=np.int32)


def worked_example() -> Tuple[int, np.ndarray]:
    """The 3-node graph of the paper's example (section 4.3).  Its figure is not
    in the text; the graph is recovered from the printed initial matrix T0
    through the one-to-one terminal rules S1 -> sc_r, S2 -> sc, S3 -> ty_r,
    S4 -> ty: T0 = [[{S1},{S3},-],[-,-,{S3}],[{S2},-,{S4}]]."""
    return 3, _edges([(0, SC_R, 0), (0, TY_R, 1), (1, TY_R, 2), (2, SC, 0), (2, TY, 2)])


def two_cycles(na: int = 64, nb: int = 63) -> Tuple[int, np.ndarray]:
    """An ``na``-node cycle of label a and an ``nb``-node cycle of label b that
    share node 0.  The a-cycle is 0 -> 1 -> ... -> na-1 -> 0; the b-cycle is
    0 -> na -> na+1 -> ... -> na+nb-2 -> 0.  n = na + nb - 1."""
    n = na + nb - 1
    e = [(i, A_LABEL, (i + 1) % na) for i in range(na)]
    bcyc = [0] + list(range(na, n))
    e += [(bcyc[t], B_LABEL, bcyc[(t + 1) % nb]) for t in range(nb)]
    return n, _edges(e)


def forest_parents(n: int, roots: int, rng: np.random.Generator, max_branch: int = 8) -> np.ndarray:
    """Parent array of a random forest built breadth first: nodes 0..roots-1
    are roots; each dequeued node draws U{1..max_branch} children, which take
    the next free ids, until n nodes exist.  parent[root] = -1."""
    parent = np.full(n, -1, dtype=np.int64)
    nxt = roots
    head = 0
    while nxt < n:
        b = int(rng.integers(1, max_branch + 1))
        for _ in range(b):
            if nxt >= n:
                break
            parent[nxt] = head
            nxt += 1
        head += 1
    return parent


def hierarchy(n: int, seed: int, roots: int = 8, ty_frac: float = 0.2, reverse: bool = False,
              rng: np.random.Generator | None = None) -> Tuple[int, np.ndarray]:
    """Class hierarchy: a random forest with sc edges child -> parent, plus
    ``ty_frac * n`` distinct nodes each given one ty edge to a uniform other
    node, plus the inverse edges sc_r / ty_r (the evaluation's RDF conversion
    adds (s, p^-1, o) for each (o, p, s), section 6).  ``reverse`` flips every
    edge direction (sc parent -> child)."""
    rng = _rng(seed) if rng is None else rng
    parent = forest_parents(n, min(roots, n), rng)
    child = np.nonzero(parent >= 0)[0]
    sc = np.stack([child, parent[child]], axis=1)
    k = int(round(ty_frac * n))
    if n >= 2 and k > 0:
        src = rng.choice(n, size=k, replace=False)
        off = rng.integers(1, n, size=k)
        dst = (src + off) % n            # uniform over the n-1 other nodes
        ty = np.stack([src, dst], axis=1)
    else:
        ty = np.zeros((0, 2), dtype=np.int64)
    if reverse:
        sc = sc[:, ::-1]
        ty = ty[:, ::-1]
    parts = [
        np.stack([sc[:, 0], np.full(len(sc), SC), sc[:, 1]], axis=1),
        np.stack([sc[:, 1], np.full(len(sc), SC_R), sc[:, 0]], axis=1),
        np.stack([ty[:, 0], np.full(len(ty), TY), ty[:, 1]], axis=1),
        np.stack([ty[:, 1], np.full(len(ty), TY_R), ty[:, 0]], axis=1),
    ]
    return n, _edges(np.concatenate(parts, axis=0))


def er_pairs(n: int, m: int, rng: np.random.Generator) -> np.ndarray:
    """``m`` distinct ordered pairs (u, v), u != v, uniform (G(n, m) model),
    in order of first draw."""
    m = min(m, n * (n - 1))
    if m <= 0:
        return np.zeros((0, 2), dtype=np.int64)
    chosen: List[np.ndarray] = []
    seen = set()
    have = 0
    while have < m:
        u = rng.integers(0, n, size=2 * (m - have) + 16)
        v = rng.integers(0, n, size=u.size)
        for a, b in zip(u.tolist(), v.tolist()):
            if a == b:
                continue
            key = a * n + b
            if key in seen:
                continue
            seen.add(key)
            chosen.append((a, b))
            have += 1
            if have == m:
                break
    return np.asarray(chosen, dtype=np.int64)


def erdos_renyi(n: int, m: int, seed: int, labels: int = 2,
                rng: np.random.Generator | None = None) -> Tuple[int, np.ndarray]:
    """G(n, m) directed graph with labels drawn uniformly from 0..labels-1."""
    rng = _rng(seed) if rng is None else rng
    p = er_pairs(n, m, rng)
    lab = rng.integers(0, labels, size=len(p))
    return n, _edges(np.stack([p[:, 0], lab, p[:, 1]], axis=1) if len(p) else [])


def erdos_renyi_hier_labels(n: int, m: int, seed: int,
                            rng: np.random.Generator | None = None) -> Tuple[int, np.ndarray]:
    """G(n, m) whose edges are labelled sc or ty uniformly, plus inverse edges,
    so the same-generation grammar can run on it."""
    rng = _rng(seed) if rng is None else rng
    p = er_pairs(n, m, rng)
    lab = np.where(rng.integers(0, 2, size=len(p)) == 0, SC, TY)
    inv = np.where(lab == SC, SC_R, TY_R)
    fwd = np.stack([p[:, 0], lab, p[:, 1]], axis=1)
    bwd = np.stack([p[:, 1], inv, p[:, 0]], axis=1)
    return n, _edges(np.concatenate([fwd, bwd], axis=0) if len(p) else [])


def induced_subgraph(n_sub: int, edges: np.ndarray) -> Tuple[int, np.ndarray]:
    """The subgraph induced on nodes 0..n_sub-1."""
    keep = (edges[:, 0] < n_sub) & (edges[:, 2] < n_sub)
    return n_sub, np.ascontiguousarray(edges[keep])


def chain(word: List[int]) -> Tuple[int, np.ndarray]:
    """A directed chain 0 -> 1 -> ... -> len(word) labelled by ``word``."""
    return len(word) + 1, _edges([(i, x, i + 1) for i, x in enumerate(word)])


def random_tiny(n: int, m: int, labels: int, seed: int, acyclic: bool = False) -> Tuple[int, np.ndarray]:
    """Small random multigraph (self-loops allowed unless ``acyclic``) for
    brute-force checks.  With ``acyclic`` every edge goes from a lower to a
    higher node id."""
    rng = _rng(seed)
    e = []
    for _ in range(m):
        u = int(rng.integers(0, n))
        v = int(rng.integers(0, n))
        if acyclic:
            if u == v:
                continue
            u, v = min(u, v), max(u, v)
        e.append((u, int(rng.integers(0, labels)), v))
    return n, _edges(e)
