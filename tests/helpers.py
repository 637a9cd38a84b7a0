"""Small helpers shared by the tests (no query arithmetic beyond set checks)."""
from __future__ import annotations

import numpy as np


def rel_from_dense(d: np.ndarray):
    return {a: set(zip(*(x.tolist() for x in np.nonzero(d[a])))) for a in range(d.shape[0])}


def closed_under_rules(dense: np.ndarray, grammar) -> bool:
    """True iff T_A contains T_B x T_C for every rule A -> B C (one extra loop of
    the closure would change nothing)."""
    for a, b, c in grammar.bin:
        prod = (dense[b].astype(np.float64) @ dense[c].astype(np.float64)) > 0.5
        if (prod & ~dense[a]).any():
            return False
    return True


def contains_init(dense: np.ndarray, n: int, edges, grammar) -> bool:
    e = np.asarray(edges).reshape(-1, 3)
    for a, x in grammar.term:
        sel = e[e[:, 1] == x]
        if len(sel) and not dense[a, sel[:, 0], sel[:, 2]].all():
            return False
    return True
