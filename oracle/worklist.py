"""ctypes front end of the C worklist oracle (``cfpq_worklist.c``).

Test infrastructure: only tests, the smoke check and the benchmark's CPU
baseline call this.  The library is built with the host C compiler.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cfpq_worklist.c")
_LIB = os.path.join(_HERE, "libcfpq_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc -O2 (no -ffast-math; integer code only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def load_library(path: str):
    lib = ctypes.CDLL(path)
    i32, i64, p = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    lib.cfpq_oracle.argtypes = [i32, i64, p, i32, i32, i32, p, i32, p, p, i64]
    lib.cfpq_oracle.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        _lib = load_library(build())
    return _lib


def row_words(n: int) -> int:
    return max(1, (n + 63) // 64)


def closure(n: int, edges: np.ndarray, grammar, lib=None) -> np.ndarray:
    """Return R as uint64 bits of shape [|N|, n, ceil(n/64)]: bit j%64 of word
    j//64 of row i of matrix A is set iff (i, j) is in R_A.  ``lib`` selects
    another build of the same source (the mutation tests use it)."""
    lib = _load() if lib is None else lib
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 3))
    term = np.ascontiguousarray(np.asarray(grammar.term, dtype=np.int32).reshape(-1, 2))
    binr = np.ascontiguousarray(np.asarray(grammar.bin, dtype=np.int32).reshape(-1, 3))
    w = row_words(n)
    out = np.zeros((grammar.n_nonterminals, n, w), dtype=np.uint64)
    rc = lib.cfpq_oracle(n, len(e), e.ctypes.data, grammar.n_nonterminals, grammar.n_terminals,
                         len(term), term.ctypes.data, len(binr), binr.ctypes.data,
                         out.ctypes.data, w)
    if rc == -1:
        raise ValueError("oracle: invalid graph or grammar")
    if rc != 0:
        raise MemoryError("oracle: out of memory")
    return out


def unpack(bits: np.ndarray, n: int) -> np.ndarray:
    """uint64 bit rows [.., n, W] -> bool [.., n, n]."""
    b = np.ascontiguousarray(bits).view(np.uint8)
    u = np.unpackbits(b, axis=-1, bitorder="little")
    return u[..., :n].astype(bool)


def pack(dense: np.ndarray) -> np.ndarray:
    """bool [.., n, n] -> uint64 bit rows [.., n, ceil(n/64)]."""
    n = dense.shape[-1]
    w = row_words(n)
    pad = np.zeros(dense.shape[:-1] + (w * 64,), dtype=np.uint8)
    pad[..., :n] = dense
    return np.packbits(pad, axis=-1, bitorder="little").view(np.uint64)


def relations(bits: np.ndarray, n: int):
    """{A: set of (i, j)} from packed bits."""
    d = unpack(bits, n)
    return {a: set(zip(*np.nonzero(d[a]))) for a in range(d.shape[0])}
