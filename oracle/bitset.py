"""ctypes front end of the bit-packed Algorithm 1 (``cfpq_bitset.c``).

Test infrastructure: only tests, the smoke check and the benchmark's CPU
baseline call this.  Algorithm 1 of section 4.2 with the simultaneous
(Jacobi) update on bit-packed rows, the rows of each product spread over
OpenMP threads: a second CPU implementation of the relational closure (the
tests hold it to the worklist oracle and to the loop counts of Lemma 3) and
the host's all-core rate for the closure and for one Boolean product.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cfpq_bitset.c")
_LIB = os.path.join(_HERE, "libcfpq_bitset_oracle.so")
_lib = None


def build(force: bool = False, src: str = _SRC, lib: str = _LIB) -> str:
    """Compile with gcc -O3 -fopenmp (integer code only; no -march, so the
    library runs on any x86-64 host, its row OR cloned for AVX2 and AVX-512)."""
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
        tmp = lib + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src])
        os.replace(tmp, lib)
    return lib


def load_library(path: str):
    lib = ctypes.CDLL(path)
    i32, i64, p = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    lib.cfpq_bitset_closure.argtypes = [i32, i64, p, i32, i32, i32, p, i32, p, i64, i32, p, p]
    lib.cfpq_bitset_closure.restype = ctypes.c_int
    lib.cfpq_bitset_product.argtypes = [i32, i64, i64, p, p, p, i32]
    lib.cfpq_bitset_product.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        _lib = load_library(build())
    return _lib


def row_words(n: int) -> int:
    return max(1, (n + 63) // 64)


def closure(n: int, edges: np.ndarray, grammar, max_loops: int | None = None, threads: int = 0, lib=None):
    """Return (bits, loops, status): bits uint64 [|N|, n, ceil(n/64)] in the
    worklist oracle's layout; status 0 at the fixpoint, 3 when ``max_loops``
    stopped it first (bits then hold T after that many loops)."""
    lib = _load() if lib is None else lib
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 3))
    term = np.ascontiguousarray(np.asarray(grammar.term, dtype=np.int32).reshape(-1, 2))
    binr = np.ascontiguousarray(np.asarray(grammar.bin, dtype=np.int32).reshape(-1, 3))
    out = np.zeros((grammar.n_nonterminals, n, (n + 63) // 64), dtype=np.uint64)
    loops = ctypes.c_int64(0)
    rc = lib.cfpq_bitset_closure(n, len(e), e.ctypes.data, grammar.n_nonterminals, grammar.n_terminals,
                                 len(term), term.ctypes.data, len(binr), binr.ctypes.data, int(max_loops or 0),
                                 int(threads), out.ctypes.data, ctypes.byref(loops))
    if rc == -1:
        raise ValueError("bitset closure: invalid graph or grammar")
    if rc == -2:
        raise MemoryError("bitset closure: out of memory")
    if n == 0:
        out = np.zeros((grammar.n_nonterminals, 0, 1), dtype=np.uint64)
    return out, int(loops.value), rc


def product(n: int, b: np.ndarray, c: np.ndarray, a: np.ndarray, rows: tuple[int, int] | None = None,
            threads: int = 0, lib=None) -> None:
    """a |= b c in place on rows [rows[0], rows[1]) of a and b (all rows by
    default); b, c, a are uint64 [n, ceil(n/64)] bit rows, C-contiguous."""
    lib = _load() if lib is None else lib
    w = (n + 63) // 64
    for m in (b, c, a):
        assert m.dtype == np.uint64 and m.shape == (n, w) and m.flags["C_CONTIGUOUS"]
    r0, r1 = rows if rows is not None else (0, n)
    rc = lib.cfpq_bitset_product(n, r0, r1, b.ctypes.data, c.ctypes.data, a.ctypes.data, int(threads))
    if rc != 0:
        raise ValueError("bitset product: invalid rows")
