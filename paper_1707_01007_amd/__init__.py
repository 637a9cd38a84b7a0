"""Context-free path querying (relational semantics) on AMD gfx950.

Python face of the C ABI in ``include/cfpq.h``.  PyTorch provides device
memory and the stream; every step of the query (matrix initialisation,
products, unions, change detection) runs in the HIP library ``libcfpq.so``.
There is no fallback: if the library is missing, importing the binding's
functions raises.

    import paper_1707_01007_amd as cfpq
    res = cfpq.closure(n, edges, grammar)          # edges: int32 [m, 3] (src, label, dst)
    bits = cfpq.result_bits(res)                   # numpy uint64 [|N|, n, ceil(n/64)]

A grammar is any object with ``n_nonterminals``, ``n_terminals``, ``term``
(pairs (A, x) for A -> x) and ``bin`` (triples (A, B, C) for A -> B C).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import _abi
from ._abi import (CfpqError, PATH_AUTO, PATH_BITS, PATH_MFMA, PATH_ROWS, PATH_COLS, PATH_FP4, SCHEDULE_INPLACE,  # noqa: F401
                   SCHEDULE_JACOBI)

_PATHS = {"auto": PATH_AUTO, "bits": PATH_BITS, "mfma": PATH_MFMA, "rows": PATH_ROWS, "cols": PATH_COLS,
          "fp4": PATH_FP4}
_SCHEDULES = {"inplace": SCHEDULE_INPLACE, "jacobi": SCHEDULE_JACOBI}


def _torch():
    import torch
    return torch


def lib():
    return _abi.load()


_LAYOUT_CACHE = {}


def _layout(n: int):
    """(padded rows, words per row) of the library's bit layout for n nodes,
    asked of the library once per n."""
    hit = _LAYOUT_CACHE.get(n)
    if hit is None:
        L = lib()
        hit = _LAYOUT_CACHE[n] = (int(L.cfpq_padded_rows(n)), int(L.cfpq_row_words(n)))
    return hit


def row_words(n: int) -> int:
    return _layout(int(n))[1]


def padded_rows(n: int) -> int:
    return _layout(int(n))[0]


_GRAMMAR_CACHE = {}


def _grammar_struct(grammar):
    """ctypes form of a grammar; memoised for hashable (frozen) grammars."""
    try:
        key = (grammar.n_nonterminals, grammar.n_terminals, tuple(grammar.term), tuple(grammar.bin))
    except TypeError:
        return _grammar_struct_new(grammar)
    hit = _GRAMMAR_CACHE.get(key)
    if hit is None:
        if len(_GRAMMAR_CACHE) > 4096:
            _GRAMMAR_CACHE.clear()
        hit = _GRAMMAR_CACHE[key] = _grammar_struct_new(grammar)
    return hit


def _grammar_struct_new(grammar):
    term = list(grammar.term)
    binr = list(grammar.bin)
    t_arr = (_abi.TermRule * max(1, len(term)))(*[_abi.TermRule(int(a), int(x)) for a, x in term])
    b_arr = (_abi.BinRule * max(1, len(binr)))(*[_abi.BinRule(int(a), int(b), int(c)) for a, b, c in binr])
    g = _abi.Grammar(int(grammar.n_nonterminals), int(grammar.n_terminals), len(term), len(binr),
                     ctypes.cast(t_arr, ctypes.POINTER(_abi.TermRule)),
                     ctypes.cast(b_arr, ctypes.POINTER(_abi.BinRule)))
    return g, (t_arr, b_arr)


def _options(path="auto", schedule="inplace", dirty=True, max_iters=0, profile=False, tile=0, capture=None,
             hybrid=None, warm_start=False):
    o = _abi.Options()
    lib().cfpq_default_options(ctypes.byref(o))
    if capture is not None:
        o.capture = int(capture)
    if hybrid is not None:
        o.hybrid = int(hybrid)
    o.warm_start = 1 if warm_start else 0
    o.profile = 1 if profile else 0
    o.tile = int(tile)
    o.path = _PATHS[path] if isinstance(path, str) else int(path)
    o.schedule = _SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule)
    o.dirty_worklist = 1 if dirty else 0
    o.max_iters = int(max_iters)
    return o


@dataclass
class Result:
    n: int
    n_nonterminals: int
    bits: "object"           # torch.int64 tensor [|N|, npad, W] on the device (uint64 bit rows)
    stats: dict
    status: int


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def closure(n: int, edges, grammar, *, path="auto", schedule="inplace", dirty=True, max_iters=0,
            device=None, stream=None, out=None, workspace=None, allow_partial=False,
            profile=False, tile=0, capture=None, hybrid=None, warm_start=False) -> Result:
    """Relational CFPQ closure (Algorithm 1) through ``cfpq_closure``.

    ``edges`` is an int32 array [m, 3] of (src, label, dst) on the host, or an
    int32 CUDA tensor of that shape (then checked on the device).  Returns a
    ``Result`` whose ``bits`` hold R_A for every nonterminal in the library's
    bit layout.  Raises ``CfpqError`` on any error (``allow_partial`` accepts
    CFPQ_ENOTCONV and returns the sound partial result).  ``path`` is "auto",
    "bits", "mfma" (dense kernel), "rows" or "cols" (every product skips the
    zeros of one operand); ``hybrid`` (None = library default, on) lets each
    product choose between the dense kernel and rows/cols.  ``warm_start``
    continues from the matrices already in ``out`` (each a subset of R)."""
    torch = _torch()
    L = lib()
    device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    g, keep = _grammar_struct(grammar)
    if isinstance(edges, torch.Tensor) and edges.is_cuda:
        e_dev = edges.to(torch.int32).contiguous().view(-1, 3)
        graph = _abi.Graph(int(n), 1, int(e_dev.shape[0]), ctypes.c_void_p(e_dev.data_ptr()))
        e_host = None
    else:
        e_host = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 3))
        graph = _abi.Graph(int(n), 0, int(e_host.shape[0]), ctypes.c_void_p(e_host.ctypes.data))
    if warm_start and out is None:
        raise ValueError("warm_start needs `out` holding the initial matrices")
    opt = _options(path, schedule, dirty, max_iters, profile, tile, capture, hybrid, warm_start)
    need = ctypes.c_size_t(0)
    _abi.check(L.cfpq_workspace_bytes(ctypes.byref(graph), ctypes.byref(g), ctypes.byref(opt), ctypes.byref(need)))
    res_words = int(L.cfpq_result_bytes(int(n), int(grammar.n_nonterminals))) // 8
    npad, W = padded_rows(n), row_words(n)
    if out is None:
        out = torch.empty(res_words, dtype=torch.int64, device=device)
    if workspace is None or workspace.numel() < need.value:
        workspace = torch.empty(max(need.value, 1), dtype=torch.uint8, device=device)
    st = _abi.Stats()
    status = L.cfpq_closure(ctypes.byref(graph), ctypes.byref(g), ctypes.byref(opt), _stream_ptr(stream),
                            ctypes.c_void_p(workspace.data_ptr()), ctypes.c_size_t(workspace.numel()),
                            ctypes.c_void_p(out.data_ptr()), ctypes.byref(st))
    del keep, e_host
    if status != _abi.CFPQ_OK and not (allow_partial and status == _abi.CFPQ_ENOTCONV):
        _abi.check(status)
    bits = out.view(int(grammar.n_nonterminals), npad, W)
    return Result(int(n), int(grammar.n_nonterminals), bits, st.as_dict(), status)


def _graph_struct(n, edges):
    torch = _torch()
    if isinstance(edges, torch.Tensor) and edges.is_cuda:
        e = edges.to(torch.int32).contiguous().view(-1, 3)
        return _abi.Graph(int(n), 1, int(e.shape[0]), ctypes.c_void_p(e.data_ptr())), e
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 3))
    return _abi.Graph(int(n), 0, int(e.shape[0]), ctypes.c_void_p(e.ctypes.data)), e


def single_path(n: int, edges, grammar, *, max_iters=0, device=None, stream=None, allow_partial=False):
    """Closure with single-path lengths (section 5) through ``cfpq_single_path``.
    Returns (Result, lengths): ``lengths`` is an int32 device tensor
    [|N|, npad, npad] holding L_A(i, j) (0 where (i, j) is not in R_A)."""
    torch = _torch()
    L = lib()
    device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    g, keep = _grammar_struct(grammar)
    graph, e = _graph_struct(n, edges)
    need = ctypes.c_size_t(0)
    _abi.check(L.cfpq_single_path_workspace_bytes(ctypes.byref(graph), ctypes.byref(g), ctypes.byref(need)))
    nnt = int(grammar.n_nonterminals)
    npad, W = padded_rows(n), row_words(n)
    out = torch.empty(int(L.cfpq_result_bytes(int(n), nnt)) // 8, dtype=torch.int64, device=device)
    lengths = torch.empty(int(L.cfpq_lengths_bytes(int(n), nnt)) // 4, dtype=torch.int32, device=device)
    ws = torch.empty(max(need.value, 1), dtype=torch.uint8, device=device)
    st = _abi.Stats()
    status = L.cfpq_single_path(ctypes.byref(graph), ctypes.byref(g), int(max_iters), _stream_ptr(stream),
                                ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                                ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(lengths.data_ptr()), ctypes.byref(st))
    del keep, e
    if status != _abi.CFPQ_OK and not (allow_partial and status == _abi.CFPQ_ENOTCONV):
        _abi.check(status)
    return (Result(int(n), nnt, out.view(nnt, npad, W), st.as_dict(), status), lengths.view(nnt, npad, npad))


def witness(n: int, edges, grammar, lengths, a: int, i: int, j: int):
    """A path i -> j of exactly L_a(i, j) edges whose label word ``a`` derives
    (``cfpq_witness``, host side).  ``lengths``: the tensor from
    ``single_path`` (copied to the host here) or a host uint32/int32 array of
    the same shape.  Returns a list of (src, label, dst)."""
    L = lib()
    torch = _torch()
    if isinstance(lengths, torch.Tensor):
        lengths = lengths.cpu().numpy()
    host = np.ascontiguousarray(np.asarray(lengths).view(np.uint32))
    e = np.ascontiguousarray(np.asarray(edges if not isinstance(edges, torch.Tensor) else edges.cpu().numpy(),
                                        dtype=np.int32).reshape(-1, 3))
    graph = _abi.Graph(int(n), 0, int(e.shape[0]), ctypes.c_void_p(e.ctypes.data))
    g, keep = _grammar_struct(grammar)
    npad = padded_rows(n)
    cap = int(host.reshape(-1, npad, npad)[a, i, j])
    buf = (_abi.Edge * max(cap, 1))()
    got = L.cfpq_witness(ctypes.byref(graph), ctypes.byref(g), ctypes.c_void_p(host.ctypes.data), int(a), int(i),
                         int(j), buf, cap)
    if got < 0:
        _abi.check(int(got))
    return [(buf[k].src, buf[k].label, buf[k].dst) for k in range(got)]


def conjunctive_closure(n: int, edges, grammar, *, path="auto", schedule="inplace", dirty=True, max_iters=0,
                        tile=0, device=None, stream=None, allow_partial=False, hybrid=None) -> Result:
    """Closure for a conjunctive grammar (``cfpq_conjunctive_closure``).
    ``grammar`` has ``nonterminals``, ``terminals``, ``term`` = [(A, x)] and
    ``conj`` = [(A, ((B1, C1), ..., (Bk, Ck)))]; one-conjunct rules are passed
    as ordinary binary rules.  ``hybrid`` (0/1, default the library's: 1) lets
    conjuncts with an edge-matrix left operand run as ROWS products."""
    torch = _torch()
    L = lib()
    device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    nnt = len(grammar.nonterminals)
    term = list(grammar.term)
    binr = [(a, parts[0][0], parts[0][1]) for a, parts in grammar.conj if len(parts) == 1]
    multi = [(a, parts) for a, parts in grammar.conj if len(parts) > 1]
    t_arr = (_abi.TermRule * max(1, len(term)))(*[_abi.TermRule(a, x) for a, x in term])
    b_arr = (_abi.BinRule * max(1, len(binr)))(*[_abi.BinRule(*r) for r in binr])
    g = _abi.Grammar(nnt, len(grammar.terminals), len(term), len(binr),
                     ctypes.cast(t_arr, ctypes.POINTER(_abi.TermRule)), ctypes.cast(b_arr, ctypes.POINTER(_abi.BinRule)))
    parts_keep = [(_abi.Conjunct * len(parts))(*[_abi.Conjunct(b, c) for b, c in parts]) for _, parts in multi]
    c_arr = (_abi.ConjRule * max(1, len(multi)))(
        *[_abi.ConjRule(a, len(parts), ctypes.cast(pk, ctypes.POINTER(_abi.Conjunct)))
          for (a, parts), pk in zip(multi, parts_keep)])
    graph, e = _graph_struct(n, edges)
    opt = _options(path, schedule, dirty, max_iters, False, tile, None, hybrid=hybrid)
    need = ctypes.c_size_t(0)
    _abi.check(L.cfpq_conjunctive_workspace_bytes(ctypes.byref(graph), ctypes.byref(g), len(multi), c_arr,
                                                  ctypes.byref(opt), ctypes.byref(need)))
    npad, W = padded_rows(n), row_words(n)
    out = torch.empty(int(L.cfpq_result_bytes(int(n), nnt)) // 8, dtype=torch.int64, device=device)
    ws = torch.empty(max(need.value, 1), dtype=torch.uint8, device=device)
    st = _abi.Stats()
    status = L.cfpq_conjunctive_closure(ctypes.byref(graph), ctypes.byref(g), len(multi), c_arr, ctypes.byref(opt),
                                        _stream_ptr(stream), ctypes.c_void_p(ws.data_ptr()),
                                        ctypes.c_size_t(ws.numel()), ctypes.c_void_p(out.data_ptr()), ctypes.byref(st))
    del e, parts_keep, t_arr, b_arr
    if status != _abi.CFPQ_OK and not (allow_partial and status == _abi.CFPQ_ENOTCONV):
        _abi.check(status)
    return Result(int(n), nnt, out.view(nnt, npad, W), st.as_dict(), status)


def closure_static(n: int, edges, grammar, *, path="auto", schedule="inplace", dirty=True, max_iters=0,
                   device=None, stream=None, out=None, allow_partial=False, tile=0, hybrid=None,
                   warm_start=False) -> Result:
    """``closure`` through ``cfpq_closure_static``: the library's own static
    device workspace instead of one allocated here (the call allocates no
    device memory; only ``out`` is allocated here when not given)."""
    torch = _torch()
    L = lib()
    device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    g, keep = _grammar_struct(grammar)
    if isinstance(edges, torch.Tensor) and edges.is_cuda:
        e_dev = edges.to(torch.int32).contiguous().view(-1, 3)
        graph = _abi.Graph(int(n), 1, int(e_dev.shape[0]), ctypes.c_void_p(e_dev.data_ptr()))
        e_host = None
    else:
        e_host = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 3))
        graph = _abi.Graph(int(n), 0, int(e_host.shape[0]), ctypes.c_void_p(e_host.ctypes.data))
    if warm_start and out is None:
        raise ValueError("warm_start needs `out` holding the initial matrices")
    opt = _options(path, schedule, dirty, max_iters, False, tile, None, hybrid, warm_start)
    res_words = int(L.cfpq_result_bytes(int(n), int(grammar.n_nonterminals))) // 8
    if out is None:
        out = torch.empty(res_words, dtype=torch.int64, device=device)
    st = _abi.Stats()
    status = L.cfpq_closure_static(ctypes.byref(graph), ctypes.byref(g), ctypes.byref(opt), _stream_ptr(stream),
                                   ctypes.c_void_p(out.data_ptr()), ctypes.byref(st))
    del keep, e_host
    if status != _abi.CFPQ_OK and not (allow_partial and status == _abi.CFPQ_ENOTCONV):
        _abi.check(status)
    bits = out.view(int(grammar.n_nonterminals), padded_rows(n), row_words(n))
    return Result(int(n), int(grammar.n_nonterminals), bits, st.as_dict(), status)


_INSTANCE_DTYPE = None


def _instance_dtype():
    """numpy record with the byte layout of ``cfpq_instance``."""
    global _INSTANCE_DTYPE
    if _INSTANCE_DTYPE is None:
        G, I = _abi.Graph, _abi.Instance
        go = I.graph.offset
        _INSTANCE_DTYPE = np.dtype({
            "names": ["n_nodes", "edges_on_device", "n_edges", "edges", "grammar", "d_result"],
            "formats": [np.int32, np.int32, np.int64, np.uintp, np.uintp, np.uintp],
            "offsets": [go + G.n_nodes.offset, go + G.edges_on_device.offset, go + G.n_edges.offset,
                        go + G.edges.offset, I.grammar.offset, I.d_result.offset],
            "itemsize": ctypes.sizeof(I)})
    return _INSTANCE_DTYPE


def _instance_array(instances, outs, device):
    """cfpq_instance records for (n, edges, grammar) triples (a pointer to
    them), the objects they point into, and one result buffer per instance
    (from ``outs`` or new).  Filled column by column: a batch holds hundreds
    of instances, and per-record ctypes structures cost more host time than
    the batch's smaller closures."""
    torch = _torch()
    L = lib()
    k = len(instances)
    keep, results_out = [], []
    gptr = {}  # id(grammar) -> address of its cfpq_grammar
    cols = ([], [], [], [], [], [])
    ns, on_dev, ms, eps, gps, rps = cols
    i32 = torch.int32
    for i, (n, edges, grammar) in enumerate(instances):
        gp = gptr.get(id(grammar))
        if gp is None:
            g, kg = _grammar_struct(grammar)
            keep.append((grammar, g, kg))
            gp = gptr[id(grammar)] = ctypes.addressof(g)
        if isinstance(edges, torch.Tensor) and edges.is_cuda:
            if edges.dtype == i32 and edges.is_contiguous() and edges.numel() % 3 == 0:
                e = edges
            else:
                e = edges.to(i32).contiguous().view(-1, 3)
            dev, m, ep = 1, e.numel() // 3, e.data_ptr()
        else:
            e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 3))
            dev, m, ep = 0, e.shape[0], e.ctypes.data
        keep.append(e)
        if outs is not None:
            out = outs[i]
        else:
            words = int(L.cfpq_result_bytes(int(n), int(grammar.n_nonterminals))) // 8
            out = torch.empty(words, dtype=torch.int64, device=device)
        results_out.append(out)
        ns.append(n)
        on_dev.append(dev)
        ms.append(m)
        eps.append(ep)
        gps.append(gp)
        rps.append(out.data_ptr())
    rec = np.zeros(max(1, k), dtype=_instance_dtype())
    if k:
        for name, col in zip(rec.dtype.names, cols):
            rec[name][:k] = col
    keep.append(rec)
    return rec.ctypes.data_as(ctypes.POINTER(_abi.Instance)), keep, results_out


_STATS_DTYPE = None


def _stats_dicts(stats, k):
    """One dict per ``cfpq_stats`` record of a ctypes array (read in bulk)."""
    global _STATS_DTYPE
    S = _abi.Stats
    names = [f for f, _ in S._fields_]
    if _STATS_DTYPE is None:
        _STATS_DTYPE = np.dtype({"names": names,
                                 "formats": [np.dtype(t) for _, t in S._fields_],
                                 "offsets": [getattr(S, f).offset for f in names],
                                 "itemsize": ctypes.sizeof(S)})
    rows = np.frombuffer(stats, dtype=_STATS_DTYPE, count=k).tolist()
    return [dict(zip(names, r)) for r in rows]


def batch_autotune(instances, *, max_per_bucket=0, reps=3, dirty=True, hybrid=None, device=None, stream=None,
                   outs=None):
    """Time the batched engine's routes per padded side on these instances
    (``cfpq_batch_autotune``) and record the fastest in the batch tuning
    table, which ``batch_closure`` and servers created afterwards use.
    Returns one dict per padded side tuned."""
    torch = _torch()
    L = lib()
    device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    k = len(instances)
    arr, keep, _ = _instance_array(instances, outs, device)
    opt = _options("auto", "inplace", dirty, 0, False, 0, None, hybrid=hybrid)
    need = ctypes.c_size_t(0)
    _abi.check(L.cfpq_batch_autotune_workspace_bytes(k, arr, ctypes.byref(opt), ctypes.byref(need)))
    ws = torch.empty(max(need.value, 1), dtype=torch.uint8, device=device)
    out = (_abi.BatchTuneEntry * 64)()
    got = ctypes.c_int32(0)
    _abi.check(L.cfpq_batch_autotune(k, arr, ctypes.byref(opt), _stream_ptr(stream), ctypes.c_void_p(ws.data_ptr()),
                                     ctypes.c_size_t(ws.numel()), int(max_per_bucket), int(reps), out, 64,
                                     ctypes.byref(got)))
    del keep
    return [out[i].as_dict() for i in range(min(got.value, 64))]


def batch_tune_get(npad: int):
    """The batch tuning table's entry for padded side npad, or None."""
    e = _abi.BatchTuneEntry()
    st = lib().cfpq_batch_tune_get(int(npad), ctypes.byref(e))
    if st == _abi.CFPQ_ENOTREADY:
        return None
    _abi.check(st)
    return e.as_dict()


def batch_tune_set(npad: int, route: str | None, tile: int = 256):
    """Set the route of padded side npad by hand ("resident", or "tiles" with
    tile 128 / 256); route None removes the entry."""
    e = _abi.BatchTuneEntry()
    e.npad = int(npad)
    e.route = {None: 0, "resident": _abi.ROUTE_RESIDENT, "tiles": _abi.ROUTE_TILES}[route]
    e.tile = int(tile) if route == "tiles" else 0
    _abi.check(lib().cfpq_batch_tune_set(ctypes.byref(e)))


def batch_closure(instances, *, dirty=True, max_iters=0, capture=None, device=None, stream=None,
                  outs=None, workspace=None, allow_partial=False, hybrid=None):
    """Closure of many independent instances in one call (``cfpq_batch_closure``).

    ``instances`` is a sequence of (n, edges, grammar); edges on the host or as
    int32 CUDA tensors.  Returns one ``Result`` per instance (each with its own
    device result buffer, or the buffers in ``outs``).  ``hybrid`` (0/1,
    default the library's: 1) lets rules of larger instances with an
    edge-matrix left operand run as row gathers."""
    torch = _torch()
    L = lib()
    device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    k = len(instances)
    arr, keep, results_out = _instance_array(instances, outs, device)
    opt = _options("auto", "inplace", dirty, max_iters, False, 0, capture, hybrid=hybrid)
    need = ctypes.c_size_t(0)
    _abi.check(L.cfpq_batch_workspace_bytes(k, arr, ctypes.byref(opt), ctypes.byref(need)))
    if workspace is None or workspace.numel() < need.value:
        workspace = torch.empty(max(need.value, 1), dtype=torch.uint8, device=device)
    stats = (_abi.Stats * max(1, k))()
    status = L.cfpq_batch_closure(k, arr, ctypes.byref(opt), _stream_ptr(stream), ctypes.c_void_p(workspace.data_ptr()),
                                  ctypes.c_size_t(workspace.numel()), stats)
    if status != _abi.CFPQ_OK and not (allow_partial and status == _abi.CFPQ_ENOTCONV):
        _abi.check(status)
    res = []
    for (n, edges, grammar), out, st in zip(instances, results_out, _stats_dicts(stats, k)):
        nnt = int(grammar.n_nonterminals)
        rows, words = _layout(int(n))
        res.append(Result(int(n), nnt, out.view(nnt, rows, words), st, status))
    del keep
    return res


class Server:
    """Continuous-batching server (``cfpq_server_*``).

    ``submit`` queues a query and returns a ticket; ``poll`` returns None while
    it runs and a dict (done, status, queue_ms, run_ms, latency_ms, stats,
    result) when it is done; ``wait`` blocks.  The result is a ``Result`` whose
    bits were written by the server into a buffer this object allocated (or the
    ``out`` given to ``submit``)."""

    def __init__(self, hbm_budget=8 << 30, max_slots=256, capture=4, max_pending=1 << 16, stream=None,
                 hybrid_lanes=None):
        torch = _torch()
        L = lib()
        cfg = _abi.ServerConfig()
        L.cfpq_server_default_config(ctypes.byref(cfg))
        cfg.hbm_budget, cfg.max_slots, cfg.capture, cfg.max_pending = int(hbm_budget), int(max_slots), int(capture), int(max_pending)
        if hybrid_lanes is not None:
            cfg.hybrid_lanes = int(hybrid_lanes)
        self._handle = ctypes.c_void_p()
        s = ctypes.c_void_p(stream.cuda_stream) if stream is not None else None
        _abi.check(L.cfpq_server_create(ctypes.byref(cfg), s, ctypes.byref(self._handle)))
        self._live = {}
        self._device = torch.device("cuda", torch.cuda.current_device())

    def submit(self, n, edges, grammar, out=None):
        torch = _torch()
        L = lib()
        g, kg = _grammar_struct(grammar)
        if isinstance(edges, torch.Tensor) and edges.is_cuda:
            e = edges.to(torch.int32).contiguous().view(-1, 3)
            graph = _abi.Graph(int(n), 1, int(e.shape[0]), ctypes.c_void_p(e.data_ptr()))
        else:
            e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 3))
            graph = _abi.Graph(int(n), 0, int(e.shape[0]), ctypes.c_void_p(e.ctypes.data))
        if out is None:
            words = int(L.cfpq_result_bytes(int(n), int(grammar.n_nonterminals))) // 8
            out = torch.empty(words, dtype=torch.int64, device=self._device)
        t = ctypes.c_int64(0)
        _abi.check(L.cfpq_server_submit(self._handle, ctypes.byref(graph), ctypes.byref(g),
                                        ctypes.c_void_p(out.data_ptr()), ctypes.byref(t)))
        self._live[t.value] = (int(n), grammar, out, e, (g, kg))
        return t.value

    def _finish(self, ticket, status, info):
        n, grammar, out, _, _ = self._live.pop(ticket)
        d = info.as_dict()
        bits = out.view(int(grammar.n_nonterminals), padded_rows(n), row_words(n))
        d["result"] = Result(n, int(grammar.n_nonterminals), bits, d["stats"], status)
        return d

    def poll(self, ticket):
        info = _abi.RequestInfo()
        st = lib().cfpq_server_poll(self._handle, ctypes.c_int64(ticket), ctypes.byref(info))
        if st == _abi.CFPQ_ENOTREADY:
            return None
        return self._finish(ticket, st, info)

    def wait(self, ticket):
        info = _abi.RequestInfo()
        st = lib().cfpq_server_wait(self._handle, ctypes.c_int64(ticket), ctypes.byref(info))
        return self._finish(ticket, st, info)

    def inject_fault(self):
        """Make the worker stop at its next turn as after a HIP error
        (``cfpq_server_inject_fault``; for tests of the failure handling)."""
        _abi.check(lib().cfpq_server_inject_fault(self._handle))

    def close(self):
        if self._handle:
            st = lib().cfpq_server_destroy(self._handle)
            self._handle = ctypes.c_void_p()
            _abi.check(st)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            if self._handle:
                lib().cfpq_server_destroy(self._handle)
        except Exception:
            pass


def result_bits(res: Result) -> np.ndarray:
    """Copy the result to the host as uint64 [|N|, n, ceil(n/64)] (padding
    stripped) -- the same layout the oracle returns."""
    w = max(1, (res.n + 63) // 64)
    host = res.bits[:, : res.n, :w].contiguous().cpu().numpy()
    return host.view(np.uint64)


def product(n: int, b, c, a, *, path="bits", tile=0, changed=None, workspace=None, stream=None):
    """``a |= b x c`` on device matrices in the bit layout (``cfpq_product``).
    Returns the device int32 change flag."""
    torch = _torch()
    L = lib()
    p = _PATHS[path] if isinstance(path, str) else int(path)
    if changed is None:
        changed = torch.zeros(1, dtype=torch.int32, device=a.device)
    need = int(L.cfpq_product_workspace_bytes(int(n), p))
    if need and (workspace is None or workspace.numel() < need):
        workspace = torch.empty(need, dtype=torch.uint8, device=a.device)
    ws_ptr = workspace.data_ptr() if workspace is not None else 0
    ws_len = workspace.numel() if workspace is not None else 0
    _abi.check(L.cfpq_product(int(n), p, int(tile), ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(c.data_ptr()),
                              ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(changed.data_ptr()),
                              ctypes.c_void_p(ws_ptr), ctypes.c_size_t(ws_len), _stream_ptr(stream)))
    return changed


def popcount(n: int, mats, count: int, stream=None):
    """Set bits per matrix for ``count`` matrices (``cfpq_popcount``); returns
    a host list of ints."""
    torch = _torch()
    counts = torch.zeros(count, dtype=torch.int64, device=mats.device)
    _abi.check(lib().cfpq_popcount(int(n), int(count), ctypes.c_void_p(mats.data_ptr()),
                                   ctypes.c_void_p(counts.data_ptr()), _stream_ptr(stream)))
    return [int(x) for x in counts.cpu().tolist()]


def new_matrices(n: int, count: int, device=None):
    """Zeroed device buffer for ``count`` matrices, shaped [count, npad, W]."""
    torch = _torch()
    return torch.zeros((count, padded_rows(n), row_words(n)), dtype=torch.int64,
                       device=device if device is not None else "cuda")


def upload_bits(n: int, host_bits: np.ndarray, device=None):
    """Host uint64 [count, n, ceil(n/64)] -> device [count, npad, W] (zero padded)."""
    torch = _torch()
    host_bits = np.asarray(host_bits, dtype=np.uint64)
    count = host_bits.shape[0]
    buf = np.zeros((count, padded_rows(n), row_words(n)), dtype=np.uint64)
    buf[:, :n, : host_bits.shape[2]] = host_bits
    return torch.from_numpy(buf.view(np.int64)).to(device if device is not None else "cuda")


def autotune(n: int, stream=None, device=None) -> dict:
    """Time every product kernel at size n and record the fastest for n's
    size bucket (``cfpq_autotune``); AUTO closures then use it."""
    torch = _torch()
    L = lib()
    device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    ws = torch.empty(int(L.cfpq_autotune_workspace_bytes(int(n))), dtype=torch.uint8, device=device)
    e = _abi.TuneEntry()
    _abi.check(L.cfpq_autotune(int(n), _stream_ptr(stream), ctypes.c_void_p(ws.data_ptr()),
                               ctypes.c_size_t(ws.numel()), ctypes.byref(e)))
    return e.as_dict()


def tune_get(n: int):
    """The recorded tuning entry for n's bucket, or None."""
    e = _abi.TuneEntry()
    st = lib().cfpq_tune_get(int(n), ctypes.byref(e))
    if st == _abi.CFPQ_ENOTREADY:
        return None
    _abi.check(st)
    return e.as_dict()


def tune_save(path: str):
    _abi.check(lib().cfpq_tune_save(str(path).encode()))


def tune_load(path: str):
    _abi.check(lib().cfpq_tune_load(str(path).encode()))


def tune_clear():
    lib().cfpq_tune_clear()
