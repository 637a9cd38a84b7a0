"""The C-ABI library loads, exports every declared symbol, and rejects bad
arguments on the host before any device work (no GPU needed)."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cfpq.h")


def _lib():
    from paper_1707_01007_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.skip("libcfpq.so not built (run __graft_entry__.build())")
    return _abi.load()


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"CFPQ_API\s+[\w\s\*]+?\b(cfpq_\w+)\s*\(", text)))


def test_header_declares_entry_points():
    syms = declared_symbols()
    assert "cfpq_closure" in syms and "cfpq_product" in syms and len(syms) >= 10


def test_library_exports_every_declared_symbol():
    lib = _lib()
    for s in declared_symbols():
        assert hasattr(lib, s), s
    from paper_1707_01007_amd import _abi
    assert set(declared_symbols()) == set(_abi.EXPORTED)


def test_layout_functions():
    lib = _lib()
    for n, w in [(0, 4), (1, 4), (64, 4), (256, 4), (257, 8), (1000, 16), (4096, 64), (16384, 256)]:
        assert lib.cfpq_row_words(n) == w
        assert lib.cfpq_padded_rows(n) == 64 * w
        assert lib.cfpq_result_bytes(n, 3) == 3 * 64 * w * w * 8
    assert lib.cfpq_abi_version() == 4


def _structs(n=4, edges=((0, 0, 1), (1, 1, 2)), n_nt=4, n_t=2, term=((2, 0), (3, 1)),
             binr=((0, 2, 3),)):
    from paper_1707_01007_amd import _abi
    e = np.asarray(edges, dtype=np.int32).reshape(-1, 3)
    t_arr = (_abi.TermRule * max(1, len(term)))(*[_abi.TermRule(*r) for r in term])
    b_arr = (_abi.BinRule * max(1, len(binr)))(*[_abi.BinRule(*r) for r in binr])
    g = _abi.Grammar(n_nt, n_t, len(term), len(binr), ctypes.cast(t_arr, ctypes.POINTER(_abi.TermRule)),
                     ctypes.cast(b_arr, ctypes.POINTER(_abi.BinRule)))
    gr = _abi.Graph(n, 0, len(e), ctypes.c_void_p(e.ctypes.data))
    return gr, g, (e, t_arr, b_arr)


def test_workspace_bytes_valid_and_invalid():
    from paper_1707_01007_amd import _abi
    lib = _lib()
    gr, g, keep = _structs()
    opt = _abi.Options()
    lib.cfpq_default_options(ctypes.byref(opt))
    assert opt.path == _abi.PATH_AUTO and opt.schedule == _abi.SCHEDULE_INPLACE and opt.dirty_worklist == 1
    sz = ctypes.c_size_t(0)
    assert lib.cfpq_workspace_bytes(ctypes.byref(gr), ctypes.byref(g), ctypes.byref(opt), ctypes.byref(sz)) == 0
    assert sz.value > 0
    opt.schedule = _abi.SCHEDULE_JACOBI
    sz2 = ctypes.c_size_t(0)
    assert lib.cfpq_workspace_bytes(ctypes.byref(gr), ctypes.byref(g), ctypes.byref(opt), ctypes.byref(sz2)) == 0
    # a graph this small runs in one resident workgroup, both Jacobi buffers in LDS
    assert sz2.value == sz.value
    opt.path = _abi.PATH_BITS  # the ordinary loop keeps a second buffer in the workspace
    assert lib.cfpq_workspace_bytes(ctypes.byref(gr), ctypes.byref(g), ctypes.byref(opt), ctypes.byref(sz2)) == 0
    opt.schedule = _abi.SCHEDULE_INPLACE
    sz3 = ctypes.c_size_t(0)
    assert lib.cfpq_workspace_bytes(ctypes.byref(gr), ctypes.byref(g), ctypes.byref(opt), ctypes.byref(sz3)) == 0
    assert sz2.value >= sz3.value + 4 * lib.cfpq_result_bytes(4, 1)  # the second buffer
    opt.schedule = _abi.SCHEDULE_JACOBI
    g.n_nonterminals = 0
    assert lib.cfpq_workspace_bytes(ctypes.byref(gr), ctypes.byref(g), ctypes.byref(opt), ctypes.byref(sz)) == _abi.CFPQ_EINVAL
    assert b"n_nonterminals" in lib.cfpq_last_error()


@pytest.mark.parametrize("case,kw", [
    ("edge_src", dict(edges=((5, 0, 1),))),
    ("edge_dst", dict(edges=((0, 0, -1),))),
    ("edge_label", dict(edges=((0, 2, 1),))),
    ("term_lhs", dict(term=((4, 0),))),
    ("term_terminal", dict(term=((0, 7),))),
    ("bin_right", dict(binr=((0, 1, 9),))),
    ("negative_n", dict(n=-1, edges=())),
])
def test_closure_rejects_bad_ids_before_device_work(case, kw):
    """Every one of these returns CFPQ_EINVAL from host validation, before the
    first HIP call (this machine has no GPU)."""
    from paper_1707_01007_amd import _abi
    lib = _lib()
    gr, g, keep = _structs(**kw)
    st = _abi.Stats()
    rc = lib.cfpq_closure(ctypes.byref(gr), ctypes.byref(g), None, None, ctypes.c_void_p(1 << 20),
                          ctypes.c_size_t(1 << 30), ctypes.c_void_p(1 << 21), ctypes.byref(st))
    assert rc == _abi.CFPQ_EINVAL, case
    assert lib.cfpq_last_error()


def test_closure_rejects_small_workspace_and_null_result():
    from paper_1707_01007_amd import _abi
    lib = _lib()
    gr, g, keep = _structs()
    rc = lib.cfpq_closure(ctypes.byref(gr), ctypes.byref(g), None, None, ctypes.c_void_p(1 << 20),
                          ctypes.c_size_t(16), ctypes.c_void_p(1 << 21), None)
    assert rc == _abi.CFPQ_ENOMEM
    rc = lib.cfpq_closure(ctypes.byref(gr), ctypes.byref(g), None, None, ctypes.c_void_p(1 << 20),
                          ctypes.c_size_t(1 << 30), None, None)
    assert rc == _abi.CFPQ_EINVAL
    opt = _abi.Options()
    lib.cfpq_default_options(ctypes.byref(opt))
    opt.schedule = 7
    rc = lib.cfpq_closure(ctypes.byref(gr), ctypes.byref(g), ctypes.byref(opt), None, ctypes.c_void_p(1 << 20),
                          ctypes.c_size_t(1 << 30), ctypes.c_void_p(1 << 21), None)
    assert rc == _abi.CFPQ_EINVAL


@pytest.mark.parametrize("field,value", [("hybrid", 5), ("warm_start", 2), ("path", 6), ("path", -1)])
def test_closure_rejects_bad_options_before_device_work(field, value):
    from paper_1707_01007_amd import _abi
    lib = _lib()
    gr, g, keep = _structs()
    opt = _abi.Options()
    lib.cfpq_default_options(ctypes.byref(opt))
    assert opt.hybrid == _abi.HYBRID_AUTO and opt.warm_start == 0
    setattr(opt, field, value)
    rc = lib.cfpq_closure(ctypes.byref(gr), ctypes.byref(g), ctypes.byref(opt), None, ctypes.c_void_p(1 << 20),
                          ctypes.c_size_t(1 << 30), ctypes.c_void_p(1 << 21), None)
    assert rc == _abi.CFPQ_EINVAL, field
    assert lib.cfpq_last_error()


@pytest.mark.parametrize("path", [3, 4])
def test_sparse_paths_take_no_tile(path):
    from paper_1707_01007_amd import _abi
    lib = _lib()
    gr, g, keep = _structs()
    opt = _abi.Options()
    lib.cfpq_default_options(ctypes.byref(opt))
    opt.path, opt.tile = path, 8
    rc = lib.cfpq_closure(ctypes.byref(gr), ctypes.byref(g), ctypes.byref(opt), None, ctypes.c_void_p(1 << 20),
                          ctypes.c_size_t(1 << 30), ctypes.c_void_p(1 << 21), None)
    assert rc == _abi.CFPQ_EINVAL
    assert b"tile" in lib.cfpq_last_error()


@pytest.mark.parametrize("tile,ok", [(0, True), (2, True), (3, True), (5, True), (1, False), (4, False),
                                     (8, False)])
def test_fp4_tile_is_a_pipeline_depth(tile, ok):
    """The FP4 path's tile names its kernel variant: register pipeline depth
    2 or 3, or 5 for the persistent kernel (0 = the default); anything else
    is refused on the host by the closure and by a single product."""
    from paper_1707_01007_amd import _abi
    lib = _lib()
    gr, g, keep = _structs()
    opt = _abi.Options()
    lib.cfpq_default_options(ctypes.byref(opt))
    opt.path, opt.tile = _abi.PATH_FP4, tile
    sz = ctypes.c_size_t(0)
    assert lib.cfpq_workspace_bytes(ctypes.byref(gr), ctypes.byref(g), ctypes.byref(opt), ctypes.byref(sz)) == 0
    rc = lib.cfpq_closure(ctypes.byref(gr), ctypes.byref(g), ctypes.byref(opt), None, ctypes.c_void_p(1 << 20),
                          ctypes.c_size_t(1 << 30), ctypes.c_void_p(1 << 21), None)
    p = ctypes.c_void_p(1 << 20)
    rc2 = lib.cfpq_product(64, _abi.PATH_FP4, tile, p, p, p, p, None, 0, None)
    if ok:  # validation passes; what follows needs a device
        assert rc != _abi.CFPQ_EINVAL and rc2 != _abi.CFPQ_EINVAL
    else:
        assert rc == _abi.CFPQ_EINVAL and rc2 == _abi.CFPQ_EINVAL
        assert b"FP4 tile" in lib.cfpq_last_error()


def test_workspace_grows_with_sparse_temporaries():
    """COLS needs the transposed right operands plus two temporaries, the
    hybrid choice (padded sizes >= 4096) more; ROWS needs none."""
    from paper_1707_01007_amd import _abi
    lib = _lib()
    n = 5000
    gr, g, keep = _structs(n=n, edges=((0, 0, 1),))
    mat = lib.cfpq_result_bytes(n, 1)
    opt = _abi.Options()
    lib.cfpq_default_options(ctypes.byref(opt))
    sizes = {}
    for name, path, hybrid in [("mfma_dense", 2, 0), ("fp4_dense", 5, 0), ("bits_dense", 1, 0), ("rows", 3, 0),
                               ("cols", 4, 0), ("bits_hybrid", 1, 1)]:
        opt.path, opt.hybrid = path, hybrid
        sz = ctypes.c_size_t(0)
        assert lib.cfpq_workspace_bytes(ctypes.byref(gr), ctypes.byref(g), ctypes.byref(opt), ctypes.byref(sz)) == 0
        sizes[name] = sz.value
    rs = lib.cfpq_product_workspace_bytes(n, 3)  # the row product's scratch
    kwords = (n + 63) // 64
    assert rs >= lib.cfpq_padded_rows(n) * (kwords // 16 + 1) * 8 + 256 and rs % 256 == 0
    assert sizes["rows"] == sizes["bits_dense"] + rs
    assert sizes["fp4_dense"] == sizes["mfma_dense"] == sizes["bits_dense"] + mat  # one transposed right operand
    assert lib.cfpq_product_workspace_bytes(n, 5) == lib.cfpq_product_workspace_bytes(n, 2) == mat
    assert sizes["cols"] == sizes["mfma_dense"] + 2 * mat + rs  # one right operand (B) transposed in both
    # hybrid: the COLS scratch, plus a transposed right operand, loop-start
    # snapshots and gained bits of every nonterminal, and their counts
    assert sizes["bits_hybrid"] == sizes["cols"] + mat + 2 * g.n_nonterminals * mat + 256
    assert lib.cfpq_product_workspace_bytes(n, 4) == 3 * mat + rs


def test_struct_layouts_match_the_header(tmp_path):
    """ctypes mirrors of the C structs: size and every field offset as the C
    compiler lays them out from include/cfpq.h."""
    import shutil
    import subprocess
    from paper_1707_01007_amd import _abi
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    structs = {"cfpq_options": _abi.Options, "cfpq_stats": _abi.Stats, "cfpq_graph": _abi.Graph,
               "cfpq_grammar": _abi.Grammar, "cfpq_instance": _abi.Instance, "cfpq_tune_entry": _abi.TuneEntry,
               "cfpq_server_config": _abi.ServerConfig, "cfpq_request_info": _abi.RequestInfo,
               "cfpq_conjunct": _abi.Conjunct, "cfpq_conj_rule": _abi.ConjRule,
               "cfpq_batch_tune_entry": _abi.BatchTuneEntry}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "cfpq.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    c = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, cls in structs.items():
        assert c[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert c[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


def test_product_rejects_bad_arguments():
    from paper_1707_01007_amd import _abi
    lib = _lib()
    assert lib.cfpq_product(-1, 1, 0, None, None, None, None, None, 0, None) == _abi.CFPQ_EINVAL
    assert lib.cfpq_product(64, 1, 0, None, None, None, None, None, 0, None) == _abi.CFPQ_EINVAL
    p = ctypes.c_void_p(1 << 20)
    assert lib.cfpq_product(64, 9, 0, p, p, p, p, None, 0, None) == _abi.CFPQ_EINVAL
    assert lib.cfpq_product(64, 3, 8, p, p, p, p, p, 1 << 20, None) == _abi.CFPQ_EINVAL  # ROWS has no tiles
    assert lib.cfpq_product(64, 3, 0, p, p, p, p, None, 0, None) == _abi.CFPQ_ENOMEM    # ROWS needs scratch
    assert lib.cfpq_product(64, 4, 0, p, p, p, p, None, 0, None) == _abi.CFPQ_ENOMEM    # COLS needs workspace
    assert lib.cfpq_product(64, 1, 12, p, p, p, p, None, 0, None) == _abi.CFPQ_EINVAL   # no such strip width
    assert lib.cfpq_product(64, 2, 0, p, p, p, p, None, 0, None) == _abi.CFPQ_ENOMEM
    assert lib.cfpq_product(600000, 2, 0, p, p, p, p, p, 1 << 40, None) == _abi.CFPQ_EINVAL  # MFMA size bound
    assert lib.cfpq_product(64, 1, 0, p, p, p, None, None, 0, None) == _abi.CFPQ_EINVAL     # flag required
    assert lib.cfpq_product_workspace_bytes(256, 1) == 0
    assert lib.cfpq_product_workspace_bytes(256, 2) == lib.cfpq_result_bytes(256, 1)


def test_batch_validation_on_host():
    from paper_1707_01007_amd import _abi
    lib = _lib()
    gr, g, keep = _structs()
    inst = (_abi.Instance * 2)(_abi.Instance(gr, ctypes.pointer(g), ctypes.c_void_p(1 << 21)),
                               _abi.Instance(gr, ctypes.pointer(g), ctypes.c_void_p(1 << 22)))
    sz = ctypes.c_size_t(0)
    assert lib.cfpq_batch_workspace_bytes(2, inst, None, ctypes.byref(sz)) == 0 and sz.value > 0
    opt = _abi.Options()
    lib.cfpq_default_options(ctypes.byref(opt))
    opt.schedule = _abi.SCHEDULE_JACOBI
    assert lib.cfpq_batch_workspace_bytes(2, inst, ctypes.byref(opt), ctypes.byref(sz)) == _abi.CFPQ_EINVAL
    gr2, g2, keep2 = _structs(edges=((0, 5, 1),))
    inst[1] = _abi.Instance(gr2, ctypes.pointer(g2), ctypes.c_void_p(1 << 22))
    assert lib.cfpq_batch_workspace_bytes(2, inst, None, ctypes.byref(sz)) == _abi.CFPQ_EINVAL
    assert b"instance 1" in lib.cfpq_last_error()
    rc = lib.cfpq_batch_closure(2, inst, None, None, ctypes.c_void_p(1 << 20), ctypes.c_size_t(1 << 30), None)
    assert rc == _abi.CFPQ_EINVAL
    inst[1] = _abi.Instance(gr, ctypes.pointer(g), None)
    assert lib.cfpq_batch_closure(2, inst, None, None, ctypes.c_void_p(1 << 20), ctypes.c_size_t(1 << 30),
                                  None) == _abi.CFPQ_EINVAL


def test_batch_records_match_the_ctypes_structures():
    """The binding fills a batch's cfpq_instance records column by column;
    each must read back, field for field, as the ctypes structure would, and
    the library must plan the same workspace from them."""
    import torch
    import paper_1707_01007_amd as cfpq
    from paper_1707_01007_amd import _abi
    from workloads import grammars
    lib = _lib()
    gs = [grammars.dyck(), grammars.anbn(), grammars.same_generation()]
    items, outs = [], []
    for i in range(7):
        n = 40 + 97 * i
        edges = np.array([(j % n, j % 2, (3 * j + 1) % n) for j in range(2 * n + i)], np.int32)
        g = gs[i % 3]
        items.append((n, edges, g))
        outs.append(torch.empty(int(lib.cfpq_result_bytes(n, g.n_nonterminals)) // 8, dtype=torch.int64))
    ptr, keep, res_out = cfpq._instance_array(items, outs, None)
    ref = (_abi.Instance * len(items))()
    for i, (n, edges, g) in enumerate(items):
        gs_, _ = cfpq._grammar_struct(g)
        rec = ptr[i]
        assert (rec.graph.n_nodes, rec.graph.edges_on_device, rec.graph.n_edges) == (n, 0, len(edges))
        assert ctypes.addressof(rec.grammar.contents) == ctypes.addressof(gs_)
        assert rec.d_result == outs[i].data_ptr() and res_out[i] is outs[i]
        assert np.array_equal(np.ctypeslib.as_array(ctypes.cast(rec.graph.edges, ctypes.POINTER(ctypes.c_int32)),
                                                    (len(edges), 3)), edges)
        ref[i] = _abi.Instance(_abi.Graph(n, 0, len(edges), ctypes.c_void_p(rec.graph.edges)), ctypes.pointer(gs_),
                               ctypes.c_void_p(outs[i].data_ptr()))
    a, b = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert lib.cfpq_batch_workspace_bytes(len(items), ptr, None, ctypes.byref(a)) == 0
    assert lib.cfpq_batch_workspace_bytes(len(items), ref, None, ctypes.byref(b)) == 0
    assert a.value == b.value > 0
    # stats records read in bulk equal the per-record reading
    stats = (_abi.Stats * 5)()
    for i in range(5):
        stats[i].iterations, stats[i].products, stats[i].bitops, stats[i].converged = i, 3 * i, 0.5 * i, i % 2
        stats[i].sparse_ms = 1.25 * i
    assert cfpq._stats_dicts(stats, 5) == [stats[i].as_dict() for i in range(5)]
    assert cfpq._stats_dicts(stats, 2) == [stats[i].as_dict() for i in range(2)]


def test_path_variable_sizes_the_workspace(monkeypatch):
    """CFPQ_PATH replaces AUTO in cfpq_workspace_bytes as in the closure, so
    the workspace asked for fits the path the closure will take."""
    from paper_1707_01007_amd import _abi
    lib = _lib()
    gr, g, keep = _structs()

    def need(path, env):
        if env is None:
            monkeypatch.delenv("CFPQ_PATH", raising=False)
        else:
            monkeypatch.setenv("CFPQ_PATH", env)
        opt = _abi.Options()
        lib.cfpq_default_options(ctypes.byref(opt))
        opt.path = path
        sz = ctypes.c_size_t(0)
        assert lib.cfpq_workspace_bytes(ctypes.byref(gr), ctypes.byref(g), ctypes.byref(opt), ctypes.byref(sz)) == 0
        return sz.value

    for name, code in (("cols", _abi.PATH_COLS), ("rows", _abi.PATH_ROWS), ("bits", _abi.PATH_BITS)):
        assert need(_abi.PATH_AUTO, name) == need(code, None)
        assert need(code, "cols") == need(code, None)  # explicit paths are left alone
    assert need(_abi.PATH_AUTO, "nonsense") == need(_abi.PATH_AUTO, None)


def test_server_config_validation_on_host():
    from paper_1707_01007_amd import _abi
    lib = _lib()
    cfg = _abi.ServerConfig()
    lib.cfpq_server_default_config(ctypes.byref(cfg))
    assert cfg.max_slots == 256 and cfg.capture == 4 and cfg.hbm_budget == 8 << 30
    out = ctypes.c_void_p()
    for field, bad in (("max_slots", 0), ("capture", 0), ("max_pending", 0), ("hybrid_lanes", -1),
                       ("hybrid_lanes", 17)):
        c = _abi.ServerConfig()
        lib.cfpq_server_default_config(ctypes.byref(c))
        setattr(c, field, bad)
        assert lib.cfpq_server_create(ctypes.byref(c), None, ctypes.byref(out)) == _abi.CFPQ_EINVAL, field
    assert lib.cfpq_server_create(ctypes.byref(cfg), None, None) == _abi.CFPQ_EINVAL


def test_witness_host_function_on_oracle_lengths():
    """cfpq_witness is host code: fed the oracle's lengths it returns paths of
    exactly that many edges, present in the graph, whose words the
    nonterminal derives; bad cells and short buffers are errors."""
    from oracle import brute, single_path
    from workloads import grammars, graphs
    import paper_1707_01007_amd as cfpq
    n, e = graphs.erdos_renyi(30, 70, 13, labels=2)
    g = grammars.dyck()
    L, _ = single_path.lengths(n, e, g)
    npad = cfpq.padded_rows(n)
    full = np.zeros((g.n_nonterminals, npad, npad), dtype=np.uint32)
    full[:, :n, :n] = L
    edge_set = {tuple(int(v) for v in x) for x in e}
    for a, i, j in np.argwhere(L > 0)[:80]:
        path = cfpq.witness(n, e, g, full, int(a), int(i), int(j))
        assert len(path) == L[a, i, j] and path[0][0] == i and path[-1][2] == j
        assert all(tuple(p) in edge_set for p in path)
        assert all(p[2] == q[0] for p, q in zip(path, path[1:]))
        word = [p[1] for p in path]
        if len(word) <= 30:
            assert int(a) in brute.cyk_table(word, g)[0][len(word)]
    a, i, j = map(int, np.argwhere(L == 0)[0])
    with pytest.raises(cfpq.CfpqError):
        cfpq.witness(n, e, g, full, a, i, j)
    corrupt = full.copy()
    corrupt[corrupt > 1] += 1  # no split adds up any more
    a, i, j = map(int, np.argwhere(L > 1)[0])
    with pytest.raises(cfpq.CfpqError):
        cfpq.witness(n, e, g, corrupt, a, i, j)


def test_misaligned_buffers_are_rejected_before_device_work():
    from paper_1707_01007_amd import _abi
    lib = _lib()
    gr, g, keep = _structs()
    rc = lib.cfpq_closure(ctypes.byref(gr), ctypes.byref(g), None, None, ctypes.c_void_p(1 << 20),
                          ctypes.c_size_t(1 << 30), ctypes.c_void_p((1 << 21) + 8), None)
    assert rc == _abi.CFPQ_EINVAL and b"aligned" in lib.cfpq_last_error()
    p, q = ctypes.c_void_p(1 << 20), ctypes.c_void_p((1 << 20) + 8)
    assert lib.cfpq_product(64, 1, 0, p, q, p, p, None, 0, None) == _abi.CFPQ_EINVAL
    assert lib.cfpq_popcount(64, 1, q, p, None) == _abi.CFPQ_EINVAL


@pytest.mark.parametrize("case", ["head", "conjunct_id", "no_conjuncts", "path_rows"])
def test_conjunctive_rules_validated_before_device_work(case):
    from paper_1707_01007_amd import _abi
    lib = _lib()
    gr, g, keep = _structs()
    parts = (_abi.Conjunct * 2)(_abi.Conjunct(0, 0), _abi.Conjunct(0, 0))
    rule = _abi.ConjRule(0, 2, ctypes.cast(parts, ctypes.POINTER(_abi.Conjunct)))
    opt = _abi.Options()
    lib.cfpq_default_options(ctypes.byref(opt))
    if case == "head":
        rule.lhs = 5
    elif case == "conjunct_id":
        parts[1].right = 9
    elif case == "no_conjuncts":
        rule.n_conjuncts = 0
    else:
        opt.path = 3
    rules = (_abi.ConjRule * 1)(rule)
    sz = ctypes.c_size_t(0)
    assert lib.cfpq_conjunctive_workspace_bytes(ctypes.byref(gr), ctypes.byref(g), 1, rules, ctypes.byref(opt),
                                                ctypes.byref(sz)) == _abi.CFPQ_EINVAL
    assert lib.cfpq_conjunctive_closure(ctypes.byref(gr), ctypes.byref(g), 1, rules, ctypes.byref(opt), None,
                                        ctypes.c_void_p(1 << 20), ctypes.c_size_t(1 << 30), ctypes.c_void_p(1 << 21),
                                        None) == _abi.CFPQ_EINVAL


def test_static_closure_checks_on_host():
    """cfpq_closure_static refuses, before any device work, invalid inputs and
    closures whose workspace exceeds its static array."""
    from paper_1707_01007_amd import _abi
    lib = _lib()
    gr, g, keep = _structs()
    out = ctypes.c_void_p(1 << 20)
    bad = _abi.Grammar(0, 2, 0, 0, None, None)
    assert lib.cfpq_closure_static(ctypes.byref(gr), ctypes.byref(bad), None, None, out, None) == _abi.CFPQ_EINVAL
    big = _abi.Graph(20000, 0, 0, None)
    assert lib.cfpq_closure_static(ctypes.byref(big), ctypes.byref(g), None, None, out, None) == _abi.CFPQ_ENOMEM
    msg = lib.cfpq_last_error().decode()
    assert "static workspace" in msg and str(64 << 20) in msg
