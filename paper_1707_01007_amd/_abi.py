"""ctypes declarations of the C ABI in ``include/cfpq.h`` (argument
marshalling only; every step of the query runs in the HIP library)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcfpq.so")

CFPQ_OK, CFPQ_EINVAL, CFPQ_ENOMEM, CFPQ_EDEVICE, CFPQ_ENOTCONV, CFPQ_EBUSY, CFPQ_ENOTREADY = 0, -1, -2, -3, -4, -5, -6
CFPQ_ERANGE = -7
PATH_AUTO, PATH_BITS, PATH_MFMA, PATH_ROWS, PATH_COLS, PATH_FP4 = 0, 1, 2, 3, 4, 5
HYBRID_OFF, HYBRID_AUTO = 0, 1
ROUTE_RESIDENT, ROUTE_TILES = 1, 2
ABI_VERSION = 4
SCHEDULE_INPLACE, SCHEDULE_JACOBI = 0, 1
STATUS_NAMES = {0: "CFPQ_OK", -1: "CFPQ_EINVAL", -2: "CFPQ_ENOMEM", -3: "CFPQ_EDEVICE",
                -4: "CFPQ_ENOTCONV", -5: "CFPQ_EBUSY", -6: "CFPQ_ENOTREADY", -7: "CFPQ_ERANGE"}

EXPORTED = (
    "cfpq_abi_version", "cfpq_last_error", "cfpq_default_options", "cfpq_row_words",
    "cfpq_padded_rows", "cfpq_result_bytes", "cfpq_workspace_bytes", "cfpq_closure", "cfpq_closure_static",
    "cfpq_product_workspace_bytes", "cfpq_product", "cfpq_popcount",
    "cfpq_batch_workspace_bytes", "cfpq_batch_closure",
    "cfpq_server_default_config", "cfpq_server_create", "cfpq_server_submit", "cfpq_server_poll",
    "cfpq_server_wait", "cfpq_server_destroy", "cfpq_server_inject_fault",
    "cfpq_autotune_workspace_bytes", "cfpq_autotune", "cfpq_tune_get", "cfpq_tune_save", "cfpq_tune_load",
    "cfpq_tune_clear", "cfpq_batch_autotune_workspace_bytes", "cfpq_batch_autotune", "cfpq_batch_tune_get",
    "cfpq_batch_tune_set",
    "cfpq_lengths_bytes", "cfpq_single_path_workspace_bytes", "cfpq_single_path", "cfpq_witness",
    "cfpq_conjunctive_workspace_bytes", "cfpq_conjunctive_closure",
)


class Edge(ctypes.Structure):
    _fields_ = [("src", ctypes.c_int32), ("label", ctypes.c_int32), ("dst", ctypes.c_int32)]


class TermRule(ctypes.Structure):
    _fields_ = [("lhs", ctypes.c_int32), ("terminal", ctypes.c_int32)]


class BinRule(ctypes.Structure):
    _fields_ = [("lhs", ctypes.c_int32), ("left", ctypes.c_int32), ("right", ctypes.c_int32)]


class Conjunct(ctypes.Structure):
    _fields_ = [("left", ctypes.c_int32), ("right", ctypes.c_int32)]


class ConjRule(ctypes.Structure):
    _fields_ = [("lhs", ctypes.c_int32), ("n_conjuncts", ctypes.c_int32), ("conjuncts", ctypes.POINTER(Conjunct))]


class Graph(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("edges_on_device", ctypes.c_int32),
                ("n_edges", ctypes.c_int64), ("edges", ctypes.c_void_p)]


class Grammar(ctypes.Structure):
    _fields_ = [("n_nonterminals", ctypes.c_int32), ("n_terminals", ctypes.c_int32),
                ("n_term_rules", ctypes.c_int32), ("n_bin_rules", ctypes.c_int32),
                ("term_rules", ctypes.POINTER(TermRule)), ("bin_rules", ctypes.POINTER(BinRule))]


class Instance(ctypes.Structure):
    _fields_ = [("graph", Graph), ("grammar", ctypes.POINTER(Grammar)), ("d_result", ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int32), ("schedule", ctypes.c_int32), ("dirty_worklist", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("tile", ctypes.c_int32), ("capture", ctypes.c_int32),
                ("hybrid", ctypes.c_int32), ("warm_start", ctypes.c_int32), ("max_iters", ctypes.c_int64)]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("products", ctypes.c_int64), ("bitops", ctypes.c_double),
                ("device_ms", ctypes.c_double), ("product_ms", ctypes.c_double), ("path_used", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("sparse_products", ctypes.c_int64), ("delta_products", ctypes.c_int64),
                ("minplus_terms", ctypes.c_double), ("sparse_bytes", ctypes.c_double), ("sparse_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TuneEntry(ctypes.Structure):
    _fields_ = [("npad", ctypes.c_int32), ("path", ctypes.c_int32), ("tile", ctypes.c_int32), ("ms", ctypes.c_float),
                ("n_candidates", ctypes.c_int32), ("candidate_path", ctypes.c_int32 * 8),
                ("candidate_tile", ctypes.c_int32 * 8), ("candidates_ms", ctypes.c_float * 8)]

    def as_dict(self):
        names = {PATH_BITS: "bits", PATH_MFMA: "mfma", PATH_FP4: "fp4"}
        cands = {f"{names.get(self.candidate_path[k], '?')}"
                 f"{'_' + str(self.candidate_tile[k]) if self.candidate_tile[k] else ''}": round(self.candidates_ms[k], 4)
                 for k in range(self.n_candidates)}
        return {"npad": self.npad, "path": names.get(self.path, "?"), "tile": self.tile,
                "ms": round(self.ms, 4), "candidates_ms": cands}


class BatchTuneEntry(ctypes.Structure):
    _fields_ = [("npad", ctypes.c_int32), ("route", ctypes.c_int32), ("tile", ctypes.c_int32), ("ms", ctypes.c_float),
                ("instances", ctypes.c_int32), ("n_candidates", ctypes.c_int32),
                ("candidate_route", ctypes.c_int32 * 4), ("candidate_tile", ctypes.c_int32 * 4),
                ("candidates_ms", ctypes.c_float * 4)]

    @staticmethod
    def _name(route, tile):
        return "resident" if route == ROUTE_RESIDENT else f"tiles{tile}"

    def as_dict(self):
        cands = {self._name(self.candidate_route[k], self.candidate_tile[k]): round(self.candidates_ms[k], 4)
                 for k in range(self.n_candidates)}
        return {"npad": self.npad, "route": "resident" if self.route == ROUTE_RESIDENT else "tiles",
                "tile": self.tile, "ms": round(self.ms, 4), "instances": self.instances, "candidates_ms": cands}


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_slots", ctypes.c_int32), ("capture", ctypes.c_int32),
                ("max_pending", ctypes.c_int32), ("hybrid_lanes", ctypes.c_int32)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("done", ctypes.c_int32), ("status", ctypes.c_int32), ("queue_ms", ctypes.c_double),
                ("run_ms", ctypes.c_double), ("latency_ms", ctypes.c_double), ("stats", Stats)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "stats"}
        d["stats"] = self.stats.as_dict()
        return d


_lib = None


class CfpqError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def load(path: str = LIB_PATH):
    """Load the HIP library.  Raises if it has not been built: there is no
    fallback implementation."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing; build it with `python -m paper_1707_01007_amd.build`")
    lib = ctypes.CDLL(path)
    i32, i64, p, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t
    lib.cfpq_abi_version.restype = i32
    lib.cfpq_last_error.restype = ctypes.c_char_p
    lib.cfpq_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.cfpq_row_words.argtypes = [i32]
    lib.cfpq_row_words.restype = i64
    lib.cfpq_padded_rows.argtypes = [i32]
    lib.cfpq_padded_rows.restype = i64
    lib.cfpq_result_bytes.argtypes = [i32, i32]
    lib.cfpq_result_bytes.restype = sz
    lib.cfpq_workspace_bytes.argtypes = [ctypes.POINTER(Graph), ctypes.POINTER(Grammar),
                                         ctypes.POINTER(Options), ctypes.POINTER(sz)]
    lib.cfpq_workspace_bytes.restype = ctypes.c_int
    lib.cfpq_closure.argtypes = [ctypes.POINTER(Graph), ctypes.POINTER(Grammar), ctypes.POINTER(Options),
                                 p, p, sz, p, ctypes.POINTER(Stats)]
    lib.cfpq_closure.restype = ctypes.c_int
    lib.cfpq_closure_static.argtypes = [ctypes.POINTER(Graph), ctypes.POINTER(Grammar), ctypes.POINTER(Options), p,
                                        p, ctypes.POINTER(Stats)]
    lib.cfpq_closure_static.restype = ctypes.c_int
    lib.cfpq_product_workspace_bytes.argtypes = [i32, i32]
    lib.cfpq_product_workspace_bytes.restype = sz
    lib.cfpq_product.argtypes = [i32, i32, i32, p, p, p, p, p, sz, p]
    lib.cfpq_product.restype = ctypes.c_int
    lib.cfpq_popcount.argtypes = [i32, i32, p, p, p]
    lib.cfpq_popcount.restype = ctypes.c_int
    lib.cfpq_batch_workspace_bytes.argtypes = [i32, ctypes.POINTER(Instance), ctypes.POINTER(Options),
                                               ctypes.POINTER(sz)]
    lib.cfpq_batch_workspace_bytes.restype = ctypes.c_int
    lib.cfpq_batch_closure.argtypes = [i32, ctypes.POINTER(Instance), ctypes.POINTER(Options), p, p, sz,
                                       ctypes.POINTER(Stats)]
    lib.cfpq_batch_closure.restype = ctypes.c_int
    lib.cfpq_server_default_config.argtypes = [ctypes.POINTER(ServerConfig)]
    lib.cfpq_server_create.argtypes = [ctypes.POINTER(ServerConfig), p, ctypes.POINTER(p)]
    lib.cfpq_server_create.restype = ctypes.c_int
    lib.cfpq_server_submit.argtypes = [p, ctypes.POINTER(Graph), ctypes.POINTER(Grammar), p,
                                       ctypes.POINTER(ctypes.c_int64)]
    lib.cfpq_server_submit.restype = ctypes.c_int
    lib.cfpq_server_poll.argtypes = [p, ctypes.c_int64, ctypes.POINTER(RequestInfo)]
    lib.cfpq_server_poll.restype = ctypes.c_int
    lib.cfpq_server_wait.argtypes = [p, ctypes.c_int64, ctypes.POINTER(RequestInfo)]
    lib.cfpq_server_wait.restype = ctypes.c_int
    lib.cfpq_server_destroy.argtypes = [p]
    lib.cfpq_server_destroy.restype = ctypes.c_int
    lib.cfpq_server_inject_fault.argtypes = [p]
    lib.cfpq_server_inject_fault.restype = ctypes.c_int
    lib.cfpq_autotune_workspace_bytes.argtypes = [i32]
    lib.cfpq_autotune_workspace_bytes.restype = sz
    lib.cfpq_autotune.argtypes = [i32, p, p, sz, ctypes.POINTER(TuneEntry)]
    lib.cfpq_autotune.restype = ctypes.c_int
    lib.cfpq_tune_get.argtypes = [i32, ctypes.POINTER(TuneEntry)]
    lib.cfpq_tune_get.restype = ctypes.c_int
    lib.cfpq_tune_save.argtypes = [ctypes.c_char_p]
    lib.cfpq_tune_save.restype = ctypes.c_int
    lib.cfpq_tune_load.argtypes = [ctypes.c_char_p]
    lib.cfpq_tune_load.restype = ctypes.c_int
    lib.cfpq_tune_clear.argtypes = []
    lib.cfpq_tune_clear.restype = None
    lib.cfpq_batch_autotune_workspace_bytes.argtypes = [i32, ctypes.POINTER(Instance), ctypes.POINTER(Options),
                                                        ctypes.POINTER(sz)]
    lib.cfpq_batch_autotune_workspace_bytes.restype = ctypes.c_int
    lib.cfpq_batch_autotune.argtypes = [i32, ctypes.POINTER(Instance), ctypes.POINTER(Options), p, p, sz, i32, i32,
                                        ctypes.POINTER(BatchTuneEntry), i32, ctypes.POINTER(i32)]
    lib.cfpq_batch_autotune.restype = ctypes.c_int
    lib.cfpq_batch_tune_get.argtypes = [i32, ctypes.POINTER(BatchTuneEntry)]
    lib.cfpq_batch_tune_get.restype = ctypes.c_int
    lib.cfpq_batch_tune_set.argtypes = [ctypes.POINTER(BatchTuneEntry)]
    lib.cfpq_batch_tune_set.restype = ctypes.c_int
    lib.cfpq_lengths_bytes.argtypes = [i32, i32]
    lib.cfpq_lengths_bytes.restype = sz
    lib.cfpq_single_path_workspace_bytes.argtypes = [ctypes.POINTER(Graph), ctypes.POINTER(Grammar),
                                                     ctypes.POINTER(sz)]
    lib.cfpq_single_path_workspace_bytes.restype = ctypes.c_int
    lib.cfpq_single_path.argtypes = [ctypes.POINTER(Graph), ctypes.POINTER(Grammar), i64, p, p, sz, p, p,
                                     ctypes.POINTER(Stats)]
    lib.cfpq_single_path.restype = ctypes.c_int
    lib.cfpq_witness.argtypes = [ctypes.POINTER(Graph), ctypes.POINTER(Grammar), p, i32, i32, i32,
                                 ctypes.POINTER(Edge), i64]
    lib.cfpq_witness.restype = i64
    lib.cfpq_conjunctive_workspace_bytes.argtypes = [ctypes.POINTER(Graph), ctypes.POINTER(Grammar), i32,
                                                     ctypes.POINTER(ConjRule), ctypes.POINTER(Options),
                                                     ctypes.POINTER(sz)]
    lib.cfpq_conjunctive_workspace_bytes.restype = ctypes.c_int
    lib.cfpq_conjunctive_closure.argtypes = [ctypes.POINTER(Graph), ctypes.POINTER(Grammar), i32,
                                             ctypes.POINTER(ConjRule), ctypes.POINTER(Options), p, p, sz, p,
                                             ctypes.POINTER(Stats)]
    lib.cfpq_conjunctive_closure.restype = ctypes.c_int
    if lib.cfpq_abi_version() != ABI_VERSION:
        raise ImportError("libcfpq ABI version mismatch")
    _lib = lib
    return lib


def check(status: int):
    if status != CFPQ_OK:
        msg = _lib.cfpq_last_error().decode() if _lib is not None else ""
        raise CfpqError(status, msg)
