"""The five benchmark workloads as seeded, synthetic instances.

An instance is ``Instance(n, edges, grammar, tag)``.  The paper measured on RDF
ontologies that are not available here (section 6); the hierarchy graphs below,
with inverse labels added the way the paper converts RDF triples, stand in for
them.  Sizes follow the five workload descriptions:

1. two label cycles of 64 and 63 nodes sharing node 0, grammar a^n b^n;
2. a 4096-node random forest hierarchy with ty edges, same-generation grammar;
3. G(16384, 65536) with labels a/b, Dyck grammar (plus 1024/2048-node parity
   graphs from the same recipe);
4. 512 uneven instances, sizes log-uniform in [64, 2048];
5. a request stream, sizes log-uniform in [128, 8192], three grammars.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List

import numpy as np

from . import grammars as G
from . import graphs as H


@dataclass
class Instance:
    n: int
    edges: np.ndarray
    grammar: G.CNF
    tag: str = ""


def _child_rng(seed: int, i: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, i])))


def worked_example() -> Instance:
    n, e = H.worked_example()
    return Instance(n, e, G.same_generation(), "worked_example")


def config1() -> Instance:
    n, e = H.two_cycles(64, 63)
    return Instance(n, e, G.anbn(), "two_cycles_anbn_126")


def config2(reverse: bool = False, n: int = 4096, seed: int = 2) -> Instance:
    n, e = H.hierarchy(n, seed, roots=8, reverse=reverse)
    return Instance(n, e, G.same_generation(), f"hierarchy{n}{'_rev' if reverse else ''}_samegen")


def config3(n: int = 16384, avg_degree: int = 4, seed: int = 3) -> Instance:
    n, e = H.erdos_renyi(n, avg_degree * n, seed)
    return Instance(n, e, G.dyck(), f"er{n}_dyck")


def config3_induced(n_sub: int = 1024, n: int = 16384, seed: int = 3) -> Instance:
    big = config3(n, seed=seed)
    m, e = H.induced_subgraph(n_sub, big.edges)
    return Instance(m, e, G.dyck(), f"er{n}_induced{n_sub}_dyck")


def _mixed_instance(rng: np.random.Generator, n: int, er_degree: int, grammar_pool: List[str]) -> Instance:
    hier = bool(rng.integers(0, 2))
    gname = grammar_pool[int(rng.integers(0, len(grammar_pool)))]
    g = G.BY_NAME[gname]()
    if hier:
        nn, e = H.hierarchy(n, 0, roots=max(1, n // 512), rng=rng)
        g = G.for_hierarchy(g)
        kind = "hier"
    elif gname == "same_generation":
        nn, e = H.erdos_renyi_hier_labels(n, er_degree * n, 0, rng=rng)
        kind = "er"
    else:
        nn, e = H.erdos_renyi(n, er_degree * n, 0, labels=2, rng=rng)
        kind = "er"
    return Instance(nn, e, g, f"{kind}{n}_{gname}")


def log_uniform_size(rng: np.random.Generator, lo: int, hi: int) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def config4(count: int = 512, seed: int = 4, lo: int = 64, hi: int = 2048) -> List[Instance]:
    """Batch of uneven instances: size log-uniform in [lo, hi]; a fair coin picks
    hierarchy (roots = max(1, n/512)) or G(n, 3n); another coin picks the
    same-generation or the Dyck grammar."""
    out = []
    for i in range(count):
        rng = _child_rng(seed, i)
        n = log_uniform_size(rng, lo, hi)
        out.append(_mixed_instance(rng, n, 3, ["same_generation", "dyck"]))
    return out


def config5(count: int = 2100, seed: int = 5, lo: int = 128, hi: int = 8192):
    """Request stream: sizes log-uniform in [lo, hi], hierarchy or G(n, 4n),
    grammar uniform over a^n b^n, same-generation and Dyck.  Returns the
    instances and unit-rate exponential inter-arrival gaps (divide by the
    arrival rate to get seconds)."""
    insts = []
    for i in range(count):
        rng = _child_rng(seed, i)
        n = log_uniform_size(rng, lo, hi)
        insts.append(_mixed_instance(rng, n, 4, ["anbn", "same_generation", "dyck"]))
    gaps = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 10**6]))).exponential(1.0, size=count)
    return insts, gaps
