"""Seeded synthetic inputs (graphs, CNF grammars, workload configurations).

This package is shared by the oracle and the GPU path and therefore holds no
part of the query computation itself: only edge lists, grammar rule lists and
random draws.
"""
from . import grammars, graphs, configs  # noqa: F401
from .grammars import CNF  # noqa: F401
from .configs import Instance  # noqa: F401
