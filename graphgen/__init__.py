"""Seeded synthetic directed-graph generators.

This module produces inputs only: it holds none of the census arithmetic, so the
CPU oracle and the GPU path can both draw their inputs from it without sharing
any of the method's code.  Every generator is deterministic in its seed
(numpy ``default_rng``) and returns a :class:`Digraph` in int32 out-CSR form
with sorted neighbour lists, no self-loops and no repeated arcs.
"""
from .core import (
    Digraph,
    from_arcs,
    gnm_reciprocal,
    chung_lu,
    arc_switch,
    arc_switch_many,
    directed_cycle,
    directed_path,
    complete_digraph,
    transitive_tournament,
    star,
    disjoint_union,
    relabel,
    reverse,
    random_small,
    planted_hubs,
    pad_relabel,
)

__all__ = [
    "Digraph", "from_arcs", "gnm_reciprocal", "chung_lu", "arc_switch", "arc_switch_many",
    "directed_cycle", "directed_path", "complete_digraph", "transitive_tournament",
    "star", "disjoint_union", "relabel", "reverse", "random_small", "planted_hubs", "pad_relabel",
]
