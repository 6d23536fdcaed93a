"""Test helper: the undirected skeleton of the 199 directed 4-vertex classes.

Summing a directed k = 4 histogram by the skeleton of each class gives the
undirected census of the graph's undirected version G*: the six connected
4-vertex graphs in the order of oracle.UNDIRECTED4 (P4, tailed triangle,
claw, C4, K4 minus an edge, K4).  Classes are read through the oracle's
canonical codes (arc i->j at bit 3i + (j if j < i else j - 1)).
"""
from collections import Counter

import numpy as np

import oracle


def skeleton_of(k4_code: int) -> int:
    """Index into oracle.UNDIRECTED4 of the skeleton of a connected 4-vertex
    code, told apart by edge count and degree sequence."""
    und = set()
    for i in range(4):
        for j in range(4):
            if i != j and k4_code >> (i * 3 + (j if j < i else j - 1)) & 1:
                und.add((min(i, j), max(i, j)))
    deg = sorted(Counter(x for e in und for x in e).values())
    return {(3, (1, 1, 2, 2)): 0, (4, (1, 2, 2, 3)): 1, (3, (1, 1, 1, 3)): 2, (4, (2, 2, 2, 2)): 3,
            (5, (2, 2, 3, 3)): 4, (6, (3, 3, 3, 3)): 5}[(len(und), tuple(deg))]


def project(hist199) -> np.ndarray:
    _, canon, _, _ = oracle.class_table(4)
    out = np.zeros(6, np.uint64)
    for c, code in enumerate(canon):
        out[skeleton_of(int(code))] += np.uint64(hist199[c])
    return out
