"""Tiny all-subsets census checker in pure Python -- test infrastructure only.

Independent of ``oracle.c``: it walks every k-subset (itertools), tests weak
connectivity by breadth-first search on the undirected version, and
canonicalises the induced digraph by the minimum code over all k! relabellings.
The histogram is keyed by canonical code, so no class numbering is shared with
the C oracle.  Feasible for n up to about 12.
"""
from __future__ import annotations

import itertools
from collections import Counter


def _bit(k: int, i: int, j: int) -> int:
    return i * (k - 1) + (j if j < i else j - 1)


def canonical(k: int, arcset) -> int:
    best = None
    for perm in itertools.permutations(range(k)):
        c = 0
        for i, j in arcset:
            c |= 1 << _bit(k, perm[i], perm[j])
        if best is None or c < best:
            best = c
    return best


def _connected(vs, und) -> bool:
    vs = list(vs)
    seen = {vs[0]}
    frontier = [vs[0]]
    sset = set(vs)
    while frontier:
        a = frontier.pop()
        for b in und[a]:
            if b in sset and b not in seen:
                seen.add(b)
                frontier.append(b)
    return len(seen) == len(vs)


def census_by_canon(n: int, arcs, k: int) -> Counter:
    """Counter {canonical code: number of connected induced k-subsets}."""
    arcs = {(int(a), int(b)) for a, b in arcs}
    und = {v: set() for v in range(n)}
    for a, b in arcs:
        und[a].add(b)
        und[b].add(a)
    out = Counter()
    for sub in itertools.combinations(range(n), k):
        if not _connected(sub, und):
            continue
        local = [(i, j) for i, a in enumerate(sub) for j, b in enumerate(sub) if i != j and (a, b) in arcs]
        out[canonical(k, local)] += 1
    return out


def census_undirected_by_canon(n: int, edges, k: int) -> Counter:
    """Counter {canonical undirected code: number of connected induced
    k-subsets} of an undirected graph, by all k-subsets; an edge {i, j}, i < j,
    is bit i(2k - i - 1)/2 + (j - i - 1) of the code."""
    adj = {v: set() for v in range(n)}
    for a, b in edges:
        if a != b:
            adj[int(a)].add(int(b))
            adj[int(b)].add(int(a))
    bit = lambda i, j: i * (2 * k - i - 1) // 2 + (j - i - 1)  # noqa: E731
    out = Counter()
    for sub in itertools.combinations(range(n), k):
        if not _connected(sub, adj):
            continue
        best = None
        for perm in itertools.permutations(range(k)):
            c = 0
            for x in range(k):
                for y in range(x + 1, k):
                    if sub[y] in adj[sub[x]]:
                        a, b = min(perm[x], perm[y]), max(perm[x], perm[y])
                        c |= 1 << bit(a, b)
            best = c if best is None else min(best, c)
        out[best] += 1
    return out
