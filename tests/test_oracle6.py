"""Pins of the k = 6 oracle (host only): the connected 6-sets grouped by the
canonical code of their induced digraph (the extension of Problems
Motifs-3/4/5 to six vertices, the paper's stated future work).

The canonical form must be invariant under relabelling and idempotent; the
ESU census must equal the independent pure-Python all-subsets checker on
seeded small graphs and the closed forms of complete digraphs, directed
cycles, stars and transitive tournaments; the anchor multiplicity (connected
4-subsets dominating the other two vertices) is checked on graphs where it is
known by hand."""
import itertools
import math
import random

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import brute

K = 6


def _bit(i, j):
    return i * (K - 1) + (j if j < i else j - 1)


def _code(arcs):
    c = 0
    for i, j in arcs:
        c |= 1 << _bit(i, j)
    return c


def _relabel(code, perm):
    out = 0
    for i in range(K):
        for j in range(K):
            if i != j and code >> _bit(i, j) & 1:
                out |= 1 << _bit(perm[i], perm[j])
    return out


def test_canonical_form():
    rng = random.Random(6)
    for _ in range(200):
        x = rng.getrandbits(30)
        c = oracle.canon6(x)
        assert c <= x and oracle.canon6(c) == c
        perm = list(range(K))
        rng.shuffle(perm)
        assert oracle.canon6(_relabel(x, perm)) == c
    assert oracle.canon6((1 << 30) - 1) == (1 << 30) - 1
    assert oracle.canon6(0) == 0
    # a single arc relabels to the lowest bit, the arc 0 -> 1
    assert oracle.canon6(1 << _bit(3, 5)) == 1 << _bit(0, 1) == 1


@pytest.mark.parametrize("seed", range(12))
def test_census6_matches_all_subsets(seed):
    rng = np.random.default_rng(600 + seed)
    n = int(rng.integers(7, 11))
    p = float(rng.uniform(0.15, 0.45))
    arcs = [(a, b) for a in range(n) for b in range(n) if a != b and rng.random() < p]
    g = gg.from_arcs(n, np.array(arcs).reshape(-1, 2))
    want = brute.census_by_canon(n, arcs, K)
    assert oracle.census6(g) == dict(want)


def test_census6_power_law_threads():
    g = gg.chung_lu(60, 150, 2.3, 2.3, 0.2, seed=61)
    one = oracle.census6(g, threads=1)
    assert one == oracle.census6(g, threads=4)
    assert sum(one.values()) > 1000


def test_closed_forms():
    full = (1 << 30) - 1
    kn = [(a, b) for a in range(8) for b in range(8) if a != b]
    assert oracle.census6(gg.from_arcs(8, np.array(kn))) == {full: math.comb(8, 6)}
    cyc = [(i, (i + 1) % 10) for i in range(10)]
    path = oracle.canon6(_code([(i, i + 1) for i in range(5)]))
    assert oracle.census6(gg.from_arcs(10, np.array(cyc))) == {path: 10}
    star = [(0, i) for i in range(1, 9)]
    out_star = oracle.canon6(_code([(0, i) for i in range(1, 6)]))
    assert oracle.census6(gg.from_arcs(9, np.array(star))) == {out_star: math.comb(8, 5)}
    tt = [(a, b) for a in range(9) for b in range(a + 1, 9)]
    tour = oracle.canon6(_code([(a, b) for a in range(6) for b in range(a + 1, 6)]))
    assert oracle.census6(gg.from_arcs(9, np.array(tt))) == {tour: math.comb(9, 6)}
    assert oracle.census6(gg.from_arcs(12, np.zeros((0, 2), np.int64))) == {}


def test_multiplicity6():
    full = (1 << 30) - 1
    assert oracle.multiplicity(6, full) == 15                       # every 4-subset of K6
    upath = _code([(i, i + 1) for i in range(5)] + [(i + 1, i) for i in range(5)])
    assert oracle.multiplicity(6, upath) == 1                       # only the middle four
    star = _code([(0, i) for i in range(1, 6)])
    assert oracle.multiplicity(6, star) == math.comb(5, 3)          # the centre and three leaves
    g = gg.chung_lu(40, 120, 2.3, 2.3, 0.2, seed=62)
    for code in oracle.census6(g):
        assert oracle.multiplicity(6, code) >= 1                    # every connected class has an anchor
