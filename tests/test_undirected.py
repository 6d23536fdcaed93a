"""Undirected censuses (no GPU): the oracle's undirected classes and census,
pinned against the standard graph counts, an independent all-subsets
checker, closed forms and the paper's per-edge method for k = 4 (Algorithm
"und4", Table "ept"); and the library's host tables against the oracle's."""
import math
import os
from collections import Counter

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import brute

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1203_3415_amd",
                   "libmotif.so")


@pytest.mark.parametrize("k,conn,all_,labelled", [(3, 2, 4, 4), (4, 6, 11, 38), (5, 21, 34, 728)])
def test_undirected_class_counts(k, conn, all_, labelled):
    # connected graphs on k vertices, all graphs, labelled connected graphs:
    # the standard enumerations (1, 2, 6, 21 / 2, 4, 11, 34 / 1, 4, 38, 728)
    canon, cls, n_all, n_codes = oracle.undirected_class_table(k)
    assert (len(canon), n_all, n_codes) == (conn, all_, labelled)
    assert list(canon) == sorted(canon)


def _und(n, edges):
    return gg.from_arcs(n, [(a, b) for a, b in edges] + [(b, a) for a, b in edges])


def _by_canon(k, hist):
    canon = oracle.undirected_class_table(k)[0]
    return Counter({int(canon[c]): int(v) for c, v in enumerate(hist) if v})


@pytest.mark.parametrize("k", [3, 4, 5])
def test_matches_all_subsets(k):
    rng = np.random.default_rng(60 + k)
    for t in range(12):
        n = int(rng.integers(k, 11))
        g = gg.random_small(n, float(rng.uniform(0.1, 0.6)), float(rng.uniform(0, 1)), seed=6100 + 10 * k + t)
        want = brute.census_undirected_by_canon(g.n, g.arcs(), k)
        assert _by_canon(k, oracle.census_undirected(g, k)) == want, t


@pytest.mark.parametrize("k", [3, 4, 5])
def test_closed_forms(k):
    canon, cls, _, _ = oracle.undirected_class_table(k)

    def cid(edges):
        code = 0
        for a, b in edges:
            code |= 1 << oracle.und_bit(k, min(a, b), max(a, b))
        return cls[code]
    n = 9
    h = oracle.census_undirected(_und(n, [(i, j) for i in range(n) for j in range(i + 1, n)]), k)
    assert h[cid([(i, j) for i in range(k) for j in range(i + 1, k)])] == math.comb(n, k) == h.sum()
    path = cid([(i, i + 1) for i in range(k - 1)])
    h = oracle.census_undirected(_und(11, [(i, (i + 1) % 11) for i in range(11)]), k)
    assert h[path] == 11 == h.sum()
    h = oracle.census_undirected(gg.directed_path(10), k)   # direction does not matter
    assert h[path] == 10 - k + 1 == h.sum()
    h = oracle.census_undirected(gg.star(2, 3, 3), k)
    assert h[cid([(0, j) for j in range(1, k)])] == math.comb(8, k - 1) == h.sum()


def test_k4_matches_table_ept():
    canon, _, _, _ = oracle.undirected_class_table(4)
    name = {7: "claw", 13: "P4", 15: "tailed_triangle", 30: "C4", 31: "diamond", 63: "K4"}
    for g in (gg.chung_lu(300, 1500, 2.2, 2.4, 0.2, seed=4), gg.gnm_reciprocal(200, 900, 0.2, seed=6),
              gg.random_small(12, 0.4, 0.5, seed=3)):
        h = oracle.census_undirected(g, 4)
        ept = dict(zip(oracle.UNDIRECTED4, oracle.undirected4(g).tolist()))
        assert {name[int(c)]: int(h[i]) for i, c in enumerate(canon)} == ept


def test_library_undirected_tables_match_oracle():
    if not os.path.exists(LIB):
        pytest.skip("libmotif.so not built")
    import paper_1203_3415_amd as pm
    for k in (3, 4, 5):
        canon, ucls, _, _ = oracle.undirected_class_table(k)
        assert pm.num_undirected_classes(k) == len(canon)
        assert [pm.undirected_class_code(k, c) for c in range(len(canon))] == list(canon)
        # directed class -> undirected class: only the all-reciprocated ones
        _, dcanon, _, _ = oracle.class_table(k)
        for c, code in enumerate(dcanon):
            code = int(code)
            sym = all((code >> (i * (k - 1) + (j if j < i else j - 1)) & 1) ==
                      (code >> (j * (k - 1) + (i if i < j else i - 1)) & 1)
                      for i in range(k) for j in range(k) if i != j)
            want = -1
            if sym:
                u = 0
                for i in range(k):
                    for j in range(i + 1, k):
                        if code >> (i * (k - 1) + j - 1) & 1:
                            u |= 1 << oracle.und_bit(k, i, j)
                want = ucls[u]
            assert pm.class_undirected(k, c) == want, (k, c)
