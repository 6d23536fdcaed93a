"""Reading network files (host only, no GPU): Pajek .net in its arc, edge,
list and matrix notations, and plain edge lists, prepared as the paper
prepares its instances (vertices without neighbours removed; here also
self-loops dropped and repeated arcs merged).  Fixtures are hand-made
synthetic files in tests/golden/networks/; a round trip writes generated
graphs in both formats and reads them back."""
import os

import numpy as np
import pytest

import graphgen as gg

HERE = os.path.dirname(os.path.abspath(__file__))
NET = os.path.join(HERE, "golden", "networks")
LIB = os.path.join(os.path.dirname(HERE), "paper_1203_3415_amd", "libmotif.so")

# The fixture network after preparation: vertices 1, 2, 3, 4, 6, 7 of the file
# (5 has no neighbour) renumbered 0..5; arcs 1->2, 2->3, 3->1, 1->4, 2<->6, 4<->7.
WANT_OFF = [0, 2, 4, 5, 6, 7, 8]
WANT_IDX = [1, 3, 2, 4, 0, 5, 1, 3]


@pytest.fixture(scope="module")
def pm():
    if not os.path.exists(LIB):
        pytest.skip("libmotif.so not built")
    import paper_1203_3415_amd as pm
    return pm


@pytest.mark.parametrize("fname", ["tiny_arcs.net", "tiny_lists.net", "tiny_matrix.net"])
def test_pajek_notations(pm, fname):
    n, off, idx, ids, st = pm.read_network(os.path.join(NET, fname))
    assert n == 6
    assert off.tolist() == WANT_OFF and idx.tolist() == WANT_IDX
    assert ids.tolist() == [0, 1, 2, 3, 5, 6]   # 0-based file ids of the kept vertices
    assert st["self_loops_dropped"] == 1 and st["isolated_dropped"] == 1
    if fname != "tiny_matrix.net":
        assert st["arcs_read"] == 10 and st["duplicates_merged"] == 1


def test_pajek_keep_isolated(pm):
    n, off, idx, ids, st = pm.read_network(os.path.join(NET, "tiny_arcs.net"), keep_isolated=True)
    assert n == 7 and st["isolated_dropped"] == 0
    assert np.diff(off).tolist() == [2, 2, 1, 1, 0, 1, 1]   # 4 -> 4 dropped, 4 -> 7 kept


def test_edge_list(pm):
    n, off, idx, ids, st = pm.read_network(os.path.join(NET, "tiny_edges.txt"))
    assert (n, off.tolist(), idx.tolist()) == (6, WANT_OFF, WANT_IDX)
    assert ids.tolist() == [10, 20, 30, 40, 60, 70]
    assert st["self_loops_dropped"] == 1 and st["duplicates_merged"] == 1
    # as undirected edges every arc gains its reverse
    n2, off2, idx2, _, _ = pm.read_network(os.path.join(NET, "tiny_edges.txt"), undirected=True)
    a = {(u, int(v)) for u in range(n2) for v in idx2[off2[u]:off2[u + 1]]}
    assert all((v, u) in a for u, v in a) and len(a) == 12   # six undirected edges


def test_errors(pm):
    with pytest.raises(pm.MotifError) as e:
        pm.read_network(os.path.join(NET, "no_such_file.net"))
    assert e.value.name == "EIO"
    for bad in ("bad_range.net", "bad_token.txt"):
        with pytest.raises(pm.MotifError) as e:
            pm.read_network(os.path.join(NET, bad))
        assert e.value.name == "EPARSE", bad


def _write_pajek(g, path):
    a = g.arcs()
    s = set(map(tuple, a.tolist()))
    with open(path, "w") as f:
        f.write(f"*Vertices {g.n}\n*Arcs\n")
        for u, v in a.tolist():
            if (v, u) not in s:
                f.write(f"{u + 1} {v + 1}\n")
        f.write("*Edges\n")
        for u, v in a.tolist():
            if (v, u) in s and u < v:
                f.write(f"{u + 1} {v + 1} 1\n")


def test_round_trip(pm, tmp_path):
    # a generated graph with isolated vertices, written in both formats
    g = gg.pad_relabel(gg.chung_lu(400, 1600, 2.2, 2.4, 0.3, seed=9), 450, seed=3)
    keep = np.flatnonzero(np.bincount(g.arcs().ravel(), minlength=g.n) > 0)
    rank = -np.ones(g.n, np.int64)
    rank[keep] = np.arange(keep.size)
    want = gg.from_arcs(keep.size, rank[g.arcs()])
    p1 = str(tmp_path / "g.net")
    _write_pajek(g, p1)
    p2 = str(tmp_path / "g.txt")
    np.savetxt(p2, g.arcs() * 7 + 3, fmt="%d", header="tail head")
    for path in (p1, p2):
        n, off, idx, ids, st = pm.read_network(path)
        assert n == want.n and np.array_equal(off, want.out_off) and np.array_equal(idx, want.out_idx), path
    assert st["duplicates_merged"] == 0 and st["self_loops_dropped"] == 0
