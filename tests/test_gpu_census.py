"""GPU parity: the HIP census (through the C ABI) against the CPU oracle,
bit-exact, on seeded inputs covering several tiles, ragged rows, hubs, both
label-storage paths, the degenerate cases and the error paths."""
import math

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1203_3415_amd as pm
    pm.lib()
    return pm


def _dev(pm, off, idx):
    return pm.to_device(np.asarray(off), np.asarray(idx))


def gpu_census(pm, g, k, **kw):
    off, idx = _dev(pm, g.out_off, g.out_idx)
    return pm.census(off, idx, g.n, k, **kw)


def assert_parity(pm, g, k, label):
    print(f"[case] {label} n={g.n} m={g.m} k={k}", flush=True)
    got = gpu_census(pm, g, k)
    want = oracle.census(g, k)
    if not np.array_equal(got, want):
        bad = np.flatnonzero(got != want)
        raise AssertionError(f"{label} k={k}: {len(bad)} classes differ, first {bad[:6].tolist()}: "
                             f"gpu {got[bad[:6]].tolist()} oracle {want[bad[:6]].tolist()}")


@pytest.mark.parametrize("k", [3, 4, 5])
def test_small_random(pm, k):
    rng = np.random.default_rng(10 + k)
    for t in range(30 if k < 5 else 16):
        n = int(rng.integers(2, 26))
        g = gg.random_small(n, float(rng.uniform(0.05, 0.7)), float(rng.uniform(0, 1)), seed=500 * k + t)
        assert_parity(pm, g, k, f"random_small#{t}")


@pytest.mark.parametrize("k", [3, 4, 5])
def test_structured(pm, k):
    cases = {
        "complete": gg.complete_digraph(9),
        "transitive": gg.transitive_tournament(10),
        "cycle": gg.directed_cycle(12),
        "cycle_k": gg.directed_cycle(k),
        "path": gg.directed_path(12),
        "star": gg.star(4, 4, 5),
        "empty": gg.from_arcs(10, []),
        "n_lt_k": gg.complete_digraph(k - 1),
        "one_arc": gg.from_arcs(5, [(3, 1)]),
        "bidirected": gg.random_small(14, 0.3, 1.0, seed=3),
        "dag": gg.from_arcs(15, [(i, j) for i in range(15) for j in range(i + 1, 15) if (i * 7 + j * 3) % 4 == 0]),
        "isolated": gg.disjoint_union(gg.from_arcs(7, []), gg.random_small(9, 0.4, 0.3, seed=4), gg.from_arcs(5, [])),
    }
    for name, g in cases.items():
        assert_parity(pm, g, k, name)


@pytest.mark.parametrize("k", [3, 4, 5])
def test_gnm_n1000_m5500(pm, k):
    # the paper-shaped small workload: G(n=1000, m=5000) + 10% reciprocated
    assert_parity(pm, gg.gnm_reciprocal(1000, 5000, 0.1, seed=1), k, "gnm1000")


@pytest.mark.parametrize("k", [3, 4])
def test_power_law_n2000(pm, k):
    assert_parity(pm, gg.chung_lu(2000, 8000, 2.3, 2.3, 0.05, seed=3), k, "chung_lu2000")


def test_power_law_k5(pm):
    assert_parity(pm, gg.chung_lu(600, 2400, 2.2, 2.5, 0.1, seed=4), 5, "chung_lu600")


def _star_expect(k, na, nb, nc):
    C = oracle.N_CLASSES[k]
    expect = np.zeros(C, np.uint64)
    for i in range(k):
        for j in range(k - i):
            l = k - 1 - i - j
            cnt = math.comb(na, i) * math.comb(nb, j) * math.comb(nc, l)
            if not cnt:
                continue
            arcs, leaf = [], 1
            for _ in range(i):
                arcs += [(0, leaf), (leaf, 0)]; leaf += 1
            for _ in range(j):
                arcs.append((0, leaf)); leaf += 1
            for _ in range(l):
                arcs.append((leaf, 0)); leaf += 1
            expect[oracle.class_of(k, arcs)] += cnt
    return expect


@pytest.mark.parametrize("k,sizes", [(3, (3000, 2000, 1500)), (4, (2500, 2000, 1500)), (5, (90, 70, 60))])
def test_hub_star_closed_form(pm, k, sizes):
    # a hub far above the LDS sort threshold; expected values by the multinomial
    # closed form of the star (only sets containing the centre are connected)
    g = gg.star(*sizes)
    print(f"[case] star{sizes} k={k}", flush=True)
    got = gpu_census(pm, g, k)
    assert np.array_equal(got, _star_expect(k, *sizes))


@pytest.mark.parametrize("k", [4, 5])
def test_global_label_path(pm, k):
    # n above the LDS label capacity (131072 vertices at 4 bits, 65536 at 8 bits)
    base = gg.chung_lu(3000, 12000 if k == 4 else 6000, 2.3, 2.3, 0.1, seed=21)
    g = gg.relabel(gg.disjoint_union(base, gg.from_arcs(140000 - base.n, [])), seed=22)
    assert_parity(pm, g, k, "global_labels")


def _shuffled_rows(g, seed):
    rng = np.random.default_rng(seed)
    idx = g.out_idx.copy()
    for v in range(g.n):
        a, b = g.out_off[v], g.out_off[v + 1]
        idx[a:b] = rng.permutation(idx[a:b])
    return idx


def test_row_sort_paths(pm):
    """Rows of every sort path, given unsorted: in registers (up to 64
    half-edges), bitonic in LDS (65-256), bitmap in LDS (longer, while 2n bits
    fit in 64 KB) and bitmap in global memory (n = 300,000 after padding with
    isolated vertices and relabelling)."""
    g = gg.chung_lu(2500, 10000, 2.1, 2.1, 0.2, seed=24)
    h = np.diff(g.out_off) + np.bincount(g.out_idx, minlength=g.n)
    assert (h > 256).sum() >= 3 and ((h > 64) & (h <= 256)).sum() >= 10
    big = gg.pad_relabel(g, 300000, seed=25)
    want = {3: oracle.census(g, 3), 4: oracle.method_census(g, 4)}  # the method reference: ESU takes 30 s here
    for name, G in (("lds", g), ("global", big)):
        off_d, idx_d = _dev(pm, G.out_off, _shuffled_rows(G, 26))
        for k in (3, 4):
            print(f"[case] row sort paths, {name} bitmap, k={k}", flush=True)
            assert np.array_equal(pm.census(off_d, idx_d, G.n, k), want[k]), (name, k)


def test_in_csr_placement(pm):
    """A single graph with an in-CSR is placed by merging each row's out and
    in halves when every row of both CSRs is strictly increasing, and takes
    the counting scatter and sort otherwise.  Both routes give the oracle's
    census for a good in-CSR, in any mix of sorted and unsorted rows, and
    both reject a bad one before any census runs on it."""
    g = gg.chung_lu(1200, 6000, 2.2, 2.2, 0.25, seed=41)
    want = {k: oracle.census(g, k) for k in (3, 4)}
    in_off, in_idx = g.in_csr()
    off_d, idx_d = _dev(pm, g.out_off, g.out_idx)
    shuf_d = _dev(pm, g.out_off, _shuffled_rows(g, 42))[1]
    io_d, ii_d = _dev(pm, in_off, in_idx)
    rng = np.random.default_rng(43)
    ii_shuf = in_idx.copy()
    for v in range(g.n):
        a, b = in_off[v], in_off[v + 1]
        ii_shuf[a:b] = rng.permutation(ii_shuf[a:b])
    iis_d = _dev(pm, in_off, ii_shuf)[1]
    # good in-CSR: both sorted (merge placement), out rows unsorted (an
    # in-arc lookup in an unsorted out row must not count as a miss), in rows
    # unsorted, both unsorted
    for name, od, ind in (("sorted", idx_d, ii_d), ("out unsorted", shuf_d, ii_d), ("in unsorted", idx_d, iis_d),
                          ("both unsorted", shuf_d, iis_d)):
        for k in (3, 4):
            print(f"[case] in-CSR placement, good, {name}, k={k}", flush=True)
            assert np.array_equal(pm.census(off_d, od, g.n, k, in_off=io_d, in_idx=ind), want[k]), (name, k)
            outs = pm.census_multi(off_d, od, g.n, (k,), in_off=io_d, in_idx=ind)
            assert np.array_equal(outs[0], want[k]), (name, k)

    def expect(name, in_off_bad, in_idx_bad, code, od=idx_d):
        bo, bi = _dev(pm, np.asarray(in_off_bad, np.int32), np.asarray(in_idx_bad, np.int32))
        for k in (3, 4):
            print(f"[case] in-CSR placement, bad, {name}, k={k}", flush=True)
            with pytest.raises(pm.MotifError) as e:
                pm.census(off_d, od, g.n, k, in_off=bo, in_idx=bi)
            assert e.value.name == code, (name, k, e.value.name)
            with pytest.raises(pm.MotifError) as e:
                pm.census_multi(off_d, od, g.n, (3, k) if k == 4 else (k,), in_off=bo, in_idx=bi)
            assert e.value.name == code, (name, k, e.value.name)

    # a non-arc that keeps its row strictly increasing: found by the merge
    # placement's own lookups
    v = next(v for v in range(g.n) if in_off[v + 1] - in_off[v] >= 2 and in_idx[in_off[v]] > 0)
    present = set(in_idx[in_off[v]:in_off[v + 1]].tolist())
    x = next(x for x in range(in_idx[in_off[v]]) if x != v and x not in present)
    bad = in_idx.copy()
    bad[in_off[v]] = x
    expect("non-arc, rows sorted", in_off, bad, "ETRANSPOSE")
    expect("non-arc, out rows unsorted", in_off, bad, "ETRANSPOSE", od=shuf_d)
    # a repeated in-arc (its row is no longer increasing: the general route)
    dup = in_idx.copy()
    dup[in_off[v] + 1] = dup[in_off[v]]
    expect("repeated in-arc", in_off, dup, "ETRANSPOSE")
    # the right arcs in the wrong rows: every row sorted, m arcs in all
    moved = in_off.copy()
    w = next(w for w in range(g.n - 1) if moved[w + 1] - moved[w] >= 1 and moved[w + 2] - moved[w + 1] >= 1)
    moved[w + 1] -= 1
    expect("arc in the wrong row", moved, in_idx, "ETRANSPOSE")
    # an index out of range, and offsets that do not end at m
    oob = in_idx.copy()
    oob[-1] = g.n
    expect("index out of range", in_off, oob, "EINDEX")
    short = in_off.copy()
    short[-1] -= 1
    expect("offsets end below m", short, in_idx, "EINVAL_SHAPE")


@pytest.mark.parametrize("k", [3, 4])
def test_unsorted_rows_and_in_csr(pm, k):
    g = gg.chung_lu(800, 4000, 2.2, 2.2, 0.3, seed=31)
    want = oracle.census(g, k)
    rng = np.random.default_rng(5)
    idx = g.out_idx.copy()
    for v in range(g.n):
        a, b = g.out_off[v], g.out_off[v + 1]
        idx[a:b] = rng.permutation(idx[a:b])
    off_d, idx_d = _dev(pm, g.out_off, idx)
    in_off, in_idx = g.in_csr()
    in_idx_shuf = in_idx.copy()
    for v in range(g.n):
        a, b = in_off[v], in_off[v + 1]
        in_idx_shuf[a:b] = rng.permutation(in_idx_shuf[a:b])
    io_d, ii_d = _dev(pm, in_off, in_idx_shuf)
    assert np.array_equal(pm.census(off_d, idx_d, g.n, k), want)
    assert np.array_equal(pm.census(off_d, idx_d, g.n, k, in_off=io_d, in_idx=ii_d), want)
    # a wrong in-CSR: one in-arc replaced by a non-arc
    bad = in_idx.copy()
    v = int(np.argmax(np.diff(in_off)))
    a = in_off[v]
    present = set(bad[in_off[v]:in_off[v + 1]].tolist())
    bad[a] = next(x for x in range(g.n) if x != v and x not in present)
    bo_d, bi_d = _dev(pm, in_off, bad)
    with pytest.raises(pm.MotifError) as e:
        pm.census(off_d, idx_d, g.n, k, in_off=bo_d, in_idx=bi_d)
    assert e.value.name == "ETRANSPOSE"
    # a repeated in-arc (count right, one arc missing)
    dup = in_idx.copy()
    w = next(v for v in range(g.n) if in_off[v + 1] - in_off[v] >= 2)
    dup[in_off[w] + 1] = dup[in_off[w]]
    do_d, di_d = _dev(pm, in_off, dup)
    with pytest.raises(pm.MotifError) as e:
        pm.census(off_d, idx_d, g.n, k, in_off=do_d, in_idx=di_d)
    assert e.value.name == "ETRANSPOSE"


def _expect_error(pm, off, idx, n, k, name):
    print(f"[case] error {name}", flush=True)
    off_d, idx_d = _dev(pm, np.asarray(off, np.int32), np.asarray(idx, np.int32))
    with pytest.raises(pm.MotifError) as e:
        pm.census(off_d, idx_d, n, k)
    assert e.value.name == name, e.value


def test_errors(pm):
    _expect_error(pm, [0, 1, 2, 2], [1, 1], 3, 3, "ESELFLOOP")
    _expect_error(pm, [0, 2, 2, 2], [1, 1], 3, 3, "EDUP")
    _expect_error(pm, [0, 1, 2, 2], [5, 0], 3, 3, "EINDEX")
    _expect_error(pm, [0, 1, 2, 2], [-1, 0], 3, 3, "EINDEX")
    _expect_error(pm, [0, 2, 1, 2], [1, 2], 3, 4, "EINVAL_SHAPE")
    _expect_error(pm, [1, 1, 2, 2], [1, 2], 3, 4, "EINVAL_SHAPE")
    _expect_error(pm, [0, 1, 2, 3], [1, 2], 3, 4, "EINVAL_SHAPE")
    _expect_error(pm, [0, 1, 2, 2], [1, 0], 3, 6, "EINVAL_K")
    # a repeated arc in a row of each sort path: bitonic in LDS (100 keys),
    # bitmap in LDS (300, 2,000 and 5,000 keys), and bitmap in global memory
    # (n = 300,000: 2n bits no longer fit in LDS)
    for deg, n in ((100, 101), (300, 301), (2000, 2001), (5000, 5001), (5000, 300000)):
        idx = list(range(1, deg + 1)) + [7]
        _expect_error(pm, [0, deg + 1] + [deg + 1] * (n - 1), idx, n, 4, "EDUP")
    # histogram untouched on error
    import torch
    off_d, idx_d = _dev(pm, np.asarray([0, 1, 2, 2], np.int32), np.asarray([1, 1], np.int32))
    out = torch.full((13,), 7, dtype=torch.int64, device="cuda")
    with pytest.raises(pm.MotifError):
        pm.census(off_d, idx_d, 3, 3, out=out)
    assert bool((out == 7).all())


def test_async_census(pm):
    # Enqueue-only form: the stream carries the histogram and a status word.
    import torch
    g = gg.chung_lu(900, 4500, 2.2, 2.3, 0.15, seed=43)
    off, idx = _dev(pm, g.out_off, g.out_idx)
    s = torch.cuda.Stream()
    for k in (3, 4, 5):
        print(f"[case] async k={k}", flush=True)
        hist = torch.full((pm.NUM_CLASSES[k],), 7, dtype=torch.int64, device="cuda")
        status = torch.full((1,), 99, dtype=torch.int32, device="cuda")
        pm.census_async(off, idx, g.n, k, hist, status, stream=s)
        s.synchronize()
        assert int(status.item()) == 0
        # the method reference (pinned against ESU) stands in for ESU at this size
        assert np.array_equal(hist.cpu().numpy().view(np.uint64), oracle.method_census(g, k))
    # an invalid graph: the status word carries the code, the histogram is untouched
    bo, bi = _dev(pm, np.asarray([0, 1, 2, 2], np.int32), np.asarray([1, 1], np.int32))
    hist = torch.full((13,), 7, dtype=torch.int64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    pm.census_async(bo, bi, 3, 3, hist, status, stream=s)
    s.synchronize()
    assert int(status.item()) == -4   # MOTIF_ESELFLOOP
    assert bool((hist == 7).all())
    # and the next call on the same stream is unaffected
    hist4 = torch.zeros(199, dtype=torch.int64, device="cuda")
    pm.census_async(off, idx, g.n, 4, hist4, status, stream=s)
    s.synchronize()
    assert int(status.item()) == 0
    assert np.array_equal(hist4.cpu().numpy().view(np.uint64), oracle.method_census(g, 4))


@pytest.mark.parametrize("k", [3, 4, 5])
def test_invariances(pm, k):
    g = gg.chung_lu(400, 1600, 2.2, 2.4, 0.2, seed=41)
    print(f"[case] invariances k={k}", flush=True)
    h = gpu_census(pm, g, k)
    assert np.array_equal(gpu_census(pm, gg.relabel(g, 9), k), h)
    g2 = gg.gnm_reciprocal(300, 900, 0.3, seed=42)
    h2 = gpu_census(pm, g2, k)
    assert np.array_equal(gpu_census(pm, gg.disjoint_union(g, g2), k), h + h2)
    # reversing every arc sends each class to the class of its transpose
    C = len(h)
    expect = np.zeros(C, np.uint64)
    for c in range(C):
        code = pm.class_code(k, c)
        t = 0
        for i in range(k):
            for j in range(k):
                if i != j and code >> (i * (k - 1) + (j if j < i else j - 1)) & 1:
                    t |= 1 << (j * (k - 1) + (i if i < j else i - 1))
        expect[pm.class_of_code(k, t)] += h[c]
    assert np.array_equal(gpu_census(pm, gg.reverse(g), k), expect)


@pytest.mark.parametrize("k", [3, 4, 5])
def test_batch_matches_alone(pm, k):
    rng = np.random.default_rng(60 + k)
    graphs = []
    for t in range(14):
        n = int(rng.integers(20, 400 if k < 5 else 150))
        m = int(n * rng.uniform(1.5, 4.0))
        graphs.append(gg.chung_lu(n, m, 2.3, 2.3, float(rng.uniform(0, 0.2)), seed=700 + t))
    graphs.insert(3, gg.from_arcs(0, []))
    graphs.insert(7, gg.from_arcs(12, []))
    graphs.append(gg.complete_digraph(k))
    dev = [(*_dev(pm, g.out_off, g.out_idx), g.n) for g in graphs]
    print(f"[case] batch k={k} graphs={len(graphs)}", flush=True)
    hb = pm.census_batch(dev, k)
    hl = pm.census_batch_loop(dev, k)
    for i, g in enumerate(graphs):
        want = oracle.census(g, k)
        assert np.array_equal(hb[i], want), f"batch graph {i}"
        assert np.array_equal(hl[i], want), f"loop graph {i}"


def test_batch_with_in_csr_and_errors(pm):
    gs = [gg.chung_lu(200, 800, 2.3, 2.3, 0.1, seed=80 + t) for t in range(4)]
    dev = []
    for i, g in enumerate(gs):
        o, x = _dev(pm, g.out_off, g.out_idx)
        if i % 2 == 0:
            io, ii = _dev(pm, *g.in_csr())
            dev.append((o, x, g.n, io, ii))
        else:
            dev.append((o, x, g.n))
    hb = pm.census_batch(dev, 4)
    for i, g in enumerate(gs):
        assert np.array_equal(hb[i], oracle.census(g, 4))
    # one graph with a self-loop fails the whole batch
    bad_off, bad_idx = _dev(pm, np.asarray([0, 1, 1], np.int32), np.asarray([0], np.int32))
    with pytest.raises(pm.MotifError) as e:
        pm.census_batch(dev + [(bad_off, bad_idx, 2)], 4)
    assert e.value.name == "ESELFLOOP"


@pytest.mark.parametrize("k", [4, 5])
def test_tuning_variants_agree(pm, k):
    g = gg.chung_lu(700, 3000, 2.2, 2.3, 0.1, seed=90)
    want = oracle.census(g, k)
    saved = pm.get_tuning(k)
    try:
        blocks = (256, 512, 1024) if k == 4 else (512, 1024)
        for scheme in (1, 2):
            for block in blocks:
                for tile in (1, 7, 64):
                    for gpc in (1, 3):
                        pm.set_tuning(k, block=block, tile=tile, grid_per_cu=gpc, heavy=scheme)
                        print(f"[case] tuning k={k} scheme={scheme} block={block} tile={tile} gpc={gpc}", flush=True)
                        assert np.array_equal(gpu_census(pm, g, k), want)
    finally:
        pm.set_tuning(k, **saved)


@pytest.mark.parametrize("k", [4, 5])
@pytest.mark.parametrize("scheme", [1, 2])
def test_both_schemes(pm, k, scheme):
    # scheme 1: core reuse (default); scheme 2: per-anchor scan
    saved = pm.get_tuning(k)
    try:
        pm.set_tuning(k, heavy=scheme)
        rng = np.random.default_rng(200 + k)
        for t in range(16 if k == 4 else 8):
            n = int(rng.integers(3, 40 if k == 4 else 28))
            g = gg.random_small(n, float(rng.uniform(0.05, 0.7)), float(rng.uniform(0, 1)), seed=900 * k + t)
            assert_parity(pm, g, k, f"scheme{scheme} random#{t}")
        assert_parity(pm, gg.chung_lu(700, 3000, 2.1, 2.2, 0.2, seed=91), k, f"scheme{scheme} chung_lu700")
        sizes = (300, 250, 200) if k == 4 else (40, 30, 25)
        g = gg.star(*sizes)
        print(f"[case] scheme{scheme} star k={k}", flush=True)
        assert np.array_equal(gpu_census(pm, g, k), _star_expect(k, *sizes))
        base = gg.chung_lu(2500, 9000 if k == 4 else 5000, 2.3, 2.3, 0.1, seed=92)
        big = gg.relabel(gg.disjoint_union(base, gg.from_arcs(140000 - base.n, [])), seed=93)
        assert_parity(pm, big, k, f"scheme{scheme} global_labels")
    finally:
        pm.set_tuning(k, **saved)


def test_schemes_agree_on_power_law(pm):
    g = gg.chung_lu(20000, 100000, 2.1, 2.1, 0.2, seed=94)
    off, idx = pm.to_device(g.out_off, g.out_idx)
    saved = pm.get_tuning(4)
    try:
        pm.set_tuning(4, heavy=1)
        a = pm.census(off, idx, g.n, 4)
        pm.set_tuning(4, heavy=2)
        b = pm.census(off, idx, g.n, 4)
    finally:
        pm.set_tuning(4, **saved)
    assert np.array_equal(a, b)


def _partner_fan(n_part=60, d_part=30, d_a=40, seed=5):
    """Centre 0 with a heavier side 1 and many light partners (of lower rank)
    whose neighbourhoods overlap N(1), each other and side 1 itself; random
    arc types.  Each unit (0, 1) has its light partners split over several
    sub-chunks, by count and by the size of their merged neighbourhoods."""
    rng = np.random.default_rng(seed)
    arcs = set()

    def link(x, y):
        t = int(rng.integers(1, 4))
        if t & 1:
            arcs.add((x, y))
        if t & 2:
            arcs.add((y, x))

    parts = list(range(2, 2 + n_part))
    na = list(range(2 + n_part, 2 + n_part + d_a))
    nxt = 2 + n_part + d_a
    link(0, 1)
    for q in na:
        link(1, q)
    for c in parts:
        link(0, c)
        nb = set(rng.choice(na, size=int(rng.integers(2, 8)), replace=False).tolist())
        nb.update(rng.choice(parts, size=int(rng.integers(0, 4)), replace=False).tolist())
        if rng.random() < 0.3:
            nb.add(1)
        nb.discard(c)
        while len(nb) < d_part - 1:
            nb.add(nxt)
            nxt += 1
        for q in nb:
            link(c, q)
    return gg.from_arcs(nxt, sorted((x, y) for x, y in arcs if x != y))


@pytest.mark.gpu
def test_k5_light_subchunks(pm):
    """The factored k = 5 path where it splits: one unit's light partners in
    several sub-chunks, partners inside N(a), adjacent to a (triangles) and
    to each other; also relabelled, so the triangles' centres move."""
    g = _partner_fan()
    assert_parity(pm, g, 5, "partner fan")
    assert_parity(pm, gg.relabel(g, seed=6), 5, "partner fan relabelled")
    # light partners of a few hundred neighbours (one or two per sub-chunk):
    # too many connected 5-sets for the oracle, so against the per-anchor
    # kernel, itself checked against the oracle above
    g = _partner_fan(n_part=12, d_part=300, d_a=400, seed=7)
    off, idx = pm.to_device(g.out_off, g.out_idx)
    saved = pm.get_tuning(5)
    try:
        print(f"[case] wide partner fan n={g.n} m={g.m}", flush=True)
        pm.set_tuning(5, heavy=1)
        a = pm.census(off, idx, g.n, 5)
        pm.set_tuning(5, heavy=2)
        b = pm.census(off, idx, g.n, 5)
    finally:
        pm.set_tuning(5, **saved)
    assert np.array_equal(a, b)
    assert int(a.sum()) > 0


@pytest.mark.gpu
def test_census_multi_matches_single(pm):
    """One shared build for k = 3, 4, 5 gives what three separate calls give,
    in any order of ks; the errors match motif_census."""
    g = gg.chung_lu(1500, 7000, 2.2, 2.4, 0.15, seed=21)
    off, idx = pm.to_device(g.out_off, g.out_idx)
    singles = {k: pm.census(off, idx, g.n, k) for k in (3, 4, 5)}
    for ks in ((3, 4, 5), (5, 3), (4,)):
        outs = pm.census_multi(off, idx, g.n, ks)
        for k, h in zip(ks, outs):
            assert np.array_equal(h, singles[k]), (ks, k)
    assert np.array_equal(singles[3], oracle.census(g, 3))
    bad_off, bad_idx = pm.to_device(np.array([0, 1, 1], np.int32), np.array([0], np.int32))
    with pytest.raises(pm.MotifError) as e:
        pm.census_multi(bad_off, bad_idx, 2, (3, 4))
    assert e.value.name == "ESELFLOOP"
    with pytest.raises(pm.MotifError):
        pm.census_multi(off, idx, g.n, (3, 3))


@pytest.mark.gpu
def test_census_multi_in_csr(pm):
    """With an in-CSR the multi-size call checks it on its second stream,
    beside the censuses: a good one changes nothing, for one size as for
    several, and a bad one fails the call with every output left as it was."""
    import torch
    g = gg.chung_lu(1500, 7000, 2.2, 2.4, 0.15, seed=22)
    off, idx = pm.to_device(g.out_off, g.out_idx)
    in_off, in_idx = g.in_csr()
    io, ii = pm.to_device(in_off, in_idx)
    singles = {k: pm.census(off, idx, g.n, k) for k in (3, 4, 5)}
    for ks in ((3, 4), (4,), (5, 3, 4)):
        print(f"[case] census_multi in-CSR ks={ks}", flush=True)
        outs = pm.census_multi(off, idx, g.n, ks, in_off=io, in_idx=ii)
        for k, h in zip(ks, outs):
            assert np.array_equal(h, singles[k]), (ks, k)
    bad = in_idx.copy()
    v = int(np.argmax(np.diff(in_off)))
    present = set(bad[in_off[v]:in_off[v + 1]].tolist())
    bad[in_off[v]] = next(x for x in range(g.n) if x != v and x not in present)
    bo, bi = pm.to_device(in_off, bad)
    for ks in ((3, 4), (4,)):
        print(f"[case] census_multi bad in-CSR ks={ks}", flush=True)
        outs = [torch.full((pm.NUM_CLASSES[k],), 7, dtype=torch.int64, device="cuda") for k in ks]
        with pytest.raises(pm.MotifError) as e:
            pm.census_multi(off, idx, g.n, ks, in_off=bo, in_idx=bi, outs=outs)
        assert e.value.name == "ETRANSPOSE"
        assert all(bool((h == 7).all()) for h in outs)


@pytest.mark.gpu
@pytest.mark.parametrize("k,n", [(3, 400), (4, 400), (5, 60)])
def test_dense_closed_forms(pm, k, n):
    """Complete digraph and transitive tournament: every k-set induces the
    same class, C(n, k) times.  At n = 400 every k = 4 anchor is heavy and a
    flattened row layout holds more than 64 K entries (the unbucketed row
    search); at k = 5 every triple runs on the wave path."""
    full = (1 << (k * (k - 1))) - 1
    want = math.comb(n, k)
    cases = {"complete": (gg.complete_digraph(n), full)}
    # transitive tournament: arc i -> j for i < j, i.e. slot i has arcs to every later slot
    tt = 0
    for i in range(k):
        for j in range(i + 1, k):
            tt |= 1 << (i * (k - 1) + (j - 1))
    cases["transitive"] = (gg.transitive_tournament(n), tt)
    for name, (g, code) in cases.items():
        print(f"[case] dense {name} n={n} k={k}", flush=True)
        h = gpu_census(pm, g, k)
        cls = pm.class_of_code(k, code)
        assert int(h[cls]) == want, name
        assert int(h.sum()) == want, name


@pytest.mark.parametrize("k", [3, 4, 5])
def test_census_of_network_files(pm, k, tmp_path):
    # A file read the way the paper prepares its instances, censused on the
    # device and by the oracle from the same CSR.
    import os
    net = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "networks")
    g = gg.gnm_reciprocal(120, 500, 0.3, seed=21)
    path = str(tmp_path / "g.txt")
    np.savetxt(path, g.arcs() * 3 + 1, fmt="%d")
    for p in (os.path.join(net, "tiny_arcs.net"), path):
        n, off, idx, _, _ = pm.read_network(p)
        h = gg.Digraph(n, off, idx)
        print(f"[case] network file {os.path.basename(p)} n={n} m={h.m} k={k}", flush=True)
        assert_parity(pm, h, k, os.path.basename(p))


@pytest.mark.parametrize("k", [3, 4, 5])
def test_undirected_census(pm, k):
    # the undirected version of each graph, by the oracle's ESU on it
    rng = np.random.default_rng(70 + k)
    graphs = [gg.random_small(int(rng.integers(k, 20)), float(rng.uniform(0.1, 0.6)), float(rng.uniform(0, 1)),
                              seed=7100 + 10 * k + t) for t in range(8)]
    graphs += [gg.chung_lu(300 if k < 5 else 120, 1200 if k < 5 else 400, 2.2, 2.4, 0.2, seed=72 + k),
               gg.star(3, 4, 2), gg.complete_digraph(7), gg.from_arcs(5, [])]
    for t, g in enumerate(graphs):
        off, idx = _dev(pm, g.out_off, g.out_idx)
        print(f"[case] undirected k={k} graph {t} n={g.n} m={g.m}", flush=True)
        got = pm.census_undirected(off, idx, g.n, k)
        assert np.array_equal(got, oracle.census_undirected(g, k)), t
    # an undirected graph listed with each edge once or in both directions
    g = gg.chung_lu(200, 700, 2.3, 2.3, 0.0, seed=75)
    both = gg.from_arcs(g.n, np.unique(np.concatenate([g.arcs(), g.arcs()[:, ::-1]]), axis=0))
    o1, i1 = _dev(pm, g.out_off, g.out_idx)
    o2, i2 = _dev(pm, both.out_off, both.out_idx)
    assert np.array_equal(pm.census_undirected(o1, i1, g.n, k), pm.census_undirected(o2, i2, both.n, k))


def test_w_rows_reused_across_calls(pm):
    # The W rows of the core-reuse kernels are kept per stream and must be
    # left all zero by every census: alternate graphs of different sizes and
    # k on one stream and compare each result with the CPU reference.
    import torch
    s = torch.cuda.Stream()
    a = gg.chung_lu(3000, 20000, 2.1, 2.1, 0.2, seed=91)
    b = gg.chung_lu(800, 4000, 2.2, 2.3, 0.1, seed=92)
    want = {(id(a), 4): oracle.method_census(a, 4), (id(b), 4): oracle.method_census(b, 4),
            (id(b), 5): oracle.method_census(b, 5)}
    dev = {id(g): _dev(pm, g.out_off, g.out_idx) for g in (a, b)}
    for rnd, (g, k) in enumerate([(a, 4), (b, 4), (b, 5), (a, 4), (b, 5), (b, 4), (a, 4)]):
        off, idx = dev[id(g)]
        print(f"[case] W rows reuse round {rnd} n={g.n} k={k}", flush=True)
        got = pm.census(off, idx, g.n, k, stream=s)
        assert np.array_equal(got, want[(id(g), k)]), rnd


def test_profile_modes(pm):
    """Events around build and census kernel (mode 1), around the census
    kernel only (mode 2: the build reads -1), and no other modes."""
    g = gg.chung_lu(900, 4500, 2.2, 2.3, 0.15, seed=44)
    off, idx = _dev(pm, g.out_off, g.out_idx)
    try:
        pm.profile_enable(True)
        pm.census(off, idx, g.n, 4)
        km, bm = pm.profile_read(4)
        assert km > 0 and bm > 0
        pm.profile_enable(True, census_only=True)
        with pytest.raises(pm.MotifError):
            pm.profile_read(4)  # nothing recorded since the mode was set
        pm.census_multi(off, idx, g.n, (3, 4))
        for k in (3, 4):
            km, bm = pm.profile_read(k)
            assert km > 0 and bm == -1.0
    finally:
        pm.profile_enable(False)
    assert pm.lib().motif_profile_enable(3) == -13  # MOTIF_EINVAL_ARG
