"""CPU tests of host-side helpers: generators and z-scores."""
import numpy as np
import pytest

import graphgen as gg


def test_arc_switch_many_preserves_degrees_and_simplicity():
    base = gg.chung_lu(500, 2500, 2.3, 2.3, 0.1, seed=3)
    rs = gg.arc_switch_many(base, 50 * base.m, [11, 12, 13])
    a0 = base.arcs()
    for g in rs:
        a = g.arcs()   # from_arcs already rejects loops and repeated arcs
        assert g.m == base.m
        assert np.array_equal(np.bincount(a[:, 0], minlength=g.n), np.bincount(a0[:, 0], minlength=g.n))
        assert np.array_equal(np.bincount(a[:, 1], minlength=g.n), np.bincount(a0[:, 1], minlength=g.n))
        assert (a != a0).any()
    again = gg.arc_switch_many(base, 50 * base.m, [11])
    assert np.array_equal(again[0].out_idx, rs[0].out_idx)   # deterministic in the seed


def test_zscores_match_float_formula():
    from paper_1203_3415_amd.nullmodel import zscores
    rng = np.random.default_rng(2)
    h = rng.integers(0, 1000, size=(50, 13)).astype(np.uint64)
    h[:, 3] = 7                       # constant column: sd = 0 -> NaN
    z = zscores(h)
    rnd = h[1:].astype(float)
    want = (h[0].astype(float) - rnd.mean(0)) / rnd.std(0, ddof=1)
    ok = ~np.isnan(want)
    assert np.allclose(z[ok], want[ok], rtol=1e-12)
    assert np.isnan(z[3])


def test_zscores_exact_for_huge_counts():
    from paper_1203_3415_amd.nullmodel import zscores
    big = np.array([[2**62 + 5], [2**62], [2**62 + 2], [2**62 + 4]], dtype=np.uint64)
    z = zscores(big)
    # randomised rows: 0, 2, 4 above 2^62 -> mean 2, sd 2; real is +5 -> z = 1.5
    assert z[0] == pytest.approx(1.5, rel=1e-12)


def test_bench_script_on_the_host():
    """bench.py parses, refuses more than one GPU with a message, and its byte
    models order as the kernels do: core reuse reads less than the per-anchor
    method, and every model is positive on a small graph."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]
    sys.path.insert(0, root)
    import bench
    st = bench.graph_stats(gg.chung_lu(2000, 10000, 2.2, 2.2, 0.2, seed=7))
    per_anchor, reuse, k3 = bench.k4_kernel_bytes(st), bench.kr4_kernel_bytes(st), bench.k3_kernel_bytes(st)
    assert 0 < reuse < per_anchor and k3 > 0
