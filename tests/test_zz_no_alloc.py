"""GPU test of the allocation-free census entry point, through the C ABI.

motif_census_noalloc() must return exactly what motif_census() returns, on
two calls in a row with the second input smaller than the first (the shared
workspace keeps the first call's contents), for k = 3, 4, 5; a graph whose
workspace cannot fit must be refused before any work starts."""
import ctypes

import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm():
    import torch
    assert torch.cuda.is_available()
    import paper_1203_3415_amd as pm
    assert pm.lib().motif_init() == 0
    return pm


def _call(pm, fn, g, k):
    import torch
    off, idx = pm.to_device(g.out_off, g.out_idx)
    hist = torch.full((pm.NUM_CLASSES[k],), 3, dtype=torch.int64, device="cuda")
    s = torch.cuda.current_stream()
    rc = fn(ctypes.c_void_p(off.data_ptr()), ctypes.c_void_p(idx.data_ptr() if idx.numel() else 0), None, None,
            g.n, g.m, k, ctypes.c_void_p(hist.data_ptr()), ctypes.c_void_p(s.cuda_stream))
    torch.cuda.synchronize()
    return rc, hist.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("k", [3, 4, 5])
def test_noalloc_matches_census_twice(pm, k):
    L = pm.lib()
    big = gg.chung_lu(3000 if k < 5 else 1500, 15000 if k < 5 else 6000, 2.2, 2.4, 0.15, seed=60 + k)
    small = gg.chung_lu(400, 1600, 2.3, 2.3, 0.1, seed=70 + k)
    for label, g in (("first", big), ("second, smaller", small)):
        print(f"[case] noalloc k={k} {label} n={g.n} m={g.m}", flush=True)
        rc0, want = _call(pm, L.motif_census, g, k)
        rc1, got = _call(pm, L.motif_census_noalloc, g, k)
        assert rc0 == 0 and rc1 == 0, (rc0, rc1)
        assert np.array_equal(got, want)


def test_noalloc_bench_graph_k3_and_refusals(pm):
    L = pm.lib()
    g = gg.chung_lu(100_000, 1_000_000, 2.1, 2.1, 0.2, seed=2)
    print("[case] noalloc k=3 on the n=1e5 m=1e6 graph", flush=True)
    rc0, want = _call(pm, L.motif_census, g, 3)
    rc1, got = _call(pm, L.motif_census_noalloc, g, 3)
    assert rc0 == 0 and rc1 == 0 and np.array_equal(got, want)
    # invalid input: its validation code, histogram untouched
    bad = gg.from_arcs(3, [(0, 1)])
    off, idx = pm.to_device(np.array([0, 1, 2, 2], np.int32), np.array([1, 1], np.int32))
    import torch
    hist = torch.full((13,), 3, dtype=torch.int64, device="cuda")
    rc = L.motif_census_noalloc(ctypes.c_void_p(off.data_ptr()), ctypes.c_void_p(idx.data_ptr()), None, None,
                                3, 2, 3, ctypes.c_void_p(hist.data_ptr()), None)
    torch.cuda.synchronize()
    assert rc == -4 and bool((hist == 3).all()) and bad.m == 1   # MOTIF_ESELFLOOP
    # a workspace beyond the fixed array is refused before anything runs
    # (shape only: the pointers are never read)
    rc = L.motif_census_noalloc(ctypes.c_void_p(off.data_ptr()), ctypes.c_void_p(idx.data_ptr()), None, None,
                                (1 << 30) - 1, (1 << 30) - 1, 4, ctypes.c_void_p(hist.data_ptr()), None)
    assert rc == -10   # MOTIF_ETOOBIG
