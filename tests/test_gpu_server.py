"""GPU tests of the continuous-batching server: results identical alone and
in a concurrent mix, admission by footprint, cancellation."""
import threading
import time

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm():
    import torch
    assert torch.cuda.is_available()
    import paper_1203_3415_amd as pm
    pm.lib()
    return pm


def test_server_mix_equals_alone(pm):
    rng = np.random.default_rng(7)
    reqs = []
    for t in range(24):
        k = int(rng.integers(3, 6))
        n = int(rng.integers(50, 600 if k < 5 else 200))
        g = gg.chung_lu(n, int(n * rng.uniform(2, 5)), float(rng.uniform(2.1, 2.6)), 2.4, 0.1, seed=300 + t)
        reqs.append((g, k))
    print("[case] server mix", flush=True)
    with pm.Server(1 << 30, max_inflight=4) as srv:
        tickets = [srv.submit(g.out_off, g.out_idx, g.n, k) for g, k in reqs]
        mixed = [srv.wait(t) for t in tickets]
        alone = []
        for g, k in reqs:
            alone.append(srv.wait(srv.submit(g.out_off, g.out_idx, g.n, k)))
        st = srv.stats()
    for (g, k), a, b in zip(reqs, mixed, alone):
        assert np.array_equal(a, b)
        assert np.array_equal(a, oracle.census(g, k))
    assert st["completed"] == 48 and st["inflight"] == 0


def test_server_admission_and_errors(pm):
    g = gg.chung_lu(40000, 200000, 2.3, 2.3, 0.1, seed=5)
    fp = pm.request_footprint(g.n, g.m, 4)
    assert fp > (4 << 20)
    with pm.Server(max(fp // 2, 1 << 20), max_inflight=2) as srv:
        with pytest.raises(pm.MotifError) as e:
            srv.submit(g.out_off, g.out_idx, g.n, 4)
        assert e.value.name == "ETOOBIG"
    # budget for exactly one request at a time: the peak never exceeds it
    with pm.Server(int(fp * 1.5), max_inflight=4) as srv:
        ts = [srv.submit(g.out_off, g.out_idx, g.n, 4) for _ in range(4)]
        hs = [srv.wait(t) for t in ts]
        st = srv.stats()
    assert st["peak_bytes"] <= int(fp * 1.5)
    off, idx = pm.to_device(g.out_off, g.out_idx)
    want = pm.census(off, idx, g.n, 4)   # the direct (non-server) census of the same graph
    for h in hs:
        assert np.array_equal(h, want)
    # an invalid graph returns its validation error through wait()
    with pm.Server(1 << 28, max_inflight=1) as srv:
        t = srv.submit(np.array([0, 1, 1], np.int32), np.array([0], np.int32), 2, 3)
        with pytest.raises(pm.MotifError) as e:
            srv.wait(t)
        assert e.value.name == "ESELFLOOP"


def test_server_cancel(pm):
    big = gg.chung_lu(20000, 100000, 2.2, 2.2, 0.1, seed=6)
    small = gg.chung_lu(100, 300, 2.3, 2.3, 0.1, seed=7)
    with pm.Server(1 << 31, max_inflight=1) as srv:
        t0 = srv.submit(big.out_off, big.out_idx, big.n, 4)   # occupies the only worker
        t1 = srv.submit(small.out_off, small.out_idx, small.n, 3)
        rc = srv.cancel(t1)
        h0 = srv.wait(t0)
        if rc == 0:
            with pytest.raises(pm.MotifError) as e:
                srv.wait(t1)
            assert e.value.name == "ECANCELED"
        else:
            srv.wait(t1)
    assert h0.sum() > 0


def test_server_second_waiter_is_refused(pm):
    # One waiter per ticket: a second concurrent wait gets EINVAL_ARG instead
    # of racing the first waiter, which frees the request.
    import ctypes
    big = gg.chung_lu(20000, 100000, 2.2, 2.2, 0.1, seed=8)
    print("[case] second waiter", flush=True)
    with pm.Server(1 << 31, max_inflight=1) as srv:
        t0 = srv.submit(big.out_off, big.out_idx, big.n, 4)
        got = {}
        th = threading.Thread(target=lambda: got.setdefault("h", srv.wait(t0)))
        th.start()
        time.sleep(0.2)
        rc = pm.lib().motif_server_wait(srv._h, ctypes.c_uint64(t0), 0)
        th.join()
    assert rc == -13
    assert got["h"].sum() > 0
