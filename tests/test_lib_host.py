"""Host-side checks of the HIP library (no GPU needed): every symbol the
header declares is exported, and the host class tables agree with the oracle's
brute-force tables."""
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1203_3415_amd", "libmotif.so")


def _declared():
    text = open(os.path.join(ROOT, "include", "motif.h")).read()
    return sorted(set(re.findall(r"\b(motif_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libmotif.so not built")
    import paper_1203_3415_amd as pm
    return pm


def test_exports_every_declared_symbol(lib):
    import ctypes
    L = ctypes.CDLL(LIB)
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


@pytest.mark.parametrize("k", [3, 4, 5])
def test_class_tables_match_oracle(lib, k):
    cls, canon, _, _ = oracle.class_table(k)
    C = len(canon)
    assert lib.num_classes(k) == C
    for c in range(C):
        assert lib.class_code(k, c) == int(canon[c])
    step = 1 if k < 5 else 97
    for code in range(0, 1 << (k * (k - 1)), step):
        want = int(cls[code])
        assert lib.class_of_code(k, code) == (-1 if want == 0xFFFF else want)


@pytest.mark.parametrize("k", [3, 4, 5])
def test_multiplicities_match_oracle(lib, k):
    _, canon, _, _ = oracle.class_table(k)
    for c in range(len(canon)):
        assert lib.class_multiplicity(k, c) == oracle.multiplicity(k, int(canon[c]))


def test_host_argument_errors(lib):
    with pytest.raises(lib.MotifError) as e:
        lib.class_code(6, 0)
    assert e.value.name == "EINVAL_K"
    assert lib.num_classes(2) == -1
    with pytest.raises(lib.MotifError):
        lib.class_multiplicity(4, 199)


def test_shape_limit_is_checked_on_the_host(lib):
    # n and m below 2^30: the typed G* rows keep a vertex id and its two type
    # bits in one 32-bit word, and the 2m half-edges use int32 offsets.  The
    # check runs before any device call, so it holds without a GPU.
    import ctypes
    L = lib.lib()
    hist = ctypes.c_void_p(8)
    for n, m in ((1 << 30, 0), (10, 1 << 30), (-1, 0), (0, -1)):
        assert L.motif_census(None, None, None, None, n, m, 4, hist, None) == -2
        assert L.motif_census_async(None, None, None, None, n, m, 4, hist, hist, None) == -2
    assert L.motif_census(None, None, None, None, 10, 0, 6, hist, None) == -1
    # the largest accepted shape gets past the shape check (to the pointer check)
    assert L.motif_census(None, None, None, None, (1 << 30) - 1, (1 << 30) - 1, 3, hist, None) == -13


def test_tuning_fields_are_validated(lib):
    saved = lib.get_tuning(4)
    try:
        for bad in (dict(solo_deg=65), dict(light_deg=257), dict(light5=768), dict(block=300), dict(tile=5000)):
            k = 5 if "light5" in bad else 4
            with pytest.raises(lib.MotifError) as e:
                lib.set_tuning(k, **bad)
            assert e.value.name == "EINVAL_ARG"
        lib.set_tuning(4, solo_deg=32, light_deg=128)
        t = lib.get_tuning(4)
        assert (t["solo_deg"], t["light_deg"]) == (32, 128)
        assert t["block"] == saved["block"]   # 0 fields keep their value
    finally:
        lib.set_tuning(4, **saved)
    assert lib.get_tuning(4) == saved
