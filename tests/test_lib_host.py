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
