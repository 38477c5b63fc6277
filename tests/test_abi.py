"""CPU-side checks of the C ABI: the library builds for gfx950, loads, exports
every entry point include/pft.h declares, and its host-only logic (contour
plan, argument validation) behaves without touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def pft():
    from paper_1204_5434_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_1204_5434_amd import build
        build.build()
    return binding


def declared_functions():
    text = open(os.path.join(ROOT, "include", "pft.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pft_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(pft):
    lib = pft.load()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(pft.EXPORTS)


@pytest.mark.parametrize("ns,f", [(50, 0.5), (128, 0.3), (100, 0.4), (40, 0.33), (7, 0.05), (9, 0.95),
                                  (200, 0.35), (61, 0.4731)])
def test_contour_plan_matches_oracle(pft, orc, ns, f):
    h, blk, J = pft.pft_contour_plan(ns, f)
    ho, bo, Jo = orc.contour(ns, f)
    assert J == Jo and np.array_equal(blk, bo)
    assert np.array_equal(h, ho)


def test_create_rejects_bad_parameters(pft):
    lib = pft.load()
    h = ctypes.c_void_p()
    bad = [dict(f=0.0), dict(f=1.0), dict(ns=1), dict(lx=0.0), dict(C=-1.0), dict(chiN=0.0),
           dict(precision=7), dict(scheme=3)]
    for kw in bad:
        p = pft.Params(16, 16, 16, 4.0, 4.0, 4.0, 50, 0.5, 15.0)
        for k, v in kw.items():
            setattr(p, k, v)
        assert lib.pft_create(ctypes.byref(p.c()), None, ctypes.byref(h)) == pft.PFT_E_INVALID, kw
        assert not h.value
    for n in (14, 28, 100, 7):
        p = pft.Params(16, 16, n, 4.0, 4.0, 4.0, 50, 0.5, 15.0)
        assert lib.pft_create(ctypes.byref(p.c()), None, ctypes.byref(h)) == pft.PFT_E_UNSUPPORTED
    assert lib.pft_create(None, None, ctypes.byref(h)) == pft.PFT_E_INVALID


def test_null_context_and_plan_errors(pft):
    lib = pft.load()
    assert lib.pft_propagate(None, None, None) == pft.PFT_E_INVALID
    assert lib.pft_densities(None, None, None, None) == pft.PFT_E_INVALID
    assert lib.pft_num_steps(None) == -1
    assert lib.pft_status_string(pft.PFT_E_STATE) == b"PFT_E_STATE"
    h = np.zeros(4)
    b = np.zeros(4, np.int32)
    J = np.zeros(1, np.int32)
    assert lib.pft_contour_plan(1, 0.5, h.ctypes.data, b.ctypes.data, J.ctypes.data) == -1
    assert lib.pft_contour_plan(3, 1.5, h.ctypes.data, b.ctypes.data, J.ctypes.data) == -1
    assert lib.pft_noise_words(0, 0, 0, 0, 0, None, None) == pft.PFT_E_INVALID
