"""CPU checks of the C ABI: the library loads without a GPU, exports every
entry point declared in include/dig.h, and rejects invalid configurations
before touching a device."""
import ctypes
import os
import re

import pytest

import dig_workloads as wl
from paper_2501_10965_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "dig.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(?:dig_status|void|size_t|const char\*)\s+(\w+)\s*\(", text)))


def test_header_declarations_are_exported():
    lib = L.load()
    names = declared_functions()
    assert set(names) == set(L.EXPORTS), names
    for name in names:
        assert hasattr(lib, name), name
        getattr(lib, name)


def _plan(w, cap=1000):
    cfg = (L.DigConfig * 1)(L.make_config(w))
    lay = L.DigLayout()
    return L.load().dig_plan(cfg, 1, cap, ctypes.byref(lay)), lay


def test_plan_layout_is_aligned_and_disjoint():
    rc, lay = _plan(wl.cavity_2d(n=20), cap=25000)
    assert rc == L.DIG_OK
    offs = []
    for name, _ in L.DigLayout._fields_[3:]:
        v = getattr(lay, name)
        vals = list(v) if hasattr(v, "__len__") else [v]
        offs += vals
    assert all(o % 256 == 0 for o in offs)
    assert len(set(offs)) == len(offs)
    assert lay.total_bytes >= max(offs)


@pytest.mark.parametrize("field,value", [("dim", 3), ("omega", 1.2), ("alpha", 2.5),
                                         ("alpha", 0.9),
                                         ("dr", 7), ("dr", 1), ("kn", 0.0), ("dt", -1.0),
                                         ("zrot", 0.1), ("nx", 0)])
def test_invalid_configs_rejected(field, value):
    w = wl.fourier_1d()
    w[field] = value
    rc, _ = _plan(w)
    assert rc == L.DIG_ERR_INVALID
    assert L.load().dig_last_error()


def test_invalid_boundaries_rejected():
    w = wl.fourier_1d()
    w["bc"] = [("periodic", 1, (0, 0, 0)), ("diffuse", 1, (0, 0, 0))] + w["bc"][2:]
    assert _plan(w)[0] == L.DIG_ERR_INVALID
    w = wl.fourier_1d()
    w["bc"] = [("diffuse", 1, (0.3, 0, 0))] + w["bc"][1:]  # normal wall velocity
    assert _plan(w)[0] == L.DIG_ERR_INVALID
    w = wl.fourier_1d()
    assert _plan(w, cap=0)[0] == L.DIG_ERR_INVALID


def test_null_context_calls_fail_cleanly():
    lib = L.load()
    assert lib.dsmc_step(None, 1, None) == L.DIG_ERR_INVALID
    assert lib.dsmc_query(None, None, None) == L.DIG_ERR_INVALID
    lib.dsmc_destroy(None)
