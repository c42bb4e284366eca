"""The C-ABI library loads without a GPU and exports every entry point that
include/rzpic.h declares; host-only entry points agree with the oracle."""
import os
import re

import pytest

from paper_1001_2969_amd import rzpic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rzpic.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rzpic_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(rzpic.LIB_PATH):
        from paper_1001_2969_amd import build
        build.build()
    return rzpic.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(rzpic.EXPORTS)


def test_constants_agree_with_oracle(lib):
    from oracle import rzo
    a, b = rzpic.constants(), rzo.constants()
    assert a == b


def test_create_rejects_bad_configs_without_touching_the_gpu(lib):
    import ctypes as C
    base = dict(nr=33, nz=33, R=0.02, L=0.02, dt=5e-11, precision=0, weighting=0, chi_face=0,
                fixed_point_bits=0, V_dc=0, V_rf=0, f_rf=0, seed=0, mg_tol=1e-10,
                mg_max_cycles=50, mg_fixed_cycles=0, resize_every=0, sort_every=0,
                resize_wcoef=0, n_gas=1e21, T_gas=300, m_gas=6.6e-26, tile_z=0, tile_r=0)
    for bad in ({"nz": 34}, {"nr": 2}, {"R": 0.0}, {"precision": 7}, {"weighting": 3},
                {"mg_tol": 0.0}, {"fixed_point_bits": 60}, {"resize_every": 5},
                {"sort_every": -1}, {"tile_z": -2},
                {"nr": 2049, "nz": 2049, "tile_z": 1, "tile_r": 1, "sort_every": 1}):
        cfg = rzpic.Config(**{**base, **bad})
        h = C.c_void_p()
        code = lib.rzpic_create(C.byref(cfg), None, C.byref(h))
        assert code == 1, bad  # RZPIC_EINVAL, decided before any device call
        assert not h.value
        assert lib.rzpic_last_error()
