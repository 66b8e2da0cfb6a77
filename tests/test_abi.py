"""The C-ABI library loads and exports every symbol include/dpk.h declares (CPU only: no compute)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2304_09409_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "dpk.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dpk_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_2304_09409_amd import dpk
    if not os.path.exists(dpk.LIB_PATH):
        pytest.fail("libdpk.so is not built (run `python -m paper_2304_09409_amd.build`)")
    return dpk


def test_every_declared_symbol_is_exported(lib):
    L = lib.lib()
    names = _declared()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name
        assert isinstance(getattr(L, name), ctypes._CFuncPtr)


@pytest.mark.parametrize("spec", [synth.WATER_MODEL, synth.FCC_MODEL, synth.SERVE_MODEL])
def test_param_count_matches_generator(lib, spec):
    assert lib.param_count(spec) == synth.param_count(spec)


def test_model_create_validates(lib):
    p = synth.water_params()
    m = lib.Model(synth.WATER_MODEL, p)          # host-only call
    assert m.nc == 138
    with pytest.raises(lib.DpkError) as e:
        lib.Model(synth.WATER_MODEL, p[:-1])
    assert e.value.code == lib.DPK_E_INVALID_ARG
    bad = dict(synth.WATER_MODEL, emb=[16, 32, 64])
    with pytest.raises(lib.DpkError) as e:
        lib.Model(bad, np.zeros(synth.param_count(bad)))
    assert e.value.code == lib.DPK_E_UNIMPLEMENTED
    bad = dict(synth.WATER_MODEL, rcut_smth=7.0)
    with pytest.raises(lib.DpkError) as e:
        lib.Model(bad, p)
    assert e.value.code == lib.DPK_E_INVALID_ARG


def test_tabulate_validates(lib):
    m = lib.Model(synth.FCC_MODEL, synth.fcc_params())
    with pytest.raises(lib.DpkError):
        m.tabulate(0.0, 0.5)
    m.tabulate(0.01, 0.5)   # host-side table build succeeds
