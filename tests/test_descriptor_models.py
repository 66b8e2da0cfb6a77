"""Host-side checks of the descriptor kinds (no GPU): the library, the parameter generator and the
oracle count the same parameters for se_e2_a, se_e2_r and se_e3 (se_e3: a net per ordered pair of
neighbour types whatever type_one_side says; fitting input M for the M-value descriptors), and
dpk_model_create refuses an unknown kind and an se_e3 model past the three-body kernels' N_c."""
import numpy as np
import pytest

from paper_2304_09409_amd import dpk, synth


@pytest.mark.parametrize("spec", [synth.WATER_MODEL, synth.WATER_R_MODEL, synth.WATER_E3_MODEL,
                                  dict(synth.WATER_E3_MODEL, type_one_side=True),
                                  dict(synth.WATER_R_MODEL, type_one_side=True, ntypes=3, sel=[20, 40, 30])])
def test_param_counts_agree(spec):
    from oracle import Oracle
    n = synth.param_count(spec)
    assert dpk.param_count(spec) == n
    Oracle(spec, np.zeros(n))   # the oracle checks the blob size against its own count
    nt, e = spec["ntypes"], [1, 25, 50, 100]
    desc = spec.get("descriptor", "se_e2_a")
    nets = nt if spec["type_one_side"] and desc != "se_e3" else nt * nt
    width = 1600 if desc == "se_e2_a" else 100
    f = [width, 240, 240, 240, 1]
    expect = nets * sum(e[k] * e[k + 1] + 2 * e[k + 1] for k in range(3)) + \
        nt * sum(f[k] * f[k + 1] + 2 * f[k + 1] for k in range(4))
    assert n == expect


def test_unknown_descriptor_is_refused():
    import ctypes as C
    spec = synth.WATER_MODEL
    p = synth.water_params()
    d = dpk.make_desc(spec)
    d.descriptor = 3
    h = C.c_void_p()
    rc = dpk.lib().dpk_model_create(C.byref(d), p.ctypes.data_as(C.POINTER(C.c_double)), p.size, C.byref(h))
    assert rc == dpk.DPK_E_INVALID_ARG and not h.value
    with pytest.raises(KeyError):
        dpk.make_desc(dict(spec, descriptor="se_atten"))


def test_se_e3_capacity_limit():
    spec = dict(synth.WATER_E3_MODEL, sel=[60, 80])
    p = np.zeros(synth.param_count(spec))
    with pytest.raises(dpk.DpkError) as e:
        dpk.Model(spec, p)
    assert e.value.code == dpk.DPK_E_UNIMPLEMENTED
