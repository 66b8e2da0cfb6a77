"""Host-side pieces of the training path (no GPU): the learning-rate schedule of eq. learning_rate
and the prefactor schedule, from the library, against the training oracle's closed forms; and the
trainer refusing the descriptor kinds it does not cover before touching a device."""
import numpy as np
import pytest

from paper_2304_09409_amd import dpk, synth


@pytest.mark.parametrize("step", [0, 1, 4999, 5000, 12345, 99999, 100000, 250000])
def test_learning_rate_matches_oracle(step):
    from oracle.train import learning_rate
    got = dpk.learning_rate(1e-3, 3.51e-8, step, 100000, 5000)
    assert got == pytest.approx(learning_rate(1e-3, 3.51e-8, step, 100000, 5000), rel=1e-13)


@pytest.mark.parametrize("lr", [1e-3, 5e-4, 1e-6, 0.0])
def test_prefactor_matches_oracle(lr):
    from oracle.train import prefactor
    for ps, pl in ((0.02, 1.0), (1000.0, 1.0), (0.0, 0.0)):
        assert dpk.loss_prefactor(ps, pl, lr, 1e-3) == pytest.approx(prefactor(ps, pl, lr, 1e-3), rel=1e-14, abs=1e-300)


def test_trainer_refuses_other_descriptors():
    m = dpk.Model(synth.WATER_R_MODEL, synth.water_r_params())
    with pytest.raises(dpk.DpkError) as e:
        dpk.Trainer(m)
    assert e.value.code == dpk.DPK_E_UNIMPLEMENTED
