"""Pins of the model-deviation oracle (Sec. II.C) against closed forms and invariances (no GPU).

None re-types the oracle's formulas: identical members give zero; two members give half the
difference (|F_1 - F_2| / 2 and |Xi_1 - Xi_2| / (2N), the standard deviation of two values with
weight 1/n_m); four members at -3, -1, 1, 3 times a vector d give sqrt(5)|d|; a shift common to
every member leaves eps unchanged, a common scale scales it; the relative form with a huge nu is
eps / nu; the members' order does not matter; the statistics bracket one another.
"""
import numpy as np
import pytest

from oracle.devi import ensemble, model_deviation
from paper_2304_09409_amd import synth

RNG = np.random.default_rng(4)


def test_identical_members_give_zero():
    f = RNG.normal(size=(50, 3))
    v = RNG.normal(size=(3, 3))
    d = model_deviation([f, f, f, f], [v, v, v, v])
    assert np.abs(d["eps_f"]).max() <= 1e-15 and np.abs(d["eps_v"]).max() <= 1e-15


def test_two_members_half_difference():
    f1, f2 = RNG.normal(size=(40, 3)), RNG.normal(size=(40, 3))
    v1, v2 = RNG.normal(size=(3, 3)), RNG.normal(size=(3, 3))
    d = model_deviation([f1, f2], [v1, v2])
    np.testing.assert_allclose(d["eps_f"], np.linalg.norm(f1 - f2, axis=1) / 2, rtol=1e-14)
    np.testing.assert_allclose(d["eps_v"], np.abs(v1 - v2) / 2 / 40, rtol=1e-14)
    s = d["stats"]
    assert s["f_max"] == d["eps_f"].max() and s["f_min"] == d["eps_f"].min()
    assert s["v_min"] <= s["v_avg"] <= s["v_max"] and s["f_min"] <= s["f_avg"] <= s["f_max"]


def test_four_members_closed_form_and_invariances():
    base = RNG.normal(size=(30, 3))
    dvec = RNG.normal(size=(30, 3))
    fs = [base + a * dvec for a in (-3.0, -1.0, 1.0, 3.0)]
    vs = [np.eye(3) * a for a in (-3.0, -1.0, 1.0, 3.0)]
    d = model_deviation(fs, vs)
    np.testing.assert_allclose(d["eps_f"], np.sqrt(5.0) * np.linalg.norm(dvec, axis=1), rtol=1e-13)
    np.testing.assert_allclose(np.diag(d["eps_v"]), np.sqrt(5.0) / 30, rtol=1e-13)
    # shift common to all members, scale, member order
    shifted = model_deviation([f + 7.0 for f in fs], vs)
    np.testing.assert_allclose(shifted["eps_f"], d["eps_f"], rtol=1e-12)
    scaled = model_deviation([2.5 * f for f in fs], [2.5 * v for v in vs])
    np.testing.assert_allclose(scaled["eps_f"], 2.5 * d["eps_f"], rtol=1e-13)
    np.testing.assert_allclose(scaled["eps_v"], 2.5 * d["eps_v"], rtol=1e-13)
    perm = model_deviation(fs[::-1], vs[::-1])
    np.testing.assert_allclose(perm["eps_f"], d["eps_f"], rtol=1e-13)
    # the relative form: eps / (|<F_i>| + nu), and -> eps / nu for nu >> |F|
    rel = model_deviation(fs, vs, nu=0.5)
    np.testing.assert_allclose(rel["eps_f"], d["eps_f"] / (np.linalg.norm(base, axis=1) + 0.5), rtol=1e-13)
    big = model_deviation(fs, vs, nu=1e12)
    np.testing.assert_allclose(big["eps_f"] * 1e12, d["eps_f"], rtol=1e-9)


def test_ensemble_of_water_models():
    """Four perturbed copies of the water model on the 192-atom box: the per-member forces are the
    oracle's, and a member set equal to member 0 twice over drops the deviation towards zero."""
    from oracle import Oracle
    base = synth.water_params()
    ps = synth.ensemble_params(synth.WATER_MODEL, base, 4)
    c, t, b = synth.water_192()
    d = ensemble([Oracle(synth.WATER_MODEL, p) for p in ps], c, t, b)
    assert d["force"].shape == (4, 192, 3)
    s = d["stats"]
    assert 0.0 < s["f_min"] <= s["f_avg"] <= s["f_max"]
    same = ensemble([Oracle(synth.WATER_MODEL, ps[0])] * 3, c, t, b)
    assert same["stats"]["f_max"] <= 1e-13
