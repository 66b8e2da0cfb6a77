"""Pins of the oracle's other DeepPot-SE descriptors (no GPU): the radial-only two-body embedding
(se_e2_r) and the three-body embedding (se_e3, eq. descrpt-e3 and eq. nn-descrpt-e3).

Closed forms where the descriptor reduces to a few terms (checked against numpy written here from
the definitions, with the switching function and nets taken from the oracle's pinned pieces):
  * dimer, se_e2_r: one neighbour, D_m = N_c^-1 s G_m(s);
  * dimer, se_e3: one neighbour, the pair (j, j) only: theta = |R_j|^2 = 2 s^2,
    D_m = N_c^-2 theta G_m^{(a_j, a_j)}(theta);
  * trimer, se_e3: two neighbours j, k of different types: four ordered pairs, each with its own net
    (a_j, a_k) and theta = R_j . R_k;
then F = -dE/dr by central differences, invariances, zero net force and torque and the open
cluster's virial, and the tabulated se_e3 (table over theta) against the network and against its
own finite differences.
"""
import numpy as np
import pytest

from oracle import Oracle
from paper_2304_09409_amd import synth

RNG = np.random.default_rng(71)


@pytest.fixture(scope="module")
def rmodel():
    return Oracle(synth.WATER_R_MODEL, synth.water_r_params())


@pytest.fixture(scope="module")
def e3model():
    return Oracle(synth.WATER_E3_MODEL, synth.water_e3_params())


def _rvec(o, v):
    r = np.linalg.norm(v)
    s = o.switch(r)[0]
    return np.concatenate([[s], s * v / r])


@pytest.mark.parametrize("r", [0.45, 1.2, 3.3, 5.6])
def test_se_e2_r_dimer(rmodel, r):
    o = rmodel
    c = np.array([[0.0, 0.0, 0.0], [r * 0.36, r * 0.48, r * 0.8]])
    t = np.array([0, 1], dtype=np.int32)
    out = o.compute(c, t, None)
    s = o.switch(r)[0]
    for i, (ti, tj) in enumerate([(0, 1), (1, 0)]):
        G = o.embed(ti * 2 + tj, s)[0]
        e_ref = o.fit(ti, s * G / o.nc)[0]
        assert out["atom_energy"][i] == pytest.approx(e_ref, rel=1e-13, abs=1e-13)


@pytest.mark.parametrize("r", [0.45, 1.2, 3.3])
def test_se_e3_dimer(e3model, r):
    o = e3model
    c = np.array([[0.0, 0.0, 0.0], [r * 0.36, r * 0.48, r * 0.8]])
    t = np.array([0, 1], dtype=np.int32)
    out = o.compute(c, t, None)
    s = o.switch(r)[0]
    theta = 2.0 * s * s
    for i, tj in enumerate([1, 0]):
        G = o.embed(tj * 2 + tj, theta)[0]
        e_ref = o.fit(t[i], theta * G / o.nc ** 2)[0]
        assert out["atom_energy"][i] == pytest.approx(e_ref, rel=1e-13, abs=1e-13)


def test_se_e3_trimer_pair_sum(e3model):
    o = e3model
    c = np.array([[0.0, 0.0, 0.0], [1.1, 0.3, -0.2], [-0.4, 1.5, 0.7]])
    t = np.array([0, 0, 1], dtype=np.int32)
    out = o.compute(c, t, None)
    for i in range(3):
        nb = [j for j in range(3) if j != i]
        R = {j: _rvec(o, c[j] - c[i]) for j in nb}
        D = np.zeros(o.M)
        for a in nb:
            for b in nb:
                th = R[a] @ R[b]
                D += th * o.embed(t[a] * 2 + t[b], th)[0]
        e_ref = o.fit(t[i], D / o.nc ** 2)[0]
        assert out["atom_energy"][i] == pytest.approx(e_ref, rel=1e-12, abs=1e-12)


def _fd(o, c, t, box, atom, comp, h=1e-4, **kw):
    def e(delta):
        cc = c.copy()
        cc[atom, comp] += delta
        return o.energy(cc, t, box, **kw)
    return -(8 * (e(h) - e(-h)) - (e(2 * h) - e(-2 * h))) / (12 * h)


@pytest.mark.parametrize("which", ["r", "e3"])
def test_forces_match_fd(rmodel, e3model, which):
    o = rmodel if which == "r" else e3model
    c, t, b = synth.serving_frame(60, 13, 2)      # L = 8.4 A: several images within r_c
    f = o.compute(c, t, b)["force"]
    for atom in RNG.choice(len(t), 3, replace=False):
        for comp in range(3):
            assert f[atom, comp] == pytest.approx(_fd(o, c, t, b, atom, comp), abs=2e-7)


@pytest.mark.parametrize("which", ["r", "e3"])
def test_invariances_and_cluster_virial(rmodel, e3model, which):
    o = rmodel if which == "r" else e3model
    c, t = synth.serving_frame(50, 3, 2)[:2]
    a = o.compute(c, t, None)
    np.testing.assert_allclose(a["force"].sum(0), 0.0, atol=1e-11)
    np.testing.assert_allclose(np.cross(c, a["force"]).sum(0), 0.0, atol=1e-10)
    np.testing.assert_allclose(a["virial"], np.einsum("ka,kb->ab", a["force"], c), atol=1e-10)
    q = np.linalg.qr(RNG.normal(size=(3, 3)))[0]
    z = o.compute(c @ q.T + 3.0, t, None)
    assert z["energy"] == pytest.approx(a["energy"], rel=1e-12)
    np.testing.assert_allclose(z["force"], a["force"] @ q.T, atol=1e-10)
    perm = RNG.permutation(len(t))
    w = o.compute(c[perm], t[perm], None)
    assert w["energy"] == pytest.approx(a["energy"], rel=1e-12)
    np.testing.assert_allclose(w["force"], a["force"][perm], atol=1e-11)


def test_se_e3_table(e3model):
    """Tabulated three-body embedding (Sec. II.A.6: the e3 nets have a scalar input too): a table
    over theta in [0, 2 / r_s^2] with stride 0.01, close to the network, and its forces the
    negative gradient of its own energy."""
    o = e3model
    dx, nint = 0.01, 800
    coef = o.table(dx, nint)
    c, t, b = synth.serving_frame(60, 13, 2)
    tab = o.compute(c, t, b, table=coef, dx=dx)
    net = o.compute(c, t, b)
    assert tab["table_oor"] == 0
    assert abs(tab["energy"] - net["energy"]) / len(t) < 1e-7
    assert np.abs(tab["force"] - net["force"]).max() < 1e-5
    for atom in (3, 40):
        for comp in range(3):
            fd = _fd(o, c, t, b, atom, comp, table=coef, dx=dx)
            assert tab["force"][atom, comp] == pytest.approx(fd, abs=2e-7)
