"""The other DeepPot-SE descriptors on the GPU (Sec. II.A.1): se_e2_r (radial-only two-body
embedding, D of M values) and se_e3 (three-body embedding over every ordered pair of kept
neighbours, eq. descrpt-e3 and eq. nn-descrpt-e3), against the FP64 oracle element by element.

Tolerances are the se_e2_a ones (test_gpu_parity.py): FP64 forces within 1e-10 eV/A, energy within
max(1e-9 eV, 1e-12 |E|), virial within max(1e-9 eV N/1000, 1e-12 max|Xi|); mixed and FP32 forces
within 1e-3 eV/A, |dE|/N within max(1e-4 eV, 1e-5 |E|/N), |dXi|/N within 1e-3 eV. Cases: the
192-atom water box, a 700-atom 2-type periodic frame, a 60-atom open cluster, a triclinic cell and
the 12,288-atom water box (many blocks of every kernel); the tabulated nets (se_e3: a table over
theta); owned + ghost atoms; batched frames through the server; model deviation of se_e2_r."""
import sys

import numpy as np
import pytest

from paper_2304_09409_amd import synth

pytestmark = pytest.mark.gpu

SPECS = {"se_e2_r": (synth.WATER_R_MODEL, synth.water_r_params),
         "se_e3": (synth.WATER_E3_MODEL, synth.water_e3_params)}


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


_cache = {}


def model_of(desc):
    from paper_2304_09409_amd import dpk
    key = ("model", desc)
    if key not in _cache:
        spec, params = SPECS[desc]
        _cache[key] = dpk.Model(spec, params())
    return _cache[key]


def oracle_of(desc):
    from oracle import Oracle
    key = ("oracle", desc)
    if key not in _cache:
        spec, params = SPECS[desc]
        _cache[key] = Oracle(spec, params())
    return _cache[key]


def _triclinic():
    c, t, b0 = synth.serving_frame(400, 2, 2)
    b = b0 + np.array([[0, 0, 0], [4.0, 0, 0], [-3.0, 5.0, 0]])
    return (c @ np.linalg.inv(b0)) @ b, t, b


FRAMES = {
    "water192": lambda: synth.water_192(),
    "frame700_2type": lambda: synth.serving_frame(700, 9, 2),
    "open_cluster60": lambda: synth.serving_frame(60, 3, 2)[:2] + (None,),
    "triclinic400": _triclinic,
    "water12288": lambda: synth.water_12288(),
}


def frame_and_ref(desc, case):
    key = ("ref", desc, case)
    if key not in _cache:
        c, t, b = FRAMES[case]()
        _cache[key] = (c, t, b, oracle_of(desc).compute(c, t, b, dumps=len(t) < 1000))
    return _cache[key]


def check_fp64(got, ref, n):
    df = np.abs(got["force"] - ref["force"]).max()
    de = abs(got["energy"] - ref["energy"])
    dv = np.abs(got["virial"] - ref["virial"]).max()
    print(f"  max|dF| {df:.3e}  |dE| {de:.3e}  max|dXi| {dv:.3e}  max|F| {np.abs(ref['force']).max():.3e}", flush=True)
    assert df <= 1e-10
    assert de <= max(1e-9, 1e-12 * abs(ref["energy"]))
    assert dv <= max(1e-9 * max(1.0, n / 1000.0), 1e-12 * np.abs(ref["virial"]).max())


def check_mixed(got, ref, n):
    df = np.abs(got["force"] - ref["force"]).max()
    de = abs(got["energy"] - ref["energy"]) / n
    dv = np.abs(got["virial"] - ref["virial"]).max() / n
    print(f"  max|dF| {df:.3e}  |dE|/N {de:.3e}  max|dXi|/N {dv:.3e}", flush=True)
    assert df <= 1e-3
    assert de <= max(1e-4, 1e-5 * abs(ref["energy"]) / n)
    assert dv <= 1e-3


@pytest.mark.parametrize("case", list(FRAMES))
@pytest.mark.parametrize("desc", list(SPECS))
def test_fp64_matches_oracle(desc, case):
    from paper_2304_09409_amd import dpk
    c, t, b, ref = frame_and_ref(desc, case)
    say(f"{desc} fp64 {case} ({len(t)} atoms)")
    ctx = dpk.Context(model_of(desc), precision="fp64")
    got = ctx.compute(c, t, b, atom_energy=True)
    check_fp64(got, ref, len(t))
    np.testing.assert_allclose(got["atom_energy"], ref["atom_energy"], atol=1e-11)
    if "T" in ref:
        # the descriptor D_m sits in T[m][0] (se_e2_r: the full T = N_c^-1 G^T R, of which the fitting
        # reads column 0; se_e3: the other columns zero), its gradient in dT[m][0] (others zero)
        T, dT = ctx.debug_descriptor(len(t))
        np.testing.assert_allclose(T, ref["T"], atol=1e-13)
        np.testing.assert_allclose(dT, ref["dT"], atol=1e-11 * max(1.0, np.abs(ref["dT"]).max()))
        assert not dT[:, :, 1:].any()
        if desc == "se_e3":
            assert not T[:, :, 1:].any()
    ctx.close()


@pytest.mark.parametrize("precision", ["mixed", "fp32"])
@pytest.mark.parametrize("case", ["water192", "frame700_2type", "open_cluster60", "water12288"])
@pytest.mark.parametrize("desc", list(SPECS))
def test_reduced_precision_matches_oracle(desc, case, precision):
    from paper_2304_09409_amd import dpk
    c, t, b, ref = frame_and_ref(desc, case)
    say(f"{desc} {precision} {case}")
    ctx = dpk.Context(model_of(desc), precision=precision)
    check_mixed(ctx.compute(c, t, b), ref, len(t))
    ctx.close()


@pytest.mark.parametrize("desc", list(SPECS))
def test_bf16_within_its_bound(desc):
    """One BF16 product per embedding GEMM (the fitting net of an M-value descriptor runs in FP32):
    the se_e2_a BF16 bound, every force component within 0.15 eV/A and the RMS error within 2 % of
    RMS(F)."""
    from paper_2304_09409_amd import dpk
    c, t, b, ref = frame_and_ref(desc, "frame700_2type")
    say(f"{desc} bf16 frame700_2type")
    ctx = dpk.Context(model_of(desc), precision="bf16")
    got = ctx.compute(c, t, b)
    d = got["force"] - ref["force"]
    rms, frms = np.sqrt((d ** 2).mean()), np.sqrt((ref["force"] ** 2).mean())
    print(f"  max|dF| {np.abs(d).max():.3e}  rms {rms:.3e}  RMS(F) {frms:.3e}", flush=True)
    assert np.abs(d).max() <= 0.15 and rms <= 0.02 * frms
    ctx.close()


# Table ranges: s = 1/r below r_s = 0.5 A; the closest pair of the frames below is 0.378 A apart
# (the 12,288-atom box), s_max = 2.65, and theta = R_j . R_k = s_j s_k (1 + cos) stays in
# [0, 2 s_max^2] = [0, 14.0].
TABLES = {"se_e2_r": (0.005, 600), "se_e3": (0.01, 1500)}


@pytest.mark.parametrize("precision", ["fp64", "mixed", "fp32"])
@pytest.mark.parametrize("desc", list(SPECS))
def test_tabulated_matches_oracle_table(desc, precision):
    """The compressed model (Sec. II.A.6) against the oracle's evaluation of its own table of the
    same stride and range (se_e3: the table variable is theta)."""
    from paper_2304_09409_amd import dpk
    spec, params = SPECS[desc]
    dx, nint = TABLES[desc]
    o = oracle_of(desc)
    coef = o.table(dx, nint)
    m = dpk.Model(spec, params())
    m.tabulate(dx, dx * nint)
    ctx = dpk.Context(m, precision=precision)
    for case in ("frame700_2type", "water12288"):
        c, t, b = FRAMES[case]()
        say(f"{desc} table {precision} {case}")
        key = ("tabref", desc, case)
        if key not in _cache:
            _cache[key] = o.compute(c, t, b, table=coef, dx=dx)
        ref = _cache[key]
        assert ref["table_oor"] == 0
        got = ctx.compute(c, t, b)
        (check_fp64 if precision == "fp64" else check_mixed)(got, ref, len(t))
        assert ctx.stats()["table_out_of_range"] == 0
    ctx.close()


@pytest.mark.parametrize("desc", list(SPECS))
def test_ghost_bricks_against_oracle(desc):
    """One domain's owned + ghost atoms (Sec. III.B.2): forces on owned and ghost atoms, the
    owned atoms' energies, E and the virial against the oracle on the same brick."""
    from paper_2304_09409_amd import dpk
    c, t, b = synth.water_box(8, 24.85, 5)
    spec = SPECS[desc][0]
    bricks = synth.ghost_bricks(c, t, b, (2, 2, 2), halo=spec["rcut"] + 0.5, seed=1)
    ctx = dpk.Context(model_of(desc), precision="fp64")
    for k, br in enumerate(bricks[:2]):
        say(f"{desc} ghost brick {k}: {br['nlocal']} owned + {len(br['atype']) - br['nlocal']} ghosts")
        ref = oracle_of(desc).compute_ghost(br["coord"], br["atype"], br["nlocal"])
        got = ctx.compute_ghost(br["coord"], br["atype"], br["nlocal"], atom_energy=True)
        df = np.abs(got["force"] - ref["force"]).max()
        print(f"  max|dF| {df:.3e}", flush=True)
        assert df <= 1e-10
        assert abs(got["energy"] - ref["energy"]) <= max(1e-9, 1e-12 * abs(ref["energy"]))
        np.testing.assert_allclose(got["atom_energy"], ref["atom_energy"], atol=1e-11)
        np.testing.assert_allclose(got["virial"], ref["virial"], atol=1e-9 * max(1.0, len(br["atype"]) / 1000))
    ctx.close()


@pytest.mark.parametrize("desc", list(SPECS))
def test_server_batches_match_oracle(desc):
    """Frames of several sizes through the server (batched launches, per-atom virials) in FP64."""
    from paper_2304_09409_amd import dpk
    say(f"{desc} server fp64")
    fr = [synth.serving_frame(n, 40 + i, 2) for i, n in enumerate((80, 300, 57, 500))]
    srv = dpk.Server(model_of(desc), precision="fp64", nslots=2)
    tickets = [srv.submit(c, t, b) for c, t, b in fr]
    for (c, t, b), tk in zip(fr, tickets):
        ref = oracle_of(desc).compute(c, t, b)
        got = tk.result()
        assert np.abs(got["force"] - ref["force"]).max() <= 1e-10
        assert abs(got["energy"] - ref["energy"]) <= max(1e-9, 1e-12 * abs(ref["energy"]))
        assert np.abs(got["virial"] - ref["virial"]).max() <= 1e-9
    srv.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_se_e2_r_deviation(precision):
    """Model deviation (Sec. II.C) of an se_e2_r ensemble: members and eps_F against the oracle."""
    from oracle import Oracle
    from oracle.devi import ensemble
    from paper_2304_09409_amd import dpk
    spec, params = SPECS["se_e2_r"]
    ps = synth.ensemble_params(spec, params(), 3)
    c, t, b = synth.serving_frame(700, 9, 2)
    say(f"se_e2_r devi {precision}")
    ref = ensemble([Oracle(spec, p) for p in ps], c, t, b)
    dv = dpk.Deviation([dpk.Model(spec, p) for p in ps], precision=precision)
    got = dv.compute(c, t, b)
    tol = 1e-10 if precision == "fp64" else 1e-3
    assert np.abs(got["force"] - ref["force"]).max() <= tol
    assert np.abs(got["eps_f"] - ref["eps_f"]).max() <= tol
    dv.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_se_e3_deviation(precision):
    """Model deviation (Sec. II.C) of an se_e3 ensemble (the pair walk on the ensemble axis): every
    member's forces and eps_F against the oracle's members."""
    from oracle import Oracle
    from oracle.devi import ensemble
    from paper_2304_09409_amd import dpk
    spec, params = SPECS["se_e3"]
    ps = synth.ensemble_params(spec, params(), 3)
    c, t, b = synth.serving_frame(700, 9, 2)
    say(f"se_e3 devi {precision}")
    ref = ensemble([Oracle(spec, p) for p in ps], c, t, b)
    dv = dpk.Deviation([dpk.Model(spec, p) for p in ps], precision=precision)
    got = dv.compute(c, t, b)
    tol = 1e-10 if precision == "fp64" else 1e-3
    df = np.abs(got["force"] - ref["force"]).max()
    de = np.abs(got["eps_f"] - ref["eps_f"]).max()
    print(f"  max|dF| {df:.3e}  max|d eps_F| {de:.3e}", flush=True)
    assert df <= tol
    assert de <= tol
    dv.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_se_e3_one_and_three_types(precision):
    """se_e3 with one species (every pair in one type block: the k <= j walk throughout) on a
    truncated fcc box, and with three species (nine nets, three same-type blocks) on a 3-type frame."""
    from oracle import Oracle
    from paper_2304_09409_amd import dpk
    cases = [
        (dict(synth.WATER_E3_MODEL, ntypes=1, sel=[40]), synth.fcc_box(4, 3.6, 2)),
        (dict(synth.WATER_E3_MODEL, ntypes=3, sel=[20, 20, 14]), synth.serving_frame(400, 23, 3)),
    ]
    for spec, (c, t, b) in cases:
        say(f"se_e3 {spec['ntypes']} types {precision} ({len(t)} atoms)")
        p = synth.make_params(spec, 17, synth.WATER_E3_OUT_SCALE, synth.WATER_E3_FIT_IN)
        ref = Oracle(spec, p).compute(c, t, b)
        ctx = dpk.Context(dpk.Model(spec, p), precision=precision)
        got = ctx.compute(c, t, b)
        (check_fp64 if precision == "fp64" else check_mixed)(got, ref, len(t))
        assert ctx.stats()["nbr_dropped"] == ref["ndrop"]
        ctx.close()
