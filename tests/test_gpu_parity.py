"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle, element by element.

Tolerances (written here, from the target of the method's mixed-precision study):
  * FP64 mode: every force component within 1e-10 eV/A of the oracle; energy within
    max(1e-9 eV, 1e-12 |E|), virial within max(1e-9 eV N/1000, 1e-12 max|Xi|) (FP64 sums of N n_bar
    terms, resolved relative to their size); the neighbour list identical.
  * mixed mode (split-BF16 GEMMs, FP32 activations): every force component within 1e-3 eV/A;
    |dE|/N within max(1e-4 eV, 1e-5 |E|/N) (the per-atom energies carry an offset of up to 190 eV
    in the fcc model, resolved to FP32 precision); |dXi|/N within 1e-3 eV.
  * FP32 mode (FP32 MFMA GEMMs, FP32 activations and table; FP64 geometry and sums): the mixed
    mode's bounds.
  * BF16 mode: its own bound (test_bf16_within_its_bound).
"""
import sys

import numpy as np
import pytest

from paper_2304_09409_amd import synth

pytestmark = pytest.mark.gpu

F64_FORCE_TOL = 1e-10
MIX_FORCE_TOL = 1e-3


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dpk():
    from paper_2304_09409_amd import dpk as mod
    return mod


_models = {}


def model_of(dpk, name):
    if name not in _models:
        spec, params = {"water": (synth.WATER_MODEL, synth.water_params),
                        "serve": (synth.SERVE_MODEL, synth.serve_params),
                        "fcc": (synth.FCC_MODEL, synth.fcc_params)}[name]
        _models[name] = (spec, params(), dpk.Model(spec, params()))
    return _models[name]


_oracles = {}


def oracle_of(name):
    from oracle import Oracle
    if name not in _oracles:
        spec, params = {"water": (synth.WATER_MODEL, synth.water_params),
                        "serve": (synth.SERVE_MODEL, synth.serve_params),
                        "fcc": (synth.FCC_MODEL, synth.fcc_params)}[name]
        _oracles[name] = Oracle(spec, params())
    return _oracles[name]


def check_fp64(got, ref, n):
    df = np.abs(got["force"] - ref["force"]).max()
    de = abs(got["energy"] - ref["energy"])
    dv = np.abs(got["virial"] - ref["virial"]).max()
    print(f"  max|dF| {df:.3e}  |dE| {de:.3e}  max|dXi| {dv:.3e}", flush=True)
    assert df <= F64_FORCE_TOL
    assert de <= max(1e-9, 1e-12 * abs(ref["energy"]))
    # an FP64 sum over N n_bar pair terms is resolved relative to its own size, like the energy
    assert dv <= max(1e-9 * max(1.0, n / 1000.0), 1e-12 * np.abs(ref["virial"]).max())


def check_mixed(got, ref, n):
    df = np.abs(got["force"] - ref["force"]).max()
    de = abs(got["energy"] - ref["energy"]) / n
    dv = np.abs(got["virial"] - ref["virial"]).max() / n
    rms = np.sqrt(((got["force"] - ref["force"]) ** 2).mean())
    print(f"  max|dF| {df:.3e}  rms|dF| {rms:.3e}  |dE|/N {de:.3e}  max|dXi|/N {dv:.3e}", flush=True)
    assert df <= MIX_FORCE_TOL
    assert de <= max(1e-4, 1e-5 * abs(ref["energy"]) / n)
    assert dv <= 1e-3


FRAMES = {
    "water192": ("water", lambda: synth.water_192()),
    "serve50_3type_small_cell": ("serve", lambda: synth.serving_frame(50, 7, 3)),
    "serve700_2type": ("serve", lambda: synth.serving_frame(700, 9, 2)),
    "open_cluster60": ("water", lambda: synth.serving_frame(60, 3, 2)[:2] + (None,)),
    "triclinic400": ("serve", lambda: _triclinic()),
    "fcc500_truncated": ("fcc", lambda: synth.fcc_box(5, 3.6, 1)),
    "lattice512_ties": ("water", lambda: synth.tie_lattice()),
    # more than 8,192 atoms: the multi-block preparation, here with open-boundary bins
    "open_cluster9000": ("water", lambda: synth.serving_frame(9000, 5, 2)[:2] + (None,)),
}


def _triclinic():
    c, t, b0 = synth.serving_frame(400, 2, 3)
    b = b0 + np.array([[0, 0, 0], [4.0, 0, 0], [-3.0, 5.0, 0]])
    return (c @ np.linalg.inv(b0)) @ b, t, b


@pytest.mark.parametrize("case", list(FRAMES))
def test_fp64_matches_oracle(dpk, case):
    say(f"fp64 {case}")
    mname, make = FRAMES[case]
    c, t, b = make()
    spec, params, model = model_of(dpk, mname)
    ref = oracle_of(mname).compute(c, t, b, dumps=True)
    ctx = dpk.Context(model, precision="fp64")
    got = ctx.compute(c, t, b, atom_energy=True)
    check_fp64(got, ref, len(t))
    np.testing.assert_allclose(got["atom_energy"], ref["atom_energy"], atol=1e-11)
    nl = ctx.debug_nlist(len(t))
    np.testing.assert_array_equal(nl, ref["nlist"])
    T, dT = ctx.debug_descriptor(len(t))
    np.testing.assert_allclose(T, ref["T"], atol=1e-13)
    np.testing.assert_allclose(dT, ref["dT"], atol=1e-11 * max(1.0, np.abs(ref["dT"]).max()))
    st = ctx.stats()
    assert st["nbr_dropped"] == ref["ndrop"]
    ctx.close()


@pytest.mark.parametrize("precision", ["mixed", "fp32"])
@pytest.mark.parametrize("case", list(FRAMES))
def test_reduced_precision_matches_oracle(dpk, case, precision):
    say(f"{precision} {case}")
    mname, make = FRAMES[case]
    c, t, b = make()
    spec, params, model = model_of(dpk, mname)
    ref = oracle_of(mname).compute(c, t, b)
    ctx = dpk.Context(model, precision=precision)
    got = ctx.compute(c, t, b)
    check_mixed(got, ref, len(t))
    ctx.close()


@pytest.mark.parametrize("case", ["water192", "serve700_2type"])
def test_bf16_within_its_bound(dpk, case):
    """One BF16 product per GEMM: each operand keeps 8 significant bits (relative rounding 2^-9),
    so the network's outputs carry errors of order 1e-2 relative. Bound, from a numpy emulation of
    BF16 operands on the 192-atom box (max 4e-2 eV/A at RMS(F) about 1 eV/A): every force
    component within 0.15 eV/A and the RMS error within 2 % of RMS(F)."""
    say(f"bf16 {case}")
    mname, make = FRAMES[case]
    c, t, b = make()
    spec, params, model = model_of(dpk, mname)
    ref = oracle_of(mname).compute(c, t, b)
    ctx = dpk.Context(model, precision="bf16")
    got = ctx.compute(c, t, b)
    d = got["force"] - ref["force"]
    df = np.abs(d).max()
    rms, frms = np.sqrt((d ** 2).mean()), np.sqrt((ref["force"] ** 2).mean())
    print(f"  bf16 max|dF| {df:.3e}  rms|dF| {rms:.3e}  RMS(F) {frms:.3e}", flush=True)
    assert np.isfinite(got["force"]).all()
    assert df <= 0.15
    assert rms <= 0.02 * frms
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed", "fp32"])
def test_type_one_side_matches_oracle(dpk, precision):
    """Per-species embedding nets indexed by the neighbour's type only (type_one_side, Sec.
    II.A.1), with non-unit timestep vectors, on a 3-type frame and a triclinic one."""
    spec = dict(synth.SERVE_MODEL, type_one_side=True)
    params = synth.make_params(spec, 31, synth.SERVE_OUT_SCALE, synth.SERVE_FIT_IN, timestep_sigma=0.2)
    from oracle import Oracle
    o = Oracle(spec, params)
    model = dpk.Model(spec, params)
    ctx = dpk.Context(model, precision=precision)
    for name, (c, t, b) in (("serve700_3type", synth.serving_frame(700, 19, 3)), ("triclinic400", _triclinic())):
        say(f"type_one_side {precision} {name}")
        ref = o.compute(c, t, b)
        got = ctx.compute(c, t, b)
        (check_fp64 if precision == "fp64" else check_mixed)(got, ref, len(t))
    ctx.close()


def _fcc_with_close_pairs():
    """fcc 500-atom box with three atoms pushed towards a neighbour, to 1.55-1.9 A: inside r_s = 2 A,
    where s = 1/r > 0.5 lies past the table's range [0, 0.5]."""
    c, t, b = synth.fcc_box(5, 3.6, 1)
    c = c.copy()
    for i, r in ((0, 1.55), (100, 1.75), (333, 1.9)):
        d = c[i] - c[:, :]
        d -= np.round(d / b[0, 0]) * b[0, 0]
        dist = np.linalg.norm(d, axis=1)
        dist[i] = 1e9
        j = int(np.argmin(dist))
        u = (c[j] - c[i]) - np.round((c[j] - c[i]) / b[0, 0]) * b[0, 0]
        u /= np.linalg.norm(u)
        c[j] = c[i] + r * u
    return c, t, b


@pytest.mark.parametrize("precision", ["fp64", "mixed", "fp32"])
def test_table_out_of_range_inputs(dpk, precision):
    """Table inputs past its range use the last piece extrapolated (reading R9) and are counted:
    forces against the oracle's evaluation of the same table and the same count."""
    say(f"table out of range {precision}")
    spec, params = synth.FCC_MODEL, synth.fcc_params()
    model = dpk.Model(spec, params).tabulate(0.01, 0.5)
    o = oracle_of("fcc")
    c, t, b = _fcc_with_close_pairs()
    ref = o.compute(c, t, b, table=o.table(0.01, 50), dx=0.01)
    assert ref["table_oor"] >= 6
    ctx = dpk.Context(model, precision=precision)
    got = ctx.compute(c, t, b)
    (check_fp64 if precision == "fp64" else check_mixed)(got, ref, len(t))
    assert ctx.stats()["table_out_of_range"] == ref["table_oor"]
    ctx.close()


def test_fp64_full_water_12288(dpk):
    """The 12,288-atom water box in the launch configuration the benchmark times."""
    say("fp64 water12288")
    c, t, b = synth.water_12288()
    spec, params, model = model_of(dpk, "water")
    ref = oracle_of("water").compute(c, t, b)
    ctx = dpk.Context(model, precision="fp64")
    check_fp64(ctx.compute(c, t, b), ref, len(t))
    for prec in ("mixed", "fp32"):
        say(f"{prec} water12288")
        ctx2 = dpk.Context(model, precision=prec)
        check_mixed(ctx2.compute(c, t, b), ref, len(t))
        ctx2.close()
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed", "fp32"])
def test_tabulated_matches_oracle_table(dpk, precision):
    say(f"table {precision} fcc500")
    spec, params = synth.FCC_MODEL, synth.fcc_params()
    model = dpk.Model(spec, params).tabulate(0.01, 0.5)
    o = oracle_of("fcc")
    coef = o.table(0.01, 50)
    c, t, b = synth.fcc_box(5, 3.6, 1)
    ref = o.compute(c, t, b, table=coef, dx=0.01)
    ctx = dpk.Context(model, precision=precision)
    got = ctx.compute(c, t, b)
    if precision == "fp64":
        check_fp64(got, ref, len(t))
    else:
        check_mixed(got, ref, len(t))
    assert ctx.stats()["table_out_of_range"] == 0
    ctx.close()


_fcc32k = {}


@pytest.mark.parametrize("precision", ["fp64", "mixed", "fp32"])
def test_tabulated_fcc_32000(dpk, precision):
    """The 32,000-atom fcc box (20^3 cells, rc 8.0 A, sel 138) with the tabulated embedding
    (stride 0.01) at full size, every output against the oracle's evaluation of the same table."""
    say(f"table {precision} fcc32000")
    spec, params = synth.FCC_MODEL, synth.fcc_params()
    c, t, b = synth.fcc_32000()
    if not _fcc32k:
        o = oracle_of("fcc")
        _fcc32k["ref"] = o.compute(c, t, b, table=o.table(0.01, 50), dx=0.01)
        _fcc32k["model"] = dpk.Model(spec, params).tabulate(0.01, 0.5)
    ref = _fcc32k["ref"]
    ctx = dpk.Context(_fcc32k["model"], precision=precision)
    got = ctx.compute(c, t, b)
    if precision == "fp64":
        check_fp64(got, ref, len(t))
    else:
        check_mixed(got, ref, len(t))
    st = ctx.stats()
    assert st["table_out_of_range"] == 0 and st["nbr_dropped"] == ref["ndrop"]
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tabulated_fcc_32000_shuffled(dpk, precision):
    """The same box with the caller's atoms in a random order: the table backward's per-block
    force hash then finds few repeated neighbours, fills, and sends most pairs to the direct FP64
    atomics. Every output against the oracle's (forces permuted with the atoms)."""
    say(f"table {precision} fcc32000 shuffled")
    spec, params = synth.FCC_MODEL, synth.fcc_params()
    c, t, b = synth.fcc_32000()
    if not _fcc32k:
        o = oracle_of("fcc")
        _fcc32k["ref"] = o.compute(c, t, b, table=o.table(0.01, 50), dx=0.01)
        _fcc32k["model"] = dpk.Model(spec, params).tabulate(0.01, 0.5)
    ref = dict(_fcc32k["ref"])
    perm = np.random.default_rng(5).permutation(len(t))
    ref["force"] = ref["force"][perm]
    ctx = dpk.Context(_fcc32k["model"], precision=precision)
    got = ctx.compute(c[perm], t[perm], b)
    if precision == "fp64":
        check_fp64(got, ref, len(t))
    else:
        check_mixed(got, ref, len(t))
    assert ctx.stats()["table_out_of_range"] == 0
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_run_to_run_determinism(dpk, precision):
    """The same frame evaluated repeatedly (the same context twice, then a new context): energy and
    per-atom energies are bitwise equal (fixed-order sums), forces and virial, summed by FP64
    atomics in varying order, agree to rounding. The 12,288-atom water box (network) and the
    32,000-atom fcc box with its atoms shuffled (table; groups in bin order, whose order within a
    bin varies run to run)."""
    cases = [("water12288", synth.WATER_MODEL, synth.water_params, None, synth.water_12288()),
             ("fcc32000 shuffled, table", synth.FCC_MODEL, synth.fcc_params, (0.01, 0.5), None)]
    for name, spec, params, tab, frame in cases:
        say(f"determinism {precision} {name}")
        model = dpk.Model(spec, params())
        if tab:
            model.tabulate(*tab)
            c, t, b = synth.fcc_32000()
            perm = np.random.default_rng(5).permutation(len(t))
            frame = (c[perm], t[perm], b)
        c, t, b = frame
        ctx = dpk.Context(model, precision=precision)
        outs = [ctx.compute(c, t, b, atom_energy=True) for _ in range(2)]
        ctx.close()
        ctx = dpk.Context(model, precision=precision)
        outs.append(ctx.compute(c, t, b, atom_energy=True))
        ctx.close()
        a = outs[0]
        for o in outs[1:]:
            assert o["energy"] == a["energy"]
            np.testing.assert_array_equal(o["atom_energy"], a["atom_energy"])
            fs = np.abs(a["force"]).max()
            assert np.abs(o["force"] - a["force"]).max() <= 1e-13 * max(1.0, fs)
            assert np.abs(o["virial"] - a["virial"]).max() <= 1e-13 * max(1.0, np.abs(a["virial"]).max())


def test_context_keeps_the_model_it_was_created_with(dpk):
    """A context evaluates the model as it was when the context was created: tabulating the model
    afterwards (here a table that covers s < 0.1 only, so that its use shows in the out-of-range
    count) leaves the context on the network, and a new context uses the table."""
    say("tabulate after context creation")
    spec, params = synth.FCC_MODEL, synth.fcc_params()
    model = dpk.Model(spec, params)
    c, t, b = synth.fcc_box(5, 3.6, 1)
    ctx = dpk.Context(model, precision="fp64")
    model.tabulate(0.01, 0.1)
    check_fp64(ctx.compute(c, t, b), oracle_of("fcc").compute(c, t, b), len(t))
    assert ctx.stats()["table_out_of_range"] == 0
    ctx2 = dpk.Context(model, precision="fp64")
    ctx2.compute(c, t, b)
    assert ctx2.stats()["table_out_of_range"] > 0
    ctx.close()
    ctx2.close()


def _degenerate_frames():
    """Frames at the edges of the method (water model, r_s 0.5 A, r_c 6.0 A): one atom (no
    neighbours, F = 0); a pair inside r_s (the 1/r branch of the switching function) next to a pair
    in the switching band; pairs just inside and just outside r_c; atoms of one type only (the
    other type's blocks empty). Periodic boxes of 20 A and the same frames with open boundaries."""
    box = np.eye(3) * 20.0
    out = {}
    out["single"] = (np.array([[3.0, 4.0, 5.0]]), np.array([0], dtype=np.int32))
    out["pair_inside_rs"] = (np.array([[5.0, 5.0, 5.0], [5.3, 5.0, 5.0], [5.0, 7.1, 5.0]]),
                             np.array([0, 1, 1], dtype=np.int32))
    out["pairs_at_rc"] = (np.array([[2.0, 2.0, 2.0], [2.0, 2.0, 7.9999], [10.0, 10.0, 10.0],
                                    [10.0, 16.0001, 10.0]]), np.array([0, 1, 0, 1], dtype=np.int32))
    rng = np.random.default_rng(11)
    out["one_type"] = (rng.uniform(0.0, 20.0, (40, 3)), np.ones(40, dtype=np.int32))
    frames = {}
    for name, (c, t) in out.items():
        frames[name + "_periodic"] = (c, t, box)
        frames[name + "_open"] = (c, t, None)
    return frames


@pytest.mark.parametrize("precision", ["fp64", "mixed", "fp32"])
def test_degenerate_frames(dpk, precision):
    spec, params, model = model_of(dpk, "water")
    ctx = dpk.Context(model, precision=precision)
    for name, (c, t, b) in _degenerate_frames().items():
        say(f"{precision} {name}")
        ref = oracle_of("water").compute(c, t, b)
        got = ctx.compute(c, t, b)
        (check_fp64 if precision == "fp64" else check_mixed)(got, ref, len(t))
        if name.startswith("single"):
            assert np.all(got["force"] == 0.0)
    ctx.close()


def test_errors_are_reported(dpk):
    say("error paths")
    spec, params, model = model_of(dpk, "water")
    ctx = dpk.Context(model, precision="fp64")
    c, t, b = synth.water_192()
    bad = t.copy()
    bad[5] = 7
    with pytest.raises(dpk.DpkError) as e:
        ctx.compute(c, bad, b)
    assert e.value.code == dpk.DPK_E_TYPE_RANGE
    with pytest.raises(dpk.DpkError) as e:
        ctx.compute(c, t, -b)
    assert e.value.code == dpk.DPK_E_BOX
    with pytest.raises(dpk.DpkError) as e:
        ctx.compute(c[:0], t[:0], b)
    assert e.value.code == dpk.DPK_E_INVALID_ARG
    # the context still works after errors
    ref = oracle_of("water").compute(c, t, b)
    check_fp64(ctx.compute(c, t, b), ref, len(t))
    ctx.close()
