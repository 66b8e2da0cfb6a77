"""The compressed embedding of the two-body descriptor (Sec. II.A.6, eq. compress) against the
oracle's evaluation of the same table, in the shapes its product kernels take beyond the
single-type fcc box of test_gpu_parity.py:
  * two atom types (a pass per centre and neighbour type; groups of four atoms across a type
    boundary) with a table over [0, 2.7] of 270 intervals, so that a group's intervals fill many
    LDS windows (FP32 windows of at most 32 intervals, FP64 of 16);
  * three types with type_one_side nets (one pass per neighbour type covering every centre type);
  * an ensemble of tabulated models (model deviation, Sec. II.C: one launch for every model);
  * batched frames through the server (per-atom virials).
Tolerances as test_gpu_parity.py: FP64 forces within 1e-10 eV/A, energy within max(1e-9 eV,
1e-12 |E|), virial within max(1e-9 N/1000, 1e-12 max|Xi|); mixed and FP32 forces within 1e-3 eV/A,
|dE|/N within max(1e-4 eV, 1e-5 |E|/N), |dXi|/N within 1e-3 eV."""
import sys

import numpy as np
import pytest

from paper_2304_09409_amd import synth

pytestmark = pytest.mark.gpu

DX = 0.01


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def check(got, ref, n, precision):
    df = np.abs(got["force"] - ref["force"]).max()
    if precision == "fp64":
        de = abs(got["energy"] - ref["energy"])
        dv = np.abs(got["virial"] - ref["virial"]).max()
        print(f"  max|dF| {df:.3e}  |dE| {de:.3e}  max|dXi| {dv:.3e}", flush=True)
        assert df <= 1e-10
        assert de <= max(1e-9, 1e-12 * abs(ref["energy"]))
        assert dv <= max(1e-9 * max(1.0, n / 1000.0), 1e-12 * np.abs(ref["virial"]).max())
    else:
        de = abs(got["energy"] - ref["energy"]) / n
        dv = np.abs(got["virial"] - ref["virial"]).max() / n
        print(f"  max|dF| {df:.3e}  |dE|/N {de:.3e}  max|dXi|/N {dv:.3e}", flush=True)
        assert df <= 1e-3
        assert de <= max(1e-4, 1e-5 * abs(ref["energy"]) / n)
        assert dv <= 1e-3


def tos_model():
    spec = dict(synth.SERVE_MODEL, type_one_side=True)
    return spec, synth.make_params(spec, 31, synth.SERVE_OUT_SCALE, synth.SERVE_FIT_IN, timestep_sigma=0.2)


_refs = {}


def oracle_ref(key, spec, params, frame, nint):
    """The oracle's E, F, virial of a frame with its own table of nint intervals of DX."""
    from oracle import Oracle
    if key not in _refs:
        o = Oracle(spec, params)
        c, t, b = frame
        _refs[key] = o.compute(c, t, b, table=o.table(DX, nint), dx=DX)
        assert _refs[key]["table_oor"] == 0
    return _refs[key]


WATER_FRAMES = {
    "water192": lambda: synth.water_192(),
    "frame700_2type": lambda: synth.serving_frame(700, 9, 2),
    "water12288": lambda: synth.water_12288(),
}


@pytest.mark.parametrize("precision", ["fp64", "mixed", "fp32"])
def test_two_types_many_windows(precision):
    from paper_2304_09409_amd import dpk
    spec, params = synth.WATER_MODEL, synth.water_params()
    model = dpk.Model(spec, params).tabulate(DX, 2.7)
    ctx = dpk.Context(model, precision=precision)
    for name, make in WATER_FRAMES.items():
        c, t, b = make()
        say(f"table {precision} {name} (270 intervals)")
        ref = oracle_ref(("water", name), spec, params, (c, t, b), 270)
        check(ctx.compute(c, t, b), ref, len(t), precision)
        assert ctx.stats()["table_out_of_range"] == 0
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_type_one_side_three_types(precision):
    from paper_2304_09409_amd import dpk
    spec, params = tos_model()
    model = dpk.Model(spec, params).tabulate(DX, 3.0)
    ctx = dpk.Context(model, precision=precision)
    for seed, n in ((19, 300), (23, 1500)):
        c, t, b = synth.serving_frame(n, seed, 3)
        say(f"table type_one_side {precision} serve{n}_3type")
        ref = oracle_ref(("tos", n), spec, params, (c, t, b), 300)
        check(ctx.compute(c, t, b), ref, n, precision)
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tabulated_ensemble(precision):
    """Model deviation of three tabulated water models: every member's forces and eps_F against
    the oracle's members, each with its own table."""
    from oracle import Oracle
    from oracle.devi import model_deviation
    from paper_2304_09409_amd import dpk
    spec = synth.WATER_MODEL
    ps = synth.ensemble_params(spec, synth.water_params(), 3)
    c, t, b = synth.serving_frame(700, 9, 2)
    say(f"table ensemble {precision}")
    refs = []
    for p in ps:
        o = Oracle(spec, p)
        refs.append(o.compute(c, t, b, table=o.table(DX, 270), dx=DX))
    ref = model_deviation(np.stack([r["force"] for r in refs]), np.stack([r["virial"] for r in refs]))
    dv = dpk.Deviation([dpk.Model(spec, p).tabulate(DX, 2.7) for p in ps], precision=precision)
    got = dv.compute(c, t, b)
    tol = 1e-10 if precision == "fp64" else 1e-3
    for k in range(3):
        df = np.abs(got["force"][k] - refs[k]["force"]).max()
        print(f"  member {k}: max|dF| {df:.3e}", flush=True)
        assert df <= tol
    assert np.abs(got["eps_f"] - ref["eps_f"]).max() <= tol
    dv.close()


def test_tabulated_server_batches():
    """Frames of several sizes through the server (batched launches, per-atom virials), FP64."""
    from paper_2304_09409_amd import dpk
    spec, params = synth.WATER_MODEL, synth.water_params()
    model = dpk.Model(spec, params).tabulate(DX, 2.7)
    fr = [synth.serving_frame(n, 40 + i, 2) for i, n in enumerate((80, 300, 57, 500))]
    say("table server fp64")
    srv = dpk.Server(model, precision="fp64", nslots=2)
    tickets = [srv.submit(c, t, b) for c, t, b in fr]
    for k, ((c, t, b), tk) in enumerate(zip(fr, tickets)):
        ref = oracle_ref(("server", k), spec, params, (c, t, b), 270)
        got = tk.result()
        check(got, ref, len(t), "fp64")
    srv.close()
