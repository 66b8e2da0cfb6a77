"""A model loaded from its file evaluates like the in-memory model it was saved from: per-atom
energies and the energy bit for bit (fixed-order sums), forces and virial to the reordering of the
FP64 force atomics (1e-12); network and compressed models, FP64 and mixed. And the device-box entry
point (the cell in device memory) gives what the host-box entry point gives."""
import sys

import numpy as np
import pytest

from paper_2304_09409_amd import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("kind", ["water", "fcc_table"])
def test_loaded_model_evaluates_identically(tmp_path, kind, precision):
    from paper_2304_09409_amd import dpk
    say(f"model file {kind} {precision}")
    if kind == "water":
        m = dpk.Model(synth.WATER_MODEL, synth.water_params())
        c, t, b = synth.water_192()
    else:
        m = dpk.Model(synth.FCC_MODEL, synth.fcc_params()).tabulate(0.01, 0.5)
        c, t, b = synth.fcc_box(5, 3.6, 1)
    path = str(tmp_path / "m.dpk")
    m.save(path)
    m2 = dpk.Model.load(path)
    outs = []
    for model in (m, m2):
        ctx = dpk.Context(model, precision=precision)
        outs.append(ctx.compute(c, t, b, atom_energy=True))
        ctx.close()
    a, z = outs
    assert a["energy"] == z["energy"]
    np.testing.assert_array_equal(a["atom_energy"], z["atom_energy"])
    assert np.abs(a["force"] - z["force"]).max() <= 1e-12
    assert np.abs(a["virial"] - z["virial"]).max() <= 1e-12 * max(1.0, np.abs(a["virial"]).max())


def test_device_box_entry_point():
    import torch
    from paper_2304_09409_amd import dpk
    say("device box")
    m = dpk.Model(synth.SERVE_MODEL, synth.serve_params())
    ctx = dpk.Context(m, precision="fp64")
    c0, t, b0 = synth.serving_frame(400, 2, 3)
    b = b0 + np.array([[0, 0, 0], [4.0, 0, 0], [-3.0, 5.0, 0]])
    c = (c0 @ np.linalg.inv(b0)) @ b
    ref = ctx.compute(c, t, b)
    dev = torch.device("cuda:0")
    n = len(t)
    coord = torch.tensor(c, device=dev)
    atype = torch.tensor(t, dtype=torch.int32, device=dev)
    dbox = torch.tensor(b, device=dev)
    e = torch.zeros(1, dtype=torch.float64, device=dev)
    f = torch.zeros((n, 3), dtype=torch.float64, device=dev)
    v = torch.zeros(9, dtype=torch.float64, device=dev)
    s = torch.cuda.current_stream()
    dpk._check(dpk.lib().dpk_compute_device_dbox(ctx.handle, n, coord.data_ptr(), atype.data_ptr(), dbox.data_ptr(),
                                                 e.data_ptr(), f.data_ptr(), v.data_ptr(), None, s.cuda_stream))
    ctx.check()
    assert abs(e.item() - ref["energy"]) <= 1e-12 * abs(ref["energy"])
    assert np.abs(f.cpu().numpy() - ref["force"]).max() <= 1e-12
    np.testing.assert_allclose(v.cpu().numpy().reshape(3, 3), ref["virial"], rtol=1e-12, atol=1e-10)
    ctx.close()
