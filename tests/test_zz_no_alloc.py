"""The allocation-free device entry point (dpk_compute_device_noalloc) against the device entry
point it is a variant of (dpk_compute_device): the same kernels on the same inputs, so every output
agrees to the reordering of FP64 force atomics and block sums (1e-12 eV/A on forces, 1e-12
relative on the energy and virial). Two calls in a row, the second on a smaller frame, so the
second runs on what the first left in the shared region; both precisions; frames past the region's
size and open clusters are refused with a clear error."""
import sys

import numpy as np
import pytest

from paper_2304_09409_amd import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _run(ctx, frame, noalloc):
    import torch
    c, t, b = frame
    n = len(t)
    dev = torch.device("cuda:0")
    coord = torch.tensor(c, dtype=torch.float64, device=dev)
    atype = torch.tensor(t, dtype=torch.int32, device=dev)
    e = torch.zeros(1, dtype=torch.float64, device=dev)
    f = torch.full((n, 3), 7.0, dtype=torch.float64, device=dev)   # the path must overwrite it
    v = torch.zeros(9, dtype=torch.float64, device=dev)
    ae = torch.zeros(n, dtype=torch.float64, device=dev)
    ctx.compute_device(coord, atype, b, e, f, v, ae, noalloc=noalloc)
    ctx.check()
    torch.cuda.synchronize()
    return {"energy": e.item(), "force": f.cpu().numpy(), "virial": v.cpu().numpy().reshape(3, 3),
            "atom_energy": ae.cpu().numpy(), "drops": ctx.stats()["nbr_dropped"]}


def _same(a, b):
    assert np.abs(a["force"] - b["force"]).max() <= 1e-12
    assert abs(a["energy"] - b["energy"]) <= 1e-12 * max(1.0, abs(b["energy"]))
    assert np.abs(a["virial"] - b["virial"]).max() <= 1e-12 * max(1.0, np.abs(b["virial"]).max())
    assert np.abs(a["atom_energy"] - b["atom_energy"]).max() <= 1e-12 * max(1.0, np.abs(b["atom_energy"]).max())
    assert a["drops"] == b["drops"]


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_noalloc_matches_device_entry_point(precision):
    from paper_2304_09409_amd import dpk
    model = dpk.Model(synth.WATER_MODEL, synth.water_params())
    ctx = dpk.Context(model, precision=precision)
    # a large frame (multi-block preparation), then a smaller one over what it left behind
    for name, frame in (("water12288" if precision == "mixed" else "water_9000", synth.water_12288() if precision == "mixed"
                         else synth.water_box(15, 46.6, 9, n_mol=3000)),
                        ("water192", synth.water_192())):
        say(f"noalloc {precision} {name}")
        ref = _run(ctx, frame, noalloc=False)
        got = _run(ctx, frame, noalloc=True)
        _same(got, ref)
        # the context's own workspace still works after a call in the shared region
        again = _run(ctx, frame, noalloc=False)
        _same(again, ref)
    ctx.close()


def test_noalloc_refuses_what_it_cannot_hold():
    import torch
    from paper_2304_09409_amd import dpk
    say("noalloc limits")
    model = dpk.Model(synth.WATER_MODEL, synth.water_params())
    ctx = dpk.Context(model, precision="fp64")
    c, t, b = synth.water_110592()
    n = len(t)
    dev = torch.device("cuda:0")
    args = (torch.tensor(c, device=dev), torch.tensor(t, dtype=torch.int32, device=dev))
    outs = (torch.zeros(1, dtype=torch.float64, device=dev), torch.zeros((n, 3), dtype=torch.float64, device=dev),
            torch.zeros(9, dtype=torch.float64, device=dev))
    with pytest.raises(dpk.DpkError) as e:
        ctx.compute_device(*args, b, *outs, noalloc=True)
    assert e.value.code == dpk.DPK_E_BUDGET
    with pytest.raises(dpk.DpkError) as e:
        ctx.compute_device(*args, None, *outs, noalloc=True)
    assert e.value.code == dpk.DPK_E_INVALID_ARG
    ctx.close()
