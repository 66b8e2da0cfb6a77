"""The adjoint behind torch.autograd.Function on the 110,592-atom water box.

* autograd: coord.grad equals -F exactly (the backward returns the adjoint's force).
* central finite differences (h = 1e-4 A) of the energy on 64 seeded atoms, one seeded component
  each, in the FP64 instantiation of the same kernels (mixed-precision energies are resolved to
  FP32 and cannot resolve a 1e-4 A displacement): |F + dE/dr| within 1e-6 eV/A.
* the mixed path against the FP64 CPU oracle on the whole frame: every force component within
  1e-3 eV/A; the FP64 path within 1e-10 eV/A.
* the literal 71.5 A box of the same atom count (0.30 atoms/A^3, about 270 atoms within r_c, heavy
  truncation by sel): FP64 path against the oracle, neighbour drops counted identically.
"""
import sys

import numpy as np
import pytest

from paper_2304_09409_amd import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def big():
    from oracle import Oracle
    c, t, b = synth.water_110592()
    say("oracle water110592 (CPU)")
    ref = Oracle(synth.WATER_MODEL, synth.water_params()).compute(c, t, b)
    return c, t, b, ref


@pytest.fixture(scope="module")
def model():
    from paper_2304_09409_amd import dpk
    return dpk.Model(synth.WATER_MODEL, synth.water_params())


def test_autograd_and_finite_differences_fp64(big, model):
    import torch
    from paper_2304_09409_amd.torch_op import DPEnergy
    c, t, b, ref = big
    say("autograd fp64 water110592")
    mod = DPEnergy(model, precision="fp64")
    coord = torch.tensor(c, device="cuda", requires_grad=True)
    atype = torch.tensor(t, device="cuda", dtype=torch.int32)
    E, F, V = mod(coord, atype, b)
    E.sum().backward()
    assert torch.equal(coord.grad, -F)
    np.testing.assert_allclose(F.cpu().numpy(), ref["force"], atol=1e-10)
    np.testing.assert_allclose(V.cpu().numpy(), ref["virial"], atol=1e-8)
    assert abs(E.item() - ref["energy"]) <= 1e-12 * abs(ref["energy"])

    rng = np.random.default_rng(64)
    atoms = rng.choice(len(t), 64, replace=False)
    comps = rng.integers(0, 3, 64)
    h = 1e-4
    Fh = F.cpu().numpy()
    worst = 0.0
    base = coord.detach().clone()
    with torch.no_grad():
        for a, k in zip(atoms, comps):
            cp = base.clone()
            cp[a, k] += h
            ep = mod(cp, atype, b)[0].item()
            cp[a, k] -= 2 * h
            em = mod(cp, atype, b)[0].item()
            fd = -(ep - em) / (2 * h)
            worst = max(worst, abs(fd - Fh[a, k]))
    print(f"  max |F + dE/dr (FD)| over 64 atoms: {worst:.3e}", flush=True)
    assert worst <= 1e-6


def test_mixed_against_oracle_110592(big, model):
    import torch
    from paper_2304_09409_amd.torch_op import DPEnergy
    c, t, b, ref = big
    say("mixed water110592 vs oracle")
    mod = DPEnergy(model, precision="mixed")
    coord = torch.tensor(c, device="cuda", requires_grad=True)
    atype = torch.tensor(t, device="cuda", dtype=torch.int32)
    E, F, V = mod(coord, atype, b)
    E.sum().backward()
    assert torch.equal(coord.grad, -F)
    d = np.abs(F.cpu().numpy() - ref["force"])
    print(f"  mixed max|dF| {d.max():.3e} rms {np.sqrt((d ** 2).mean()):.3e} "
          f"|dE|/N {abs(E.item() - ref['energy']) / len(t):.3e}", flush=True)
    assert d.max() <= 1e-3
    assert abs(E.item() - ref["energy"]) / len(t) <= 1e-4
    assert np.abs(V.cpu().numpy() - ref["virial"]).max() / len(t) <= 1e-3


def test_dense_box_truncation_fp64(model):
    from oracle import Oracle
    from paper_2304_09409_amd import dpk
    c, t, b = synth.water_110592(box_len=71.5)
    say("oracle water110592 at 71.5 A (CPU)")
    ref = Oracle(synth.WATER_MODEL, synth.water_params()).compute(c, t, b)
    say("fp64 water110592 at 71.5 A")
    ctx = dpk.Context(model, precision="fp64")
    got = ctx.compute(c, t, b)
    st = ctx.stats()
    print(f"  drops {st['nbr_dropped']} (oracle {ref['ndrop']}), max candidates {st['max_candidates']}", flush=True)
    assert st["nbr_dropped"] == ref["ndrop"] > 0
    np.testing.assert_allclose(got["force"], ref["force"], atol=1e-10)
    ctx.close()
