"""Pins of the oracle's domain evaluation (owned + ghost atoms, Sec. III.B.2) against its periodic
evaluation (no GPU): a periodic water box cut into 2 x 2 x 2 bricks, each brick evaluated on its
owned atoms with ghost copies of every atom within r_c (as an MD code's halo exchange supplies them),
then the ghosts' forces added to their owners (the reverse exchange): the energies, per-atom
energies, forces and virials of the bricks add up to those of the periodic frame. A halo wider than
r_c, and ghosts in another order, change nothing."""
import numpy as np
import pytest

from oracle import Oracle
from paper_2304_09409_amd import synth


def _reassemble(o, bricks, n):
    e, f, v, ei = 0.0, np.zeros((n, 3)), np.zeros((3, 3)), np.full(n, np.nan)
    for br in bricks:
        r = o.compute_ghost(br["coord"], br["atype"], br["nlocal"])
        e += r["energy"]
        np.add.at(f, br["owner"], r["force"])
        v += r["virial"]
        ei[br["owner"][:br["nlocal"]]] = r["atom_energy"]
    return e, f, v, ei


@pytest.mark.parametrize("halo,seed", [(6.0, None), (7.5, 3)])
def test_bricks_add_up_to_the_periodic_frame(water_oracle, halo, seed):
    c, t, b = synth.water_box(8, 24.85, 5)      # 1,536 atoms, L = 24.85 A, 4 r_c bricks of 12.4 A
    ref = water_oracle.compute(c, t, b)
    bricks = synth.ghost_bricks(c, t, b, (2, 2, 2), halo=halo, seed=seed)
    assert sum(br["nlocal"] for br in bricks) == len(t)
    e, f, v, ei = _reassemble(water_oracle, bricks, len(t))
    assert e == pytest.approx(ref["energy"], rel=1e-12)
    np.testing.assert_allclose(ei, ref["atom_energy"], atol=1e-11)
    np.testing.assert_allclose(f, ref["force"], atol=1e-11)
    np.testing.assert_allclose(v, ref["virial"], atol=1e-9)


def test_single_domain_without_ghosts_is_the_open_cluster(water_oracle):
    c, t = synth.serving_frame(120, 3, 2)[:2]
    ref = water_oracle.compute(c, t, None)
    got = water_oracle.compute_ghost(c, t, len(t))
    assert got["energy"] == ref["energy"]
    np.testing.assert_array_equal(got["force"], ref["force"])
