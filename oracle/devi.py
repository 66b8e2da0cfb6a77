"""TEST INFRASTRUCTURE ONLY: model deviation of an ensemble, written out from its definition.

Sec. II.C (model deviation): for an ensemble of n_m models with the ensemble average
<y> = n_m^-1 sum_k y_k,
    eps_F,i   = sqrt(< |F_i - <F_i>|^2 >)                       (per atom),
    eps_Xi,ab = N^-1 sqrt(< (Xi_ab - <Xi_ab>)^2 >)               (per virial component),
the relative forms eps_F,i / (|<F_i>| + nu) and eps_Xi,ab / (|<Xi_ab>| + nu) (the paper's |<Xi>|
read per component), and the max / average / min of eps_F,i over the atoms and of eps_Xi,ab over
the nine components. The per-model forces and virials come from the FP64 oracle (dp_oracle.c), one
model at a time. Plain loops over the models; numpy over atoms.

Only tests/ and the benchmark's CPU-baseline leg may import this module.
"""
from __future__ import annotations

import numpy as np


def model_deviation(forces, virials, nu=None) -> dict:
    """forces [n_m][N][3], virials [n_m][3][3] (FP64). nu None: absolute deviations."""
    forces = np.asarray(forces, dtype=np.float64)
    virials = np.asarray(virials, dtype=np.float64).reshape(len(forces), 3, 3)
    nm, n = forces.shape[0], forces.shape[1]
    mean_f = np.zeros((n, 3))
    for k in range(nm):
        mean_f += forces[k]
    mean_f /= nm
    sq = np.zeros(n)
    for k in range(nm):
        d = forces[k] - mean_f
        sq += (d * d).sum(axis=1)
    eps_f = np.sqrt(sq / nm)
    mean_v = np.zeros((3, 3))
    for k in range(nm):
        mean_v += virials[k]
    mean_v /= nm
    sqv = np.zeros((3, 3))
    for k in range(nm):
        sqv += (virials[k] - mean_v) ** 2
    eps_v = np.sqrt(sqv / nm) / n
    if nu is not None:
        eps_f = eps_f / (np.sqrt((mean_f * mean_f).sum(axis=1)) + nu)
        eps_v = eps_v / (np.abs(mean_v) + nu)
    stats = {"f_max": float(eps_f.max()), "f_avg": float(eps_f.sum() / n), "f_min": float(eps_f.min()),
             "v_max": float(eps_v.max()), "v_avg": float(eps_v.sum() / 9.0), "v_min": float(eps_v.min())}
    return {"eps_f": eps_f, "eps_v": eps_v, "stats": stats}


def ensemble(oracles, coord, atype, box, nu=None, **kw) -> dict:
    """Every model of the ensemble on one frame (FP64 oracle), then their deviation."""
    outs = [o.compute(coord, atype, box, **kw) for o in oracles]
    dev = model_deviation([r["force"] for r in outs], [r["virial"] for r in outs], nu)
    dev.update(energy=np.array([r["energy"] for r in outs]), force=np.stack([r["force"] for r in outs]),
               virial=np.stack([r["virial"] for r in outs]))
    return dev
