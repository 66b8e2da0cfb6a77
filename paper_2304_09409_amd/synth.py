"""Seeded synthetic inputs: atomic frames and random-initialised model parameters.

This module only draws numbers. It holds none of the Deep Potential arithmetic, so both the
HIP path and the CPU oracle may take their inputs from it.

Frames (all lengths in Angstrom):
  * ``water_box``: water-like liquid. Molecule sites sit on a cubic lattice; O is at the site and
    the two H atoms at 0.9572 A with an H-O-H angle of 104.52 deg in a random orientation; every
    atom is then jittered by N(0, sigma) per component. Atom order is O,H,H per molecule
    (types 0,1,1), so the caller order interleaves the types.
  * ``fcc_box``: single-type fcc metal, 4-atom basis, thermal jitter.
  * ``serving_frame``: atomic simple-cubic lattice at a given density, a random subset of the
    sites, jitter, and a seeded type shuffle (2 types in ratio 1:2 or 3 types in ratio 2:1:1).

Models: ``make_params`` draws a flat float64 parameter blob in the layout documented in
``include/dpk.h`` (embedding nets first, then fitting nets; per layer W row-major [in x out],
then the bias b, then the timestep vector w_hat).
"""
from __future__ import annotations

import math

import numpy as np

# Model shapes used by the workloads. sel = per-type neighbour capacity; emb = embedding widths;
# fit = fitting hidden widths; axis = M_<.
WATER_MODEL = dict(ntypes=2, sel=[46, 92], rcut=6.0, rcut_smth=0.5, emb=[25, 50, 100],
                   axis=16, fit=[240, 240, 240], type_one_side=False)
FCC_MODEL = dict(ntypes=1, sel=[138], rcut=8.0, rcut_smth=2.0, emb=[25, 50, 100],
                 axis=16, fit=[240, 240, 240], type_one_side=False)
# One 3-type model serves both the 2-type (1:2) and the 3-type (2:1:1) request frames; its
# capacities are about twice the mean neighbour count of each type at 0.1 atoms/A^3 and rc = 6 A.
SERVE_MODEL = dict(ntypes=3, sel=[92, 92, 46], rcut=6.0, rcut_smth=0.5, emb=[25, 50, 100],
                   axis=16, fit=[240, 240, 240], type_one_side=False)

# The other DeepPot-SE descriptors on the water-like systems: radial-only two-body embedding
# (se_e2_r, same cut-offs and capacities) and the three-body embedding (se_e3, whose pair sum over
# neighbour pairs grows as the square of the neighbour count: shorter cut-off, smaller capacities).
WATER_R_MODEL = dict(WATER_MODEL, descriptor="se_e2_r")
WATER_E3_MODEL = dict(ntypes=2, sel=[20, 40], rcut=4.0, rcut_smth=0.5, emb=[25, 50, 100],
                      axis=16, fit=[240, 240, 240], type_one_side=False, descriptor="se_e3")

# Scales of the first fitting layer and of the output layer, chosen once so that the random
# models respond to geometry like trained ones: RMS force component about 1 eV/A on the
# 12,288-atom water box, and about 0.2 eV/A (a thermal metal) on the 32,000-atom fcc box.
WATER_FIT_IN, WATER_OUT_SCALE = 1000.0, 5.07
FCC_FIT_IN, FCC_OUT_SCALE = 30.0, 300.0
SERVE_FIT_IN, SERVE_OUT_SCALE = 1000.0, 5.07
WATER_R_FIT_IN, WATER_R_OUT_SCALE = 30.0, 10.0
WATER_E3_FIT_IN, WATER_E3_OUT_SCALE = 300.0, 11.0

PARAM_SEED = 2304


def _rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """n uniformly random rotation matrices (unit quaternions from 4 Gaussians)."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    r = np.empty((n, 3, 3))
    r[:, 0, 0] = 1 - 2 * (y * y + z * z)
    r[:, 0, 1] = 2 * (x * y - z * w)
    r[:, 0, 2] = 2 * (x * z + y * w)
    r[:, 1, 0] = 2 * (x * y + z * w)
    r[:, 1, 1] = 1 - 2 * (x * x + z * z)
    r[:, 1, 2] = 2 * (y * z - x * w)
    r[:, 2, 0] = 2 * (x * z - y * w)
    r[:, 2, 1] = 2 * (y * z + x * w)
    r[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return r


def water_box(n_side: int, box_len: float, seed: int, sigma: float = 0.1,
              n_mol: int | None = None):
    """Water-like frame: returns (coord [N,3] f64, atype [N] i32, box [3,3] f64)."""
    rng = np.random.default_rng(seed)
    a = box_len / n_side
    idx = np.arange(n_side ** 3)
    if n_mol is not None and n_mol < idx.size:
        idx = np.sort(rng.choice(idx.size, size=n_mol, replace=False))
    ix, iy, iz = idx // (n_side * n_side), (idx // n_side) % n_side, idx % n_side
    sites = (np.stack([ix, iy, iz], axis=1) + 0.5) * a
    nm = sites.shape[0]
    bond, half = 0.9572, math.radians(104.52) / 2.0
    local = np.array([[0.0, 0.0, 0.0],
                      [bond * math.sin(half), 0.0, bond * math.cos(half)],
                      [-bond * math.sin(half), 0.0, bond * math.cos(half)]])
    rot = _rotations(rng, nm)
    mol = sites[:, None, :] + np.einsum("mij,aj->mai", rot, local)
    coord = mol.reshape(-1, 3) + rng.normal(0.0, sigma, (3 * nm, 3))
    atype = np.tile(np.array([0, 1, 1], dtype=np.int32), nm)
    return coord.astype(np.float64), atype, np.diag([box_len] * 3).astype(np.float64)


def fcc_box(n_cell: int, lattice: float, seed: int, sigma: float = 0.05):
    """Single-type fcc frame: returns (coord, atype, box)."""
    rng = np.random.default_rng(seed)
    basis = np.array([[0, 0, 0], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])
    g = np.arange(n_cell)
    cells = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    coord = ((cells[:, None, :] + basis[None]) * lattice).reshape(-1, 3)
    coord = coord + rng.normal(0.0, sigma, coord.shape)
    atype = np.zeros(coord.shape[0], dtype=np.int32)
    box = np.diag([n_cell * lattice] * 3)
    return coord.astype(np.float64), atype, box.astype(np.float64)


def tie_lattice(n: int = 8, spacing: float = 2.0):
    """Unjittered 2-type simple-cubic frame (types by the parity of i + j + k) in a cubic cell of
    n * spacing: with spacing and cell length powers of two every coordinate, wrapped position and
    squared distance is exact, so many neighbours sit at exactly equal distances (ties)."""
    g = np.arange(n)
    sites = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    coord = sites.astype(np.float64) * spacing
    atype = (sites.sum(axis=1) % 2).astype(np.int32)
    return coord, atype, np.diag([n * spacing] * 3).astype(np.float64)


def serving_frame(natoms: int, seed: int, ntypes: int, density: float = 0.1,
                  sigma: float = 0.1):
    """One request frame: simple-cubic sites at the given density, random subset, jitter."""
    rng = np.random.default_rng(seed)
    box_len = (natoms / density) ** (1.0 / 3.0)
    n = int(math.ceil(natoms ** (1.0 / 3.0) - 1e-9))
    a = box_len / n
    idx = np.sort(rng.choice(n ** 3, size=natoms, replace=False))
    sites = np.stack([idx // (n * n), (idx // n) % n, idx % n], axis=1).astype(np.float64)
    coord = (sites + 0.5) * a + rng.normal(0.0, sigma, (natoms, 3))
    if ntypes == 2:
        ratio = np.array([1, 2])
    elif ntypes == 3:
        ratio = np.array([2, 1, 1])
    else:
        raise ValueError("serving frames use 2 or 3 types")
    counts = np.floor(natoms * ratio / ratio.sum()).astype(int)
    counts[0] += natoms - counts.sum()
    atype = np.repeat(np.arange(ntypes), counts).astype(np.int32)
    rng.shuffle(atype)
    return coord, atype, np.diag([box_len] * 3)


def serving_stream(n_req: int, seed: int, n_min: int = 50, n_max: int = 3000):
    """Request sizes (log-uniform) and type counts for a serving stream."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(math.log(n_min), math.log(n_max), n_req)).astype(int)
    ntypes = rng.choice([2, 3], size=n_req)
    seeds = rng.integers(0, 2 ** 31 - 1, size=n_req)
    return sizes, ntypes, seeds


def layer_shapes(model: dict):
    """(n_in, n_out) of every layer, embedding nets first, then fitting nets. The descriptor kind
    ("se_e2_a" default, "se_e2_r", "se_e3") sets the fitting input width (M x M_< or M) and the
    net count (se_e3: a net per ordered pair of neighbour types)."""
    nt = model["ntypes"]
    desc = model.get("descriptor", "se_e2_a")
    n_emb = nt if (model["type_one_side"] and desc != "se_e3") else nt * nt
    emb = [1] + list(model["emb"])
    width = model["emb"][-1] * model["axis"] if desc == "se_e2_a" else model["emb"][-1]
    fit = [width] + list(model["fit"]) + [1]
    shapes = []
    for _ in range(n_emb):
        shapes += [(emb[k], emb[k + 1]) for k in range(len(emb) - 1)]
    for _ in range(nt):
        shapes += [(fit[k], fit[k + 1]) for k in range(len(fit) - 1)]
    return shapes


def param_count(model: dict) -> int:
    return sum(i * o + 2 * o for i, o in layer_shapes(model))


def make_params(model: dict, seed: int = PARAM_SEED, out_scale: float = 1.0,
                fit_in_scale: float = 1.0, timestep_sigma: float = 0.0) -> np.ndarray:
    """Random-initialised FP64 parameters: W ~ N(0, 1/sqrt(n_in+n_out)), b ~ N(0, 1),
    w_hat = 1 (+ optional N(0, timestep_sigma) noise). The first fitting layer's W is multiplied
    by fit_in_scale (the descriptor is not normalised, so its entries are ~1e-3 and a unit-scale
    layer would leave the energy almost independent of the geometry); the output layer's W is
    multiplied by out_scale and its bias is 0."""
    rng = np.random.default_rng(seed)
    nt = model["ntypes"]
    n_emb = nt if (model["type_one_side"] and model.get("descriptor", "se_e2_a") != "se_e3") else nt * nt
    n_emb_layers = n_emb * len(model["emb"])
    shapes = layer_shapes(model)
    n_fit_layers = len(model["fit"]) + 1
    out = []
    for li, (i, o) in enumerate(shapes):
        w = rng.normal(0.0, 1.0 / math.sqrt(i + o), (i, o))
        b = rng.normal(0.0, 1.0, o)
        wh = np.ones(o) + (rng.normal(0.0, timestep_sigma, o) if timestep_sigma else 0.0)
        fit_layer = (li - n_emb_layers) % n_fit_layers if li >= n_emb_layers else -1
        if fit_layer == 0:
            w = w * fit_in_scale
        if fit_layer == n_fit_layers - 1:
            w = w * out_scale
            b = np.zeros(o)
        out += [w.ravel(), b, wh]
    p = np.concatenate(out).astype(np.float64)
    assert p.size == param_count(model)
    return p


# ----------------------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------------------

def water_192(seed: int = 1):
    """192-atom water-like box (64 molecules), cubic 12.42 A."""
    return water_box(4, 12.42, seed)


def water_12288(seed: int = 2):
    """12,288-atom water-like box (4,096 molecules), cubic 49.7 A."""
    return water_box(16, 49.7, seed)


def water_110592(seed: int = 4, box_len: float = 103.38):
    """110,592-atom water-like box (36,864 molecules) at water density (103.38 A)."""
    return water_box(34, box_len, seed, n_mol=36864)


def fcc_32000(seed: int = 3):
    """32,000-atom fcc box, a = 3.6 A, 20^3 cells, jitter 0.05 A."""
    return fcc_box(20, 3.6, seed)


def ghost_bricks(coord, atype, box, nsplit=(2, 2, 2), halo: float = 6.0, seed: int | None = None):
    """Domain decomposition of a frame in an orthorhombic periodic cell, as an MD code's spatial
    decomposition hands it to each domain: the cell is cut into nsplit bricks; a brick owns the atoms
    whose wrapped position lies in it, and receives as ghosts every periodic image of every atom
    within `halo` of the brick (outside it, or inside as another image). Returns one dict per brick:
    coord (owned first, then ghosts), atype, nlocal, and owner (the frame index of each atom, so a
    ghost's force can be added to its owner). seed: shuffle the ghosts' order."""
    L = np.diag(np.asarray(box, dtype=np.float64))
    assert np.allclose(np.asarray(box) - np.diag(L), 0.0), "orthorhombic cells only"
    x = np.asarray(coord, dtype=np.float64)
    x = x - np.floor(x / L) * L
    nsplit = np.asarray(nsplit)
    w = L / nsplit
    cell = np.minimum((x // w).astype(int), nsplit - 1)
    shifts = np.array([[a, b, c] for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)], dtype=float)
    rng = None if seed is None else np.random.default_rng(seed)
    out = []
    for bx in range(nsplit[0]):
        for by in range(nsplit[1]):
            for bz in range(nsplit[2]):
                b = np.array([bx, by, bz])
                lo, hi = b * w, (b + 1) * w
                own = np.nonzero(np.all(cell == b, axis=1))[0]
                gidx, gpos = [], []
                for sh in shifts:
                    p = x + sh * L
                    inside = np.all((p >= lo - halo) & (p < hi + halo), axis=1)
                    if not sh.any():
                        inside &= ~np.all(cell == b, axis=1)
                    k = np.nonzero(inside)[0]
                    gidx.append(k)
                    gpos.append(p[k])
                gidx, gpos = np.concatenate(gidx), np.concatenate(gpos)
                if rng is not None:
                    pr = rng.permutation(len(gidx))
                    gidx, gpos = gidx[pr], gpos[pr]
                out.append({"coord": np.concatenate([x[own], gpos]),
                            "atype": np.concatenate([np.asarray(atype)[own], np.asarray(atype)[gidx]]).astype(np.int32),
                            "nlocal": len(own), "owner": np.concatenate([own, gidx])})
    return out


def ensemble_params(model: dict, base: np.ndarray, n_models: int, rel: float = 0.02, seed: int = 77):
    """Parameters of an ensemble of n_models members: the base parameters with every value
    multiplied by 1 + N(0, rel) (member 0 included), seeded. A stand-in for models trained from
    independent initialisations on the same data, whose predictions differ slightly."""
    rng = np.random.default_rng(seed)
    return [base * (1.0 + rng.normal(0.0, rel, base.size)) for _ in range(n_models)]


def water_params(seed: int = PARAM_SEED) -> np.ndarray:
    return make_params(WATER_MODEL, seed, WATER_OUT_SCALE, WATER_FIT_IN)


def water_r_params(seed: int = PARAM_SEED + 7) -> np.ndarray:
    return make_params(WATER_R_MODEL, seed, WATER_R_OUT_SCALE, WATER_R_FIT_IN)


def water_e3_params(seed: int = PARAM_SEED + 7) -> np.ndarray:
    return make_params(WATER_E3_MODEL, seed, WATER_E3_OUT_SCALE, WATER_E3_FIT_IN)


def fcc_params(seed: int = PARAM_SEED + 1) -> np.ndarray:
    return make_params(FCC_MODEL, seed, FCC_OUT_SCALE, FCC_FIT_IN)


def serve_params(seed: int = PARAM_SEED + 2) -> np.ndarray:
    return make_params(SERVE_MODEL, seed, SERVE_OUT_SCALE, SERVE_FIT_IN)
