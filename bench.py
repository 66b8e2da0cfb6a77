#!/usr/bin/env python
"""Benchmark: se_e2_a energy + forces + virial on the 12,288-atom water box, one MI355X.

One step = one full evaluation (neighbour list, embedding + contraction, fitting, adjoint, force
and virial reductions) of the whole frame, inputs resident in HBM. The FP64 path and the mixed
path (split-BF16 MFMA GEMMs, FP32 activations, FP64 geometry and sums) are timed back to back;
the JSON line's value is the mixed path's atom-steps/s, with the FP64 figures, the speedup and each
path's force error against the FP64 CPU oracle beside it.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X peaks used for the roofline fields: AMD's published dense figures, and the vector-ALU
# rate from the unit counts. All HIP code here is built with packed FP32 disabled, so the FP32
# vector peak is the non-packed one: 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz.
PEAK = {
    "hbm": 8000.0,          # GB/s
    "fp64": 78.6,           # TFLOP/s, FP64 matrix = FP64 vector
    "fp32_mfma": 157.3,     # TFLOP/s
    "bf16_mfma": 2500.0,    # TFLOP/s, dense
    "fp32_valu": 78.6,      # TFLOP/s, non-packed
}

# Algorithmic work per unit (the method's arithmetic on real, kept neighbours only; forward and
# input gradient, no weight gradients):
#   embedding net, per pair: 2 (25 + 25*50 + 50*100) = 12,550 flop forward; the input-gradient
#     pass needs the same products again (12,550) on top of the contraction's;
#   tabulated embedding, per pair: 100 features x 5 FMA for G (1,000 flop) and x 4 FMA for dG/ds
#     (800 flop) (the kernels reach the same result with less arithmetic, as products of the table
#     with per-interval moments; the fraction counts the method's work per second);
#   contraction, per pair: T += G^T R 800 flop, dE/dR = G dT and dE/dG . R 1,600 flop;
#   environment row and chain rule, per pair: about 50 flop (FP64);
#   fitting, per atom: D = T T_<^T 12,800 + dE/dT 25,600 + 2 x 2 (1600*240 + 2*240^2 + 240)
#     = 2,036,160 flop.
NET_PAIR, TAB_VAL_PAIR, TAB_DER_PAIR = 12550.0, 1000.0, 800.0
CONTRACT_FWD, CONTRACT_BWD, ENV_PAIR = 800.0, 1600.0, 50.0
FIT_ATOM = 2036160.0

# FP32 vector work per pair of the BF16-path network kernels (activations, derivatives, the
# contractions, the chain rule), a second view beside the matrix roofline, in FMA-equivalent flop
# (2 per issue slot). A tanh counts 10.5: calib/valu_rates.hip measures v_exp_f32 and v_rcp_f32 at
# about 1.8 FMA issue slots each on this device, not overlapped with FMA issue, and the whole
# tanh at 5.3 slots (profiles/valu_rates.md).
#   forward: layer 1 25 x (2 + 10.5 + 1) + layer 2 50 x (1 + 10.5 + 2) + layer 3 100 x (1 + 10.5 + 2 + 8)
#            = 3,162.5 flop
#   adjoint: layer 1 25 x (2 + 10.5 + 1 + 4) + layer 2 50 x (1 + 10.5 + 2 + 5)
#            + layer 3 100 x (1 + 10.5 + 2 + 5 + 8 + 8) + chain rule ~50 = 4,862.5 flop
VALU_FLOP_PER_PAIR = {"embed_fwd": 3162.5, "embed_bwd": 4862.5}

# End-to-end ceilings (atom-steps/s) of each workload and mode: the binding unit's time per
# atom-step from the algorithmic work above.
#   water FP64: 4.53 MFLOP at 78.6 TF -> 1.73e7; water mixed: about 16.6 k tanh + epilogues on the
#   vector ALU, BF16 matrix work 1.8 ns -> 1.6e8; water FP32: 4.27 MFLOP of dense GEMM at 157.3 TF
#   (27 ns) -> 3.7e7; fcc tabulated FP32: the fitting GEMM, 2.04 MFLOP at 157.3 TF -> 7.9e7;
#   fcc tabulated FP64: 2.62 MFLOP at 78.6 TF -> 3.0e7; fcc tabulated mixed: the table and
#   contraction on the vector ALU, 138 x 5,300 flop at 78.6 TF (9.3 ns; the split-BF16 fitting
#   needs 2.4 ns) -> 1.07e8.
CEILING = {("water", "fp64"): 1.73e7, ("water", "mixed"): 1.6e8, ("water", "fp32"): 3.7e7,
           ("water", "bf16"): 1.6e8, ("fcc_table", "fp32"): 7.9e7, ("fcc_table", "fp64"): 3.0e7,
           ("fcc_table", "mixed"): 1.07e8}


def matrix_peak(precision: str):
    return {"fp64": PEAK["fp64"], "fp32": PEAK["fp32_mfma"]}.get(precision, PEAK["bf16_mfma"])


def work_per_launch(stage: str, precision: str, natoms: int, npairs: int, nc: int, table: bool = False):
    """Algorithmic work of one launch of a stage and the peak of the unit it is priced against:
    (bound, amount, peak, unit). Network kernels and the fitting net against the matrix peak of
    the precision their GEMMs run in (split BF16: the BF16 peak, three products per algorithmic
    flop, so a saturated kernel would show 1/3); tabulated embedding kernels (no GEMM) against the
    vector peak of their precision; the neighbour list against HBM."""
    if stage == "nlist":
        bytes_ = natoms * (nc * 28 + 8 + 24 + 4)
        return "hbm", bytes_ / 1e9, PEAK["hbm"], "GB/s"
    if stage == "fit":
        return "mfma", FIT_ATOM * natoms / 1e12, matrix_peak(precision), "TFLOP/s"
    if table:
        # the forward pass needs G only; the adjoint needs G and dG/ds
        per = (TAB_VAL_PAIR + CONTRACT_FWD if stage == "embed_fwd" else TAB_VAL_PAIR + TAB_DER_PAIR + CONTRACT_BWD) + ENV_PAIR
        peak = PEAK["fp64"] if precision == "fp64" else PEAK["fp32_valu"]
        return "alu", per * npairs / 1e12, peak, "TFLOP/s"
    per = NET_PAIR + ENV_PAIR + (CONTRACT_FWD if stage == "embed_fwd" else CONTRACT_BWD)
    return "mfma", per * npairs / 1e12, matrix_peak(precision), "TFLOP/s"


def stage_rooflines(stage_ms: dict, precision: str, natoms: int, npairs: int, nc: int, table: bool = False):
    out = {}
    for st in ("nlist", "embed_fwd", "fit", "embed_bwd"):
        b_, a_, p_, u_ = work_per_launch(st, precision, natoms, npairs, nc, table)
        ach = a_ / (stage_ms[st] * 1e-3)
        out[st] = {"bound": b_, "achieved": ach, "peak": p_, "unit": u_, "frac": ach / p_, "ms": stage_ms[st]}
        if not table and precision in ("mixed", "bf16") and st in VALU_FLOP_PER_PAIR:
            v = VALU_FLOP_PER_PAIR[st] * npairs / 1e12 / (stage_ms[st] * 1e-3)
            out[st]["valu_view"] = {"achieved": v, "peak": PEAK["fp32_valu"], "unit": "TFLOP/s",
                                    "frac": v / PEAK["fp32_valu"]}
    return out


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_water12288.txt")
KERNEL_SOURCES = ("paper_2304_09409_amd/csrc/kernels_nn.hip", "paper_2304_09409_amd/csrc/kernels_geom.hip",
                  "paper_2304_09409_amd/csrc/dpk_internal.h", "paper_2304_09409_amd/csrc/kernels_fit.hip",
                  "paper_2304_09409_amd/csrc/kernels_tab.hip", "paper_2304_09409_amd/csrc/dpk_device.h")


def kernel_source_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def stored_traffic(stage: str, precision: str):
    """HBM bytes (read + written) per launch of a stage, from the stored counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a copy-kernel calibration); None when the summary is
    missing or the kernel sources have changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            lines = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    except OSError:
        return None
    digest = next((ln[1] for ln in lines if ln[0] == "source_sha256"), None)
    if digest != kernel_source_digest():
        return None
    for ln in lines:
        if ln[0] == "traffic" and ln[1] == precision and ln[2] == stage:
            return float(ln[3]) + float(ln[4])
    return None


FIXED_RATES = (2000, 4000, 6000)   # requests/s


def serving_bench(dpk, synth, n_sims=16, steps=64, slots=4, load=0.7, seed=2023, budget_frames=3.0):
    """Requests from n_sims concurrent simulations (sizes log-uniform in [50, 3000], 2-type 1:2 or
    3-type 2:1:1 frames at 0.1 atoms/A^3; consecutive frames of a simulation are small random
    displacements), round-robin over the simulations. After one untimed pass of all requests (the
    server's steady state: every slot's workspace has grown to the batches it serves), all requests
    at once (saturated throughput X, median of three passes), then Poisson arrivals at
    load * X / mean size; latency = completion - arrival.
    HBM budget: the model plus budget_frames times the workspace of the largest frame (admission
    limits batch sizes to what that holds). Python's garbage collector is paused during the timed
    loops: its pauses (tens of ms with torch loaded) belong to this client, not to the server."""
    import gc
    import math
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(math.log(50), math.log(3000), n_sims)).astype(int)
    kinds = rng.choice([2, 3], size=n_sims)
    sims = [synth.serving_frame(int(n), int(rng.integers(1 << 30)), int(k)) for n, k in zip(sizes, kinds)]
    reqs = []
    for step in range(steps):
        for sid, (c, t, b) in enumerate(sims):
            reqs.append((c + rng.normal(0.0, 0.01 * (step + 1) ** 0.5, c.shape), t, b, sid))
    model = dpk.Model(synth.SERVE_MODEL, synth.serve_params())
    probe = dpk.Context(model, precision="mixed")
    model_bytes = probe.stats()["workspace_bytes"]
    big = max(probe.workspace_bytes(len(t)) for _, t, _ in sims) - model_bytes
    probe.close()
    budget = int(model_bytes + budget_frames * big)
    total_atoms = sum(len(r[1]) for r in reqs)
    srv = dpk.Server(model, precision="mixed", nslots=slots, budget_bytes=budget)
    # warm-up: one pass of every request (a workspace that grows waits for the device)
    for tk in [srv.submit(c, t, b, simulation=sid) for c, t, b, sid in reqs]:
        tk.result()
    gc.collect()
    gc.disable()
    try:
        return _serving_timed(srv, sims, reqs, rng, load, slots, budget, n_sims)
    finally:
        gc.enable()


def _serving_timed(srv, sims, reqs, rng, load, slots, budget, n_sims):
    total_atoms = sum(len(r[1]) for r in reqs)
    s0 = srv.stats()
    rates = []
    for _ in range(3):   # a pass lasts tens of ms: the median of three
        t0 = time.monotonic_ns()
        tickets = [srv.submit(c, t, b, simulation=sid) for c, t, b, sid in reqs]
        for tk in tickets:
            tk.result()
        t1 = time.monotonic_ns()
        rates.append(total_atoms / ((t1 - t0) * 1e-9))
    s1 = srv.stats()
    x_sat = float(np.median(rates))
    mean_n = total_atoms / len(reqs)
    lam = load * x_sat / mean_n
    gaps = rng.exponential(1.0 / lam, len(reqs))
    arrivals = np.cumsum(gaps)
    start = time.monotonic_ns() + 2_000_000
    tickets, when = [], []
    for (c, t, b, sid), a in zip(reqs, arrivals):
        due = start + int(a * 1e9)
        while time.monotonic_ns() < due:
            pass
        tickets.append(srv.submit(c, t, b, simulation=sid))
        when.append(due)
    lat = []
    last = 0
    records = []
    for (c, t, b, sid), tk, due in zip(reqs, tickets, when):
        tk.result()
        ts = srv.times(tk)
        done = int(ts[2])
        lat.append((done - due) * 1e-6)
        last = max(last, done)
        records.append({"simulation": int(sid), "atoms": int(len(t)), "arrival_ns": int(due), "submit_ns": int(ts[0]),
                        "start_ns": int(ts[1]), "done_ns": done, "latency_ms": (done - due) * 1e-6})
    st = srv.stats()
    # latency against fixed Poisson arrival rates (the saturated rate X above is measured with
    # every request queued, i.e. the largest batches; Poisson arrivals batch less)
    fixed = {}
    for rate in FIXED_RATES:
        arr = np.cumsum(rng.exponential(1.0 / rate, len(reqs)))
        t_start = time.monotonic_ns() + 2_000_000
        tks, dues = [], []
        for (c, t, b, sid), a in zip(reqs, arr):
            due = t_start + int(a * 1e9)
            while time.monotonic_ns() < due:
                pass
            tks.append(srv.submit(c, t, b, simulation=sid))
            dues.append(due)
        lf = []
        for tk, due in zip(tks, dues):
            tk.result()
            lf.append((int(srv.times(tk)[2]) - due) * 1e-6)
        lf = np.array(lf)
        fixed[str(rate)] = {"p50_ms": float(np.percentile(lf, 50)), "p90_ms": float(np.percentile(lf, 90)),
                            "p99_ms": float(np.percentile(lf, 99))}
    srv.close()
    lat = np.array(lat)
    batch_sat = (s1["completed"] - s0["completed"]) / max(1, s1["launches"] - s0["launches"])
    batch_poisson = (st["completed"] - s1["completed"]) / max(1, st["launches"] - s1["launches"])
    return {"requests": len(reqs), "simulations": n_sims, "slots": slots, "budget_bytes": budget,
            "mean_atoms": mean_n, "saturated_atom_steps_per_s": x_sat, "load": load,
            "arrival_rate_req_per_s": lam, "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "max_ms": float(lat.max()),
            "throughput_atom_steps_per_s": total_atoms / ((last - start) * 1e-9),
            "peak_bytes": st["peak_bytes"], "budget_waits": st["budget_waits"],
            "slot_reuse": st["slot_reuse"], "fixed_rate_latency": fixed, "mean_batch_saturated": batch_sat,
            "mean_batch_poisson": batch_poisson, "precision": "mixed", "_records": records}


def time_frame(dpk, torch, model, prec, c, t, b, steps, warmup, median_of=0):
    """Device-resident timing of one frame: warm-up, then `steps` evaluations back to back (mean
    ms/step; no events between the stages), then as many again with the stage profiler on (its
    events between the stages cost a few microseconds each: the stage times and the kernel
    rooflines come from this second loop); with median_of > 0 also that many single synchronised
    evaluations (median ms). Returns the result dict and the context (caller closes it)."""
    n = len(t)
    dev = torch.device("cuda:0")
    coord = torch.tensor(c, dtype=torch.float64, device=dev)
    atype = torch.tensor(t, dtype=torch.int32, device=dev)
    energy = torch.zeros(1, dtype=torch.float64, device=dev)
    force = torch.zeros((n, 3), dtype=torch.float64, device=dev)
    virial = torch.zeros(9, dtype=torch.float64, device=dev)
    ctx = dpk.Context(model, precision=prec)
    for _ in range(warmup):
        ctx.compute_device(coord, atype, b, energy, force, virial)
    ctx.check()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.compute_device(coord, atype, b, energy, force, virial)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.profile(True)
    for _ in range(steps):
        ctx.compute_device(coord, atype, b, energy, force, virial)
    torch.cuda.synchronize()
    stage_ms, nframes = ctx.profile_read()
    ctx.profile(False)
    ctx.check()
    ms = (t1 - t0) * 1e3 / steps
    out = dict(ms_per_step=ms, value=n / (ms * 1e-3), stage_ms={k: v / nframes for k, v in stage_ms.items()},
               stats=ctx.stats())
    if median_of:
        single = []
        for _ in range(median_of):
            torch.cuda.synchronize()
            ts = time.perf_counter()
            ctx.compute_device(coord, atype, b, energy, force, virial)
            torch.cuda.synchronize()
            single.append((time.perf_counter() - ts) * 1e3)
        ctx.check()
        out["median_ms"] = float(np.median(single))
        out["median_value"] = n / (out["median_ms"] * 1e-3)
    out["force"] = force.cpu().numpy().copy()
    out["energy"] = float(energy.item())
    out["virial"] = virial.cpu().numpy().reshape(3, 3).copy()
    out["_inputs"] = (coord, atype, energy, force, virial)
    return out, ctx


# The same derivation with a tanh at its measured cost (5.3 vector issue slots, calib/valu_rates.hip)
# instead of the 11 assumed above: 16.6 k tanh per atom-step plus the epilogues, about 3.9 ns per
# atom-step on the vector ALU. Reported beside the ceiling above, never in its place.
CEILING_CALIBRATED = {("water", "mixed"): 2.6e8, ("water", "bf16"): 2.6e8}


def e2e(workload: str, prec: str, value: float):
    ceil = CEILING.get((workload, prec))
    if ceil is None:
        return None
    out = {"ceiling": ceil, "unit": "atom-steps/s", "frac": value / ceil}
    cal = CEILING_CALIBRATED.get((workload, prec))
    if cal is not None:
        out["calibrated"] = {"ceiling": cal, "frac": value / cal}
    return out


def public(run: dict, keep=("ms_per_step", "value", "median_ms", "median_value", "stage_ms")):
    return {k: run[k] for k in keep if k in run}


def tabulated_bench(dpk, synth, torch, steps, warmup, precisions):
    """The 32,000-atom fcc box (20^3 cells, rc 8.0 A, sel 138) with the tabulated embedding (stride
    0.01): ms/step, atom-steps/s, stage times and stage rooflines per precision. Its parity with
    the oracle's table is tested at this size; here it is timed only."""
    c, t, b = synth.fcc_32000()
    n = len(t)
    model = dpk.Model(synth.FCC_MODEL, synth.fcc_params()).tabulate(0.01, 0.5)
    out = {"workload": "fcc metal, 32,000 atoms (20^3 cells, a 3.6 A, jitter 0.05 A), periodic; se_e2_a rc 8.0 A, "
                       "rc_smth 2.0 A, sel [138], tabulated embedding (stride 0.01), fitting (240,240,240,1)",
           "atoms": n}
    npairs = None
    for prec in precisions:
        r, ctx = time_frame(dpk, torch, model, prec, c, t, b, steps, warmup)
        if npairs is None:
            npairs = int((ctx.debug_nlist(n) >= 0).sum())
            out["neighbour_pairs"] = npairs
        ctx.close()
        out[prec] = public(r)
        out[prec]["neighbours_dropped_by_sel"] = r["stats"]["nbr_dropped"]
        out[prec]["stage_roofline"] = stage_rooflines(r["stage_ms"], prec, n, npairs, model.nc, table=True)
        out[prec]["e2e_roofline"] = e2e("fcc_table", prec, r["value"])
        print(f"# tabulated fcc32000 {prec}: {r['ms_per_step']:.3f} ms/step, {r['value']:.4g} atom-steps/s, stages (ms) "
              + ", ".join(f"{k} {v:.3f}" for k, v in r["stage_ms"].items()), file=sys.stderr, flush=True)
    return out


def large_bench(dpk, synth, torch, precisions, median_of=10):
    """The 110,592-atom water box (36,864 molecules at water density, 103.38 A): median of
    `median_of` synchronised evaluations per precision, with stage times."""
    c, t, b = synth.water_110592()
    n = len(t)
    model = dpk.Model(synth.WATER_MODEL, synth.water_params())
    out = {"workload": "water-like box, 110,592 atoms (36,864 molecules), cubic 103.38 A periodic, water model",
           "atoms": n}
    for prec in precisions:
        r, ctx = time_frame(dpk, torch, model, prec, c, t, b, 3, 2, median_of=median_of)
        ctx.close()
        out[prec] = public(r)
        out[prec]["e2e_roofline"] = e2e("water", prec, r["median_value"])
        print(f"# water110592 {prec}: median {r['median_ms']:.3f} ms/step, {r['median_value']:.4g} atom-steps/s",
              file=sys.stderr, flush=True)
    return out


# Work per unit of the other DeepPot-SE descriptors (forward and input gradient):
#   se_e2_r, per neighbour: the embedding net 12,550 flop each way; contraction D_m += s G_m 200,
#     dE/dG . s and G . dD 400; environment row and chain rule 50; fitting per atom
#     2 x 2 (100*240 + 2*240^2 + 240) = 557,760 flop.
#   se_e3, per ordered neighbour pair (j, k), j = k included: theta 7 flop, the net 12,550 each way,
#     D_m += theta G_m 200, dE/dtheta 400, the two row gradients 16; per neighbour the chain rule
#     50; the same fitting as se_e2_r.
FIT_ATOM_M = 557760.0
E3_PAIR_FWD, E3_PAIR_BWD = NET_PAIR + 207.0, NET_PAIR + 416.0
R_PAIR_FWD, R_PAIR_BWD = NET_PAIR + 250.0, NET_PAIR + 450.0


def descriptor_bench(dpk, synth, torch, steps, warmup, precisions):
    """se_e2_r (rc 6.0 A, sel [46, 92]) and se_e3 (rc 4.0 A, sel [20, 40]) on the 12,288-atom water
    box: ms/step, atom-steps/s, stage times, and the embedding and fitting stages against the
    matrix peak of their precision (work per launch from the counts above: neighbours for se_e2_r,
    ordered neighbour pairs for se_e3). Parity at this size is tested (test_gpu_descriptors.py)."""
    c, t, b = synth.water_12288()
    n = len(t)
    out = {}
    for name, spec, params in (("se_e2_r", synth.WATER_R_MODEL, synth.water_r_params),
                               ("se_e3", synth.WATER_E3_MODEL, synth.water_e3_params)):
        model = dpk.Model(spec, params())
        res = {"workload": f"water-like box, 12,288 atoms; {name} rc {spec['rcut']} A, sel {spec['sel']}, "
                           "embedding (25,50,100), fitting (240,240,240,1)", "atoms": n}
        units = None
        for prec in precisions:
            r, ctx = time_frame(dpk, torch, model, prec, c, t, b, steps, warmup)
            if units is None:
                kept = (ctx.debug_nlist(n) >= 0).sum(axis=1).astype(np.int64)
                units = int(kept.sum()) if name == "se_e2_r" else int((kept ** 2).sum())
                res["neighbours" if name == "se_e2_r" else "neighbour_pairs_jk"] = units
                res["neighbours_total"] = int(kept.sum())
            ctx.close()
            fw, bw = (R_PAIR_FWD, R_PAIR_BWD) if name == "se_e2_r" else (E3_PAIR_FWD, E3_PAIR_BWD)
            chain = 0.0 if name == "se_e2_r" else ENV_PAIR * res["neighbours_total"]
            work = {"embed_fwd": fw * units, "fit": FIT_ATOM_M * n, "embed_bwd": bw * units + chain}
            roof = {}
            for st, w in work.items():
                ach = w / 1e12 / (r["stage_ms"][st] * 1e-3)
                pk = matrix_peak(prec)
                roof[st] = {"bound": "mfma", "achieved": ach, "peak": pk, "unit": "TFLOP/s", "frac": ach / pk,
                            "ms": r["stage_ms"][st]}
            res[prec] = dict(public(r), stage_roofline=roof)
            print(f"# {name} water12288 {prec}: {r['ms_per_step']:.3f} ms/step, {r['value']:.4g} atom-steps/s, "
                  "stages (ms) " + ", ".join(f"{k} {v:.3f}" for k, v in r["stage_ms"].items()),
                  file=sys.stderr, flush=True)
        out[name] = res
    return out


def next_rows_bench(dpk, synth, reps=10):
    """Model deviation (Sec. II.C) and one domain of a spatial decomposition with ghost atoms
    (Sec. III.B.2), through their host-buffer entry points (synchronous, host-to-device and
    device-to-host copies included, so the rates are lower bounds of device-resident ones); medians
    of `reps` calls after one warm-up call, each beside the same model's single-frame host-buffer
    time. Parity of both is tested (test_gpu_devi.py, test_gpu_ghost.py)."""
    out = {}
    med = lambda f: float(np.median([_wall_ms(f) for _ in range(reps)]))
    # model deviation: four members (perturbed water parameters) on the 12,288-atom box
    c, t, b = synth.water_12288()
    n = len(t)
    nm = 4
    models = [dpk.Model(synth.WATER_MODEL, p) for p in synth.ensemble_params(synth.WATER_MODEL, synth.water_params(), nm)]
    res = {"workload": f"water-like box, 12,288 atoms; {nm} se_e2_a water models (parameters x (1 + N(0, 0.02)))",
           "atoms": n, "models": nm, "entry_point": "dpk_devi_compute (host buffers)"}
    for prec in ("mixed", "fp64"):
        dv = dpk.Deviation(models, precision=prec)
        dv.compute(c, t, b)
        ms = med(lambda: dv.compute(c, t, b))
        dv.close()
        ctx = dpk.Context(models[0], precision=prec)
        ctx.compute(c, t, b)
        one = med(lambda: ctx.compute(c, t, b))
        ctx.close()
        res[prec] = {"ms": ms, "model_atom_steps_per_s": nm * n / (ms * 1e-3), "single_model_ms": one,
                     "vs_separate_models": ms / (nm * one)}
        print(f"# model deviation ({nm} models) water12288 {prec}: {ms:.3f} ms per frame "
              f"({res[prec]['model_atom_steps_per_s']:.4g} model-atom-steps/s; one model {one:.3f} ms, "
              f"ensemble / {nm} separate evaluations {res[prec]['vs_separate_models']:.2f})",
              file=sys.stderr, flush=True)
    out["model_deviation"] = res
    # one brick of eight of the 110,592-atom box, with the ghosts within r_c of it
    c, t, b = synth.water_110592()
    br = synth.ghost_bricks(c, t, b, (2, 2, 2), halo=synth.WATER_MODEL["rcut"])[0]
    nl, ntot = int(br["nlocal"]), len(br["atype"])
    model = dpk.Model(synth.WATER_MODEL, synth.water_params())
    res = {"workload": "one of 2 x 2 x 2 bricks of the 110,592-atom water box (51.7 A cube), ghosts within "
                       "r_c = 6 A", "owned": nl, "ghosts": ntot - nl, "entry_point": "dpk_compute_ghost (host buffers)"}
    for prec in ("mixed", "fp64"):
        ctx = dpk.Context(model, precision=prec)
        ctx.compute_ghost(br["coord"], br["atype"], nl)
        ms = med(lambda: ctx.compute_ghost(br["coord"], br["atype"], nl))
        ctx.close()
        res[prec] = {"ms": ms, "owned_atom_steps_per_s": nl / (ms * 1e-3)}
        print(f"# ghost brick ({nl} owned + {ntot - nl} ghosts) {prec}: {ms:.3f} ms per frame "
              f"({res[prec]['owned_atom_steps_per_s']:.4g} owned atom-steps/s)", file=sys.stderr, flush=True)
    out["ghost_domain"] = res
    return out


def _wall_ms(f):
    t0 = time.perf_counter()
    f()
    return (time.perf_counter() - t0) * 1e3


# Training step (Sec. II.B) per frame, FP64: inference (embedding with its unit tangent 2 x 12,550
# flop per pair, pair forces 1,600; fitting forward and input gradient 2 x 998,400 per atom), the
# training pass (fitting forward with tangent 2 x 998,400, reverse of values and tangents
# 2 x 998,400, weight gradients 2 x 998,400 per atom; embedding reverse 2 x 12,550 and weight
# gradients 2 x 12,550 per pair; contraction with tangent about 3,200 per pair).
TRAIN_PAIR = 4 * NET_PAIR + 2 * NET_PAIR + 1600.0 + 3200.0
TRAIN_ATOM = 8 * 998400.0


def training_bench(dpk, synth, steps):
    """One training step on the 12,288-atom water box: the frame's loss and full parameter gradient
    (energy, force and virial terms) through dpk_trainer_accumulate, then an Adam step; the time of
    the whole step (host copies and the host-side pair list included), against the FP64 peak."""
    c, t, b = synth.water_12288()
    n = len(t)
    # synthetic labels: a perturbed model's prediction (outside the timed loop)
    params = synth.water_params()
    p2 = synth.ensemble_params(synth.WATER_MODEL, params, 2, rel=0.05, seed=5)[1]
    lctx = dpk.Context(dpk.Model(synth.WATER_MODEL, p2), precision="fp64")
    ref = lctx.compute(c, t, b)
    lctx.close()
    tr = dpk.Trainer(dpk.Model(synth.WATER_MODEL, params))
    kw = dict(energy=ref["energy"], force=ref["force"], virial=ref["virial"], pe=0.02, pf=1000.0, pv=0.02)
    r = tr.accumulate(c, t, b, **kw)
    tr.adam_step(1e-3)
    ts = time.perf_counter()
    losses = []
    for _ in range(steps):
        r = tr.accumulate(c, t, b, **kw)
        tr.adam_step(1e-3)
        losses.append(r["loss"])
    ms = (time.perf_counter() - ts) * 1e3 / steps
    tr.close()
    npairs = None
    try:
        m = dpk.Model(synth.WATER_MODEL, params)
        ctx = dpk.Context(m, precision="fp64")
        ctx.compute(c, t, b)
        npairs = int((ctx.debug_nlist(n) >= 0).sum())
        ctx.close()
    except Exception:
        pass
    work = (TRAIN_PAIR * npairs + TRAIN_ATOM * n) / 1e12 if npairs else None
    out = {"workload": "water-like box, 12,288 atoms, water model; loss with energy, force and virial terms; "
                       "FP64 gradient of every parameter + Adam step",
           "atoms": n, "neighbour_pairs": npairs, "ms_per_step": ms, "frames_per_s": 1e3 / ms,
           "loss_first_last": [losses[0], losses[-1]]}
    if work:
        out["roofline"] = {"bound": "fp64", "achieved": work / (ms * 1e-3), "peak": PEAK["fp64"], "unit": "TFLOP/s",
                           "frac": work / (ms * 1e-3) / PEAK["fp64"]}
    print(f"# training water12288: {ms:.2f} ms/step, loss {losses[0]:.4g} -> {losses[-1]:.4g}", file=sys.stderr,
          flush=True)
    return out


def host_cpu():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": usable, "logical_cpus": os.cpu_count()}


def cpu_baseline(synth, c, t, b):
    """The FP64 oracle (test infrastructure, never tuned) on the host: the full 12,288-atom frame
    once on all threads (also the reference of the force errors), and the 192-atom box on one
    thread. A bounded sample: about 1-3 s of CPU work."""
    from oracle import Oracle
    o = Oracle(synth.WATER_MODEL, synth.water_params())
    threads = o.threads()
    ts = time.perf_counter()
    ref = o.compute(c, t, b)
    full = time.perf_counter() - ts
    c0, t0, b0 = synth.water_192()
    o.set_threads(1)
    reps, el = 0, 0.0
    while reps < 20 and (reps == 0 or el < 1.0):
        ts = time.perf_counter()
        o.compute(c0, t0, b0)
        el += time.perf_counter() - ts
        reps += 1
    o.set_threads(threads)
    info = host_cpu()
    cpu = {"value": len(t) / full, "unit": "atom-steps/s", "cores": threads, "kind": "oracle",
           "sample": f"the full 12,288-atom frame (E+F+virial) once on {threads} OpenMP threads, {full:.2f} s",
           "single_thread": {"value": len(t0) * reps / el, "unit": "atom-steps/s",
                             "sample": f"the 192-atom water box, {reps} evaluations on 1 thread, {el:.2f} s"},
           **info}
    return cpu, ref


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving (latency) section")
    ap.add_argument("--no-table", action="store_true", help="skip the tabulated-embedding (fcc) section")
    ap.add_argument("--no-large", action="store_true", help="skip the 110,592-atom water box")
    ap.add_argument("--no-descriptors", action="store_true", help="skip the se_e2_r / se_e3 section")
    ap.add_argument("--no-train", action="store_true", help="skip the training-step section")
    ap.add_argument("--no-next", action="store_true", help="skip the model-deviation and ghost-domain section")
    ap.add_argument("--requests-log", default=None,
                    help="write one JSON record per served request of the Poisson phases to this file")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 256 MiB device-to-device (the reference for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; multi-GPU runs are not part of it "
              "(use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2304_09409_amd import dpk, synth

    if args.copy_calibration:
        src = torch.ones(1 << 25, dtype=torch.float64, device="cuda")   # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    c, t, b = synth.water_12288()
    n = len(t)
    model = dpk.Model(synth.WATER_MODEL, synth.water_params())
    runs = {}
    npairs = None
    for prec in PRECISIONS_TIMED:
        r, ctx = time_frame(dpk, torch, model, prec, c, t, b, args.steps, args.warmup)
        if npairs is None:
            npairs = int((ctx.debug_nlist(n) >= 0).sum())
        print(f"# {prec}: {r['ms_per_step']:.3f} ms/step, {r['value']:.4g} atom-steps/s, stages (ms) "
              + ", ".join(f"{k} {v:.3f}" for k, v in r["stage_ms"].items()), file=sys.stderr, flush=True)
        # the same frame through the host-buffer entry point (synchronous; host-to-device and
        # device-to-host copies included): reported beside the device-resident rate, never as it
        ctx.compute(c, t, b)
        hreps = max(3, args.steps // 4)
        t0 = time.perf_counter()
        for _ in range(hreps):
            ctx.compute(c, t, b)
        r["host_buffer_ms_per_step"] = (time.perf_counter() - t0) * 1e3 / hreps
        print(f"# {prec}: host-buffer entry point {r['host_buffer_ms_per_step']:.3f} ms/step",
              file=sys.stderr, flush=True)
        ctx.close()
        runs[prec] = r

    large = None if args.no_large else large_bench(dpk, synth, torch, ("fp64", "mixed"))
    tabulated = None if args.no_table else tabulated_bench(dpk, synth, torch, max(1, args.steps // 2),
                                                            max(1, args.warmup // 2), TABLE_PRECISIONS)
    descriptors = None if args.no_descriptors else descriptor_bench(dpk, synth, torch, max(1, args.steps // 2),
                                                                    max(1, args.warmup // 2), ("fp64", "mixed", "fp32"))
    training = None if args.no_train else training_bench(dpk, synth, max(2, args.steps // 4))
    next_rows = None if args.no_next else next_rows_bench(dpk, synth)
    # two operating points of the same server: the latency point (four slots, a budget of three
    # of the largest frame's workspaces, which binds) and a throughput point (four slots, 48
    # workspaces: batches grow to the scheduler's 12,288-atom target)
    serving = None if args.no_serving else serving_bench(dpk, synth)
    if serving:
        serving["throughput_point"] = serving_bench(dpk, synth, slots=4, budget_frames=48.0)
        # per-request records (arrival, submission, start on the device, completion): to a file if
        # asked for, never into the JSON line
        recs = [("latency", serving.pop("_records")), ("throughput", serving["throughput_point"].pop("_records"))]
        if args.requests_log:
            with open(args.requests_log, "w") as fh:
                for point, rr in recs:
                    for r in rr:
                        fh.write(json.dumps(dict(point=point, **r)) + "\n")
        for name, sv in (("serving", serving), ("serving (throughput point)", serving["throughput_point"])):
            print(f"# {name}: p50 {sv['p50_ms']:.3f} ms, p99 {sv['p99_ms']:.3f} ms at "
                  f"{sv['arrival_rate_req_per_s']:.0f} req/s; saturated {sv['saturated_atom_steps_per_s']:.4g} "
                  f"atom-steps/s; mean batch {sv['mean_batch_saturated']:.1f} (saturated), "
                  f"{sv['mean_batch_poisson']:.1f} (Poisson), budget waits {sv['budget_waits']}; fixed rates: "
                  + ", ".join(f"{k} req/s p50 {v['p50_ms']:.3f} p99 {v['p99_ms']:.3f} ms"
                              for k, v in sv["fixed_rate_latency"].items()),
                  file=sys.stderr, flush=True)

    cpu, errs = None, {}
    if not args.no_cpu:
        cpu, ref = cpu_baseline(synth, c, t, b)
        for prec, r in runs.items():
            d = r["force"] - ref["force"]
            errs[prec] = {"max_abs_force_err": float(np.abs(d).max()),
                          "rms_force_err": float(np.sqrt((d ** 2).mean())),
                          "energy_err_per_atom": abs(r["energy"] - ref["energy"]) / n,
                          "max_virial_err_per_atom": float(np.abs(r["virial"] - ref["virial"]).max()) / n}
        errs["rms_force"] = float(np.sqrt((ref["force"] ** 2).mean()))

    head = runs["mixed"]
    stage_roof = {p: stage_rooflines(r["stage_ms"], p, n, npairs, model.nc) for p, r in runs.items()}
    kernel_stages = ("nlist", "embed_fwd", "fit", "embed_bwd")
    dom = max(kernel_stages, key=lambda k: head["stage_ms"][k])
    sr = stage_roof["mixed"][dom]
    roof = {"kernel": dom, "bound": sr["bound"], "achieved": sr["achieved"], "peak": sr["peak"], "unit": sr["unit"],
            "frac": sr["frac"], "traffic": stored_traffic(dom, "mixed")}
    if "valu_view" in sr:
        roof["valu_view"] = sr["valu_view"]
    others = {}
    for p, r in runs.items():
        if p == "mixed":
            continue
        d = max(kernel_stages, key=lambda k: r["stage_ms"][k])
        q = stage_roof[p][d]
        others[p] = dict(public(r), host_buffer_ms_per_step=r["host_buffer_ms_per_step"],
                         roofline={"kernel": d, "bound": q["bound"], "achieved": q["achieved"], "peak": q["peak"],
                                   "unit": q["unit"], "frac": q["frac"], "traffic": stored_traffic(d, p)},
                         e2e_roofline=e2e("water", p, r["value"]))

    line = {
        "metric": "atom-steps/s (E+F+virial) mixed vs FP64 at stated force error; p50/p99 latency",
        "value": head["value"],
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3-mfma/f32/f64",
        "data": "synthetic",
        "config": {"workload": "water-like box, 12,288 atoms (4,096 molecules), cubic 49.7 A periodic; "
                               "se_e2_a rc 6.0 A, rc_smth 0.5 A, sel [46,92], embedding (25,50,100), "
                               "M_< 16, fitting (240,240,240,1), 2 types",
                   "atoms": n, "neighbour_pairs": npairs, "mode": "mixed"},
        "roofline": roof,
        "e2e_roofline": e2e("water", "mixed", head["value"]),
        "cpu_baseline": cpu,
        "mixed_stage_ms": head["stage_ms"],
        "host_buffer_ms_per_step": {p: runs[p]["host_buffer_ms_per_step"] for p in runs},
        "speedup_mixed_vs_fp64": head["value"] / runs["fp64"]["value"],
        "force_error_vs_oracle": errs or None,
        "stage_roofline": stage_roof,
        "large_frame": large,
        "tabulated": tabulated,
        "descriptors": descriptors,
        "training": training,
        "model_deviation": None if next_rows is None else next_rows["model_deviation"],
        "ghost_domain": None if next_rows is None else next_rows["ghost_domain"],
        "serving": serving,
    }
    line.update(others)
    print(json.dumps(line))


PRECISIONS_TIMED = ("fp64", "mixed", "fp32")
TABLE_PRECISIONS = ("mixed", "fp32", "fp64")

if __name__ == "__main__":
    main()
