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

# Published MI355X peaks (dense) used for the roofline fields.
PEAK = {
    "hbm": 8000.0,          # GB/s
    "fp64_mfma": 78.6,      # TFLOP/s
    "bf16_mfma": 2500.0,    # TFLOP/s
    "fp32_valu": 157.3,     # TFLOP/s (256 CU x 4 SIMD x 16 lanes x 2 flop x 2 (packed) x 2.4 GHz)
}

# Algorithmic FP32 vector work per real neighbour pair of the BF16-path embedding kernels (the
# GEMMs of layers 2 and 3 run on the matrix cores and are not counted here). tanh is counted as
# 6 flop (scale, exp, add, reciprocal, fused multiply-add), an FMA as 2.
#   forward: layer 1 25 x (2 pre + 6 tanh + 1 scale) + layer 2 50 x (1 bias + 6 + 2 skip)
#            + layer 3 100 x (1 + 6 + 2 + 8 for T += G R)                         = 2,375 flop
#   adjoint: layer 1 25 x (2 + 6 + 1 + 4 derivative) + layer 2 50 x (1 + 6 + 2 + 5)
#            + layer 3 100 x (1 + 6 + 2 + 5 + 8 dE/dR + 8 dE/ds) + chain rule ~50  = 4,075 flop
VALU_FLOP_PER_PAIR = {"embed_fwd": 2375.0, "embed_bwd": 4075.0}


def work_per_launch(stage: str, precision: str, natoms: int, npairs: int, nc: int):
    """Algorithmic work of one launch of a stage against the unit that bounds it: (bound, amount,
    peak, unit).

    Matrix work per real neighbour pair: embedding layers 2 + 3 = 2 (25*50 + 50*100) = 12,500
    flop, layer 1 50 flop, contraction G^T R 800 flop. The forward kernel computes G once (13,350
    flop per pair); the adjoint re-evaluates G and dG/ds (25,100), then dE/dR = G dT and (dG/ds)
    dT (1,600) and the chain rule (~50): 26,750 flop per pair. Fitting per atom: D = T T_<^T
    12,800, forward 2 (1600*240 + 2*240^2 + 240) = 998,880, input gradient 2 (1600*240 +
    2*240^2) = 998,400, dT 25,600: 2,035,680 flop. The neighbour list moves, per atom, the
    coordinates of the candidates it reads once (24 B x 27 bins' atoms is served from cache) and
    writes its list: N_c (4 B index + 24 B vector) + the per-type counts.

    FP64 path: every stage is priced against the FP64 matrix peak. BF16 paths: the fitting net
    against the BF16 matrix peak (each FP32-accurate product is three BF16 products, so a
    saturated kernel shows 1/3); the embedding kernels are bound by the vector ALU (the
    activations and their derivatives; counters show the VALU far busier than the matrix cores)
    and are priced by VALU_FLOP_PER_PAIR against the FP32 vector peak."""
    if stage == "embed_fwd":
        flops = 13350.0 * npairs
    elif stage == "embed_bwd":
        flops = 26750.0 * npairs
    elif stage == "fit":
        flops = 2035680.0 * natoms
    else:
        bytes_ = natoms * (nc * 28 + 8 + 24 + 4)
        return "hbm", bytes_ / 1e9, PEAK["hbm"], "GB/s"
    if precision == "fp64":
        return "mfma", flops / 1e12, PEAK["fp64_mfma"], "TFLOP/s"
    if stage in VALU_FLOP_PER_PAIR:
        return "alu", VALU_FLOP_PER_PAIR[stage] * npairs / 1e12, PEAK["fp32_valu"], "TFLOP/s"
    return "mfma", flops / 1e12, PEAK["bf16_mfma"], "TFLOP/s"


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_water12288.txt")
KERNEL_SOURCES = ("paper_2304_09409_amd/csrc/kernels_nn.hip", "paper_2304_09409_amd/csrc/kernels_geom.hip",
                  "paper_2304_09409_amd/csrc/dpk_internal.h", "paper_2304_09409_amd/csrc/kernels_fit.hip")


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


def serving_bench(dpk, synth, n_sims=16, steps=16, slots=4, load=0.7, seed=2023, budget_frames=8.0):
    """Requests from n_sims concurrent simulations (sizes log-uniform in [50, 3000], 2-type 1:2 or
    3-type 2:1:1 frames at 0.1 atoms/A^3; consecutive frames of a simulation are small random
    displacements), round-robin over the simulations. First all requests at once (saturated
    throughput X, median of three passes), then Poisson arrivals at load * X / mean size;
    latency = completion - arrival.
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
    # warm-up: one frame per simulation
    for tk in [srv.submit(c, t, b, simulation=sid) for sid, (c, t, b) in enumerate(sims)]:
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
    for tk, due in zip(tickets, when):
        tk.result()
        done = int(srv.times(tk)[2])
        lat.append((done - due) * 1e-6)
        last = max(last, done)
    st = srv.stats()
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
            "slot_reuse": st["slot_reuse"], "mean_batch_saturated": batch_sat,
            "mean_batch_poisson": batch_poisson, "precision": "mixed"}


def tabulated_bench(dpk, synth, torch, steps, warmup):
    """The 32,000-atom fcc box (20^3 cells, rc 8.0 A, sel 138) with the tabulated embedding (stride
    0.01): ms/step, atom-steps/s and stage times of the mixed and FP64 paths. Its parity with the
    oracle's table is tested at this size; here it is timed only."""
    c, t, b = synth.fcc_32000()
    n = len(t)
    model = dpk.Model(synth.FCC_MODEL, synth.fcc_params()).tabulate(0.01, 0.5)
    dev = torch.device("cuda:0")
    coord = torch.tensor(c, dtype=torch.float64, device=dev)
    atype = torch.tensor(t, dtype=torch.int32, device=dev)
    energy = torch.zeros(1, dtype=torch.float64, device=dev)
    force = torch.zeros((n, 3), dtype=torch.float64, device=dev)
    virial = torch.zeros(9, dtype=torch.float64, device=dev)
    out = {"workload": "fcc metal, 32,000 atoms (20^3 cells, a 3.6 A, jitter 0.05 A), periodic; se_e2_a rc 8.0 A, "
                       "rc_smth 2.0 A, sel [138], tabulated embedding (stride 0.01), fitting (240,240,240,1)",
           "atoms": n}
    for prec in ("mixed", "fp64"):
        ctx = dpk.Context(model, precision=prec)
        for _ in range(warmup):
            ctx.compute_device(coord, atype, b, energy, force, virial)
        ctx.check()
        torch.cuda.synchronize()
        ctx.profile(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.compute_device(coord, atype, b, energy, force, virial)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        stage_ms, nframes = ctx.profile_read()
        ctx.profile(False)
        ctx.check()
        ms = (t1 - t0) * 1e3 / steps
        out[prec] = {"ms_per_step": ms, "value": n / (ms * 1e-3),
                     "stage_ms": {k: v / nframes for k, v in stage_ms.items()},
                     "neighbours_dropped_by_sel": ctx.stats()["nbr_dropped"]}
        print(f"# tabulated fcc32000 {prec}: {ms:.3f} ms/step, {n / (ms * 1e-3):.4g} atom-steps/s, stages (ms) "
              + ", ".join(f"{k} {v:.3f}" for k, v in out[prec]["stage_ms"].items()), file=sys.stderr, flush=True)
        ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving (latency) section")
    ap.add_argument("--no-table", action="store_true", help="skip the tabulated-embedding (fcc) section")
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
    dev = torch.device("cuda:0")
    coord = torch.tensor(c, dtype=torch.float64, device=dev)
    atype = torch.tensor(t, dtype=torch.int32, device=dev)
    energy = torch.zeros(1, dtype=torch.float64, device=dev)
    force = torch.zeros((n, 3), dtype=torch.float64, device=dev)
    virial = torch.zeros(9, dtype=torch.float64, device=dev)
    runs = {}
    npairs = None
    for prec in ("fp64", "mixed"):
        ctx = dpk.Context(model, precision=prec)
        for _ in range(args.warmup):
            ctx.compute_device(coord, atype, b, energy, force, virial)
        ctx.check()
        if npairs is None:
            npairs = int((ctx.debug_nlist(n) >= 0).sum())
        torch.cuda.synchronize()
        ctx.profile(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.compute_device(coord, atype, b, energy, force, virial)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        stage_ms, nframes = ctx.profile_read()
        ctx.profile(False)
        ctx.check()
        st = ctx.stats()
        ms = (t1 - t0) * 1e3 / args.steps
        runs[prec] = dict(ms_per_step=ms, value=n / (ms * 1e-3),
                          stage_ms={k: v / nframes for k, v in stage_ms.items()},
                          force=force.cpu().numpy().copy(), energy=float(energy.item()),
                          virial=virial.cpu().numpy().reshape(3, 3).copy(), stats=st)
        print(f"# {prec}: {ms:.3f} ms/step, {n / (ms * 1e-3):.4g} atom-steps/s, stages (ms) "
              + ", ".join(f"{k} {v:.3f}" for k, v in runs[prec]["stage_ms"].items()), file=sys.stderr, flush=True)
        # the same frame through the host-buffer entry point (synchronous; host-to-device and
        # device-to-host copies included): reported beside the device-resident rate, never as it
        ctx.compute(c, t, b)
        hreps = max(3, args.steps // 4)
        t0 = time.perf_counter()
        for _ in range(hreps):
            ctx.compute(c, t, b)
        runs[prec]["host_buffer_ms_per_step"] = (time.perf_counter() - t0) * 1e3 / hreps
        print(f"# {prec}: host-buffer entry point {runs[prec]['host_buffer_ms_per_step']:.3f} ms/step",
              file=sys.stderr, flush=True)
        ctx.close()

    tabulated = None if args.no_table else tabulated_bench(dpk, synth, torch, max(1, args.steps // 2),
                                                            max(1, args.warmup // 2))
    serving = None if args.no_serving else serving_bench(dpk, synth)
    if serving:
        print(f"# serving: p50 {serving['p50_ms']:.3f} ms, p99 {serving['p99_ms']:.3f} ms at "
              f"{serving['arrival_rate_req_per_s']:.0f} req/s; saturated {serving['saturated_atom_steps_per_s']:.4g} "
              f"atom-steps/s; mean batch {serving['mean_batch_saturated']:.1f} (saturated), "
              f"{serving['mean_batch_poisson']:.1f} (Poisson)", file=sys.stderr, flush=True)

    cpu = None
    errs = {}
    if not args.no_cpu:
        from oracle import Oracle
        o = Oracle(synth.WATER_MODEL, synth.water_params())
        reps, elapsed, ref = 0, 0.0, None
        # whole frames until about 10 s of oracle work (at least one, at most 30)
        while reps < 30 and (reps == 0 or elapsed < 10.0):
            ts = time.perf_counter()
            ref = o.compute(c, t, b)
            elapsed += time.perf_counter() - ts
            reps += 1
        cpu = {"value": n * reps / elapsed, "unit": "atom-steps/s", "cores": o.threads(), "kind": "oracle",
               "sample": f"the full 12,288-atom frame (E+F+virial), {reps} evaluation(s), {elapsed:.1f} s"}
        for prec, r in runs.items():
            d = r["force"] - ref["force"]
            errs[prec] = {"max_abs_force_err": float(np.abs(d).max()),
                          "rms_force_err": float(np.sqrt((d ** 2).mean())),
                          "energy_err_per_atom": abs(r["energy"] - ref["energy"]) / n,
                          "max_virial_err_per_atom": float(np.abs(r["virial"] - ref["virial"]).max()) / n}
        errs["rms_force"] = float(np.sqrt((ref["force"] ** 2).mean()))

    head = runs["mixed"]
    dom = max(head["stage_ms"], key=head["stage_ms"].get)
    bound, amount, peak, unit = work_per_launch(dom, "mixed", n, npairs, model.nc)
    achieved = amount / (head["stage_ms"][dom] * 1e-3)
    roof = {"kernel": dom, "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": stored_traffic(dom, "mixed")}
    stage_roof = {}
    for st in ("nlist", "embed_fwd", "fit", "embed_bwd"):
        b_, a_, p_, u_ = work_per_launch(st, "mixed", n, npairs, model.nc)
        ach = a_ / (head["stage_ms"][st] * 1e-3)
        stage_roof[st] = {"bound": b_, "achieved": ach, "peak": p_, "unit": u_, "frac": ach / p_,
                          "ms": head["stage_ms"][st]}
    fp64_dom = max(runs["fp64"]["stage_ms"], key=runs["fp64"]["stage_ms"].get)
    b2, a2, p2, u2 = work_per_launch(fp64_dom, "fp64", n, npairs, model.nc)
    ach2 = a2 / (runs["fp64"]["stage_ms"][fp64_dom] * 1e-3)

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
        "fp64": {"value": runs["fp64"]["value"], "ms_per_step": runs["fp64"]["ms_per_step"],
                 "stage_ms": runs["fp64"]["stage_ms"],
                 "roofline": {"kernel": fp64_dom, "bound": b2, "achieved": ach2, "peak": p2, "unit": u2,
                              "frac": ach2 / p2, "traffic": stored_traffic(fp64_dom, "fp64")}},
        "mixed_stage_ms": head["stage_ms"],
        "host_buffer_ms_per_step": {p: runs[p]["host_buffer_ms_per_step"] for p in runs},
        "speedup_mixed_vs_fp64": head["value"] / runs["fp64"]["value"],
        "force_error_vs_oracle": errs or None,
        "roofline": roof,
        "stage_roofline": stage_roof,
        "tabulated": tabulated,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
