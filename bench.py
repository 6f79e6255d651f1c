#!/usr/bin/env python3
"""Benchmark of the GL-ECSIM step on one MI355X.

One step = the whole hot path on one batch of synthetic particles already
resident in HBM: deposit (mass matrices, current, moments) -> grid pass
(node assembly, smoothed bulk velocity, comoving current, limited LF
coefficients, RHS) -> FP64 GMRES solve to 1e-8 -> field update -> implicit push
with stable re-binning.  Prints one JSON line.

Workload (default): the 3D3V reconnection case at HBM scale (256x128x128
cells, 64 macro-particles per cell per species, m_i/m_e = 100, double Harris
sheet with a 0.2c guide flow), FP32 particle path, FP64 field solve.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "particle-steps/s (push+deposit); GMRES s/step plain vs NN-precond at 1e-8"


# what each synthetic workload stands for
KIND = {"c1": "1D3V shock tube", "c2": "2D3V uniform fast flow", "c3": "2D3V Harris-sheet reconnection",
        "c4": "3D3V colliding-flow shock", "c5": "3D3V double-Harris reconnection with a 0.2c guide flow",
        "ff1d": "1D3V uniform fast flow (solar wind)"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(wl, nsp, counts):
    """Compulsory HBM bytes of one launch of the particle kernels (FP32, 3D):
    deposit: particle state read once (28 B), the run table of each species
    (27 x 8 B per cell), node-averaged B (12 B per node) and the per-cell sums
    written once (558 x 4 B per cell with two species);
    push (per species): particle state read and written once (2 x 28 B), run
    table read and written (2 x 27 x 8 B per cell), segment offsets (4 B per
    cell), E and B at nodes (24 B per node)."""
    N = wl.ncells
    nd = 3 ** wl.dim
    nc = 2 ** wl.dim
    es = 4 if wl.fp32 else 8
    per_p = (wl.dim + 3 + 1) * es
    q_used = 18 * nd + nc * (7 + nsp)
    dep = sum(counts) * per_p + N * (nsp * nd * 8 + 3 * es + q_used * es)
    push = sum(c * 2 * per_p for c in counts) + nsp * N * (2 * nd * 8 + 4 + 6 * es)
    return {"deposit": dep, "push": push}


def measured_traffic(kernel_file, record):
    """HBM bytes per launch of the dominant kernel from the committed counter
    record (profiles/), or None when the kernel source changed since the
    counters were taken (the record holds the source's SHA-256)."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, record)))
        src = open(os.path.join(ROOT, kernel_file), "rb").read()
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != hashlib.sha256(src).hexdigest():
        return None
    return float(rec["traffic_bytes"])


def cpu_baseline(wl, box=24):
    """The FP64 oracle, as it stands, timed on a bounded sample of the same
    workload: one full step of a periodic box^3-cell sub-box built with the
    same recipe (ppc, dx, dt, species)."""
    import oracle as O
    import synth
    sub = synth.small("cpu_sample", dim=3, n=(box, box, box), ppc=wl.ppc, base="c5")
    G = O.grid(3, sub.n, sub.dx)
    E, B = synth.fields(sub)
    sp = []
    for s in range(sub.nsp):
        p = synth.particles(sub, s, f32=True)
        sp.append(O.Species(sub.q[s], sub.m[s], O.global_positions(G, p["cell"], p["off"].astype(np.float64)),
                            p["v"].astype(np.float64).T, p["w"].astype(np.float64)))
    npart = sum(s.w.size for s in sp)
    t0 = time.perf_counter()
    O.step(G, sp, E, B, dt=sub.dt, theta=sub.theta, comoving=True, lf_E=True, lf_B=True, beta_lim=sub.beta_lim,
           a_mode=sub.a_mode, tol=1e-8, restart=30)
    dt = time.perf_counter() - t0
    return {"value": npart / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"1 full step (deposit, comoving current, GMRES to 1e-8, B/E update, push) of a "
                      f"{box}^3-cell periodic sub-box with the same recipe ({npart} particles), "
                      f"single-threaded FP64 C oracle, {dt:.1f} s"}


def nn_compare(sim, args):
    """Learned preconditioner, after the timed steps: harvest (residual,
    correction) pairs from plain solves, train on the GPU, then solve each of
    the next steps both ways from the same state (plain GMRES, then
    CNN-preconditioned FGMRES, both to the same true residual) and push with
    the second answer."""
    from paper_2506_11320_amd import GE_HARVEST_KRYLOV, GE_HARVEST_SOLUTION, GE_PC_CNN
    sim.cnn_init(1, max_pairs=args.nn_pairs)
    sim.cnn_harvest({"solution": GE_HARVEST_SOLUTION, "krylov": GE_HARVEST_KRYLOV,
                     "both": GE_HARVEST_SOLUTION | GE_HARVEST_KRYLOV}[args.nn_data])
    for k in range(args.nn_harvest):
        r = sim.step(tol=args.tol, maxit=500, restart=30, precond=0)
        log(f"harvest step {k}: {r['iterations']} iterations")
    sim.cnn_harvest(0)
    tr = sim.cnn_train(crop=args.nn_crop, batch=args.nn_batch, iters=args.nn_iters, lr=args.nn_lr, seed=7)
    log(f"trained: {tr}")
    res = {"plain": [], "nn": []}
    for k in range(args.nn_eval):
        sim.deposit()
        rp = sim.solve(tol=args.tol, maxit=500, restart=30, precond=0)
        rc = sim.solve(tol=args.tol, maxit=500, restart=30, precond=GE_PC_CNN)
        if not (rp["converged"] and rc["converged"]):
            log(f"eval step {k}: not converged (plain {rp['relres']:.2e}, nn {rc['relres']:.2e})")
        res["plain"].append((rp["seconds"], rp["iterations"]))
        res["nn"].append((rc["seconds"], rc["iterations"], rc["fallback"], rc["relres"]))
        log(f"eval step {k}: plain {rp['iterations']} it {rp['seconds'] * 1e3:.2f} ms, "
            f"nn {rc['iterations']} it {rc['seconds'] * 1e3:.2f} ms (relres {rc['relres']:.2e})")
        sim.push()
        sim.update_fields()
    sim.sync()
    return {
        "plain": {"seconds": float(np.mean([a[0] for a in res["plain"]])),
                  "iterations": float(np.mean([a[1] for a in res["plain"]]))},
        "nn": {"seconds": float(np.mean([a[0] for a in res["nn"]])),
               "iterations": float(np.mean([a[1] for a in res["nn"]])),
               "fallbacks": int(sum(a[2] for a in res["nn"])),
               "max_relres": float(max(a[3] for a in res["nn"]))},
        "train": {"pairs": tr["pairs"], "data": args.nn_data, "steps": tr["steps"], "crop": args.nn_crop,
                  "batch": args.nn_batch, "lr": args.nn_lr,
                  "loss_first": tr["loss_first"], "loss_last": tr["loss_last"], "seconds": tr["seconds"]},
        "eval_steps": args.nn_eval,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c5")
    ap.add_argument("--precond", default="none", choices=["none", "jacobi"])
    ap.add_argument("--precision", default="workload", choices=["workload", "fp32", "fp64"],
                    help="particle precision: the workload's own, or forced")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--compare-precond", action="store_true", help="also time a Jacobi-preconditioned solve")
    ap.add_argument("--no-nn", action="store_true", help="skip the learned-preconditioner comparison")
    ap.add_argument("--nn-harvest", type=int, default=8, help="plain solves whose (residual, correction) pairs train")
    ap.add_argument("--nn-iters", type=int, default=300, help="training steps")
    ap.add_argument("--nn-crop", type=int, default=16)
    ap.add_argument("--nn-batch", type=int, default=16)
    ap.add_argument("--nn-lr", type=float, default=1e-3)
    ap.add_argument("--nn-eval", type=int, default=4, help="steps solved both ways after training")
    ap.add_argument("--nn-pairs", type=int, default=96, help="pair store capacity")
    ap.add_argument("--nn-data", default="both", choices=["solution", "krylov", "both"],
                    help="training pairs: (r0, e) of each solve, (A v_j, v_j) of its Arnoldi vectors, or both")
    ap.add_argument("--ns-j", type=int, default=0, help="current smoothing passes (Sec. 3.2); 0 = off")
    ap.add_argument("--dedner", action="store_true", help="divergence cleaning of B (Sec. 2.3)")
    ap.add_argument("--explicit-current", type=int, default=0, metavar="K",
                    help="also time K calls of the explicit-PIC current (Sec. 3.1) at the final particle state")
    ap.add_argument("--explicit-steps", type=int, default=0, metavar="K",
                    help="also time K explicit PIC steps (ge_explicit_step) on the same workload with dt = 0.25, "
                         "which keeps c dt below dx / sqrt(3)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of 4 GiB (reference for the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path (got --gpus {args.gpus}); "
              "the sharding design is described in DESIGN.md", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2506_11320_amd import Simulation

    if args.copy_probe:
        a = torch.ones(1 << 29, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": a.numel() * 8, "copy_probe_bytes_written": b.numel() * 8}))
        return

    wl = synth.workloads()[args.workload]
    if args.precision != "workload":
        wl = wl.replace(fp32=args.precision == "fp32")
    log(f"workload {wl.name}: cells {wl.n[:wl.dim]}, ppc {wl.ppc}, species {wl.nsp}")
    sim = Simulation(wl.dim, wl.n, wl.dx, theta=wl.theta, dt=wl.dt, lf_E=wl.lf_E, lf_B=wl.lf_B,
                     beta_lim=wl.beta_lim, a_mode=wl.a_mode, comoving=wl.comoving, n_smooth_u=wl.n_smooth_u,
                     fp32=wl.fp32, ns_j=args.ns_j, dedner=args.dedner)
    counts = []
    t0 = time.perf_counter()
    for s in range(wl.nsp):
        p = synth.particles(wl, s, f32=wl.fp32)
        t = {k: torch.from_numpy(v).cuda() for k, v in p.items()}
        del p
        sim.add_species(wl.q[s], wl.m[s], t["cell"], t["off"], t["v"], t["w"])
        counts.append(int(t["cell"].numel()))
        del t
        torch.cuda.synchronize()
        log(f"species {s} loaded ({counts[-1]} particles)")
    E, B = synth.fields(wl)
    sim.set_fields(torch.from_numpy(E).cuda(), torch.from_numpy(B).cuda())
    torch.cuda.synchronize()
    log(f"setup {time.perf_counter() - t0:.1f} s")
    pc = {"none": 0, "jacobi": 1}[args.precond]
    for k in range(args.warmup):
        r = sim.step(tol=args.tol, maxit=500, restart=30, precond=pc)
        log(f"warmup step {k}: {r['iterations']} GMRES iterations, relres {r['relres']:.2e}")
    sim.timings()  # reset the per-phase accumulators
    iters = []
    solve_s = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        r = sim.step(tol=args.tol, maxit=500, restart=30, precond=pc)
        iters.append(r["iterations"])
        solve_s.append(r["seconds"])
        if not r["converged"]:
            log(f"step {k}: GMRES did not converge (relres {r['relres']:.2e})")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tm = sim.timings()
    log(f"timed {args.steps} steps in {elapsed:.3f} s")
    npart = sum(counts)
    ms_step = elapsed / args.steps * 1e3
    phase = {"push_rebin": tm[0] * 1e3, "deposit": tm[1] * 1e3, "assemble": tm[2] * 1e3, "grid_rest": tm[3] * 1e3,
             "update": tm[4] * 1e3, "solve": tm[5] * 1e3}
    pd_s = tm[0] + tm[1]
    ab = algorithmic_bytes(wl, wl.nsp, counts)
    dom = "deposit" if tm[1] >= tm[0] else "push"
    dom_t = tm[1] if dom == "deposit" else tm[0]
    achieved = ab[dom] / dom_t / 1e9
    tname = f"{'float' if wl.fp32 else 'double'},{wl.dim}"
    roof = {"bound": "hbm", "kernel": f"k_deposit<{tname}>" if dom == "deposit" else f"k_push<{tname}> (x2 species)",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic("paper_2506_11320_amd/csrc/ge_particles.hip", "profiles/c5_deposit_traffic.json")
            if (dom == "deposit" and args.workload == "c5" and wl.fp32) else None,
            "algorithmic_bytes_per_launch": ab[dom], "launch_ms": round(dom_t * 1e3, 4)}
    precond_cmp = None
    if args.compare_precond:
        pcs = {}
        for name, code in [("plain", 0), ("jacobi", 1)]:
            sim.deposit()
            rep = sim.solve(tol=args.tol, maxit=500, restart=30, precond=code)
            pcs[name] = {"seconds": rep["seconds"], "iterations": rep["iterations"]}
        precond_cmp = pcs
    nn = None
    if not args.no_nn and wl.dim == 3:
        nn = nn_compare(sim, args)
    expl = None
    if args.explicit_current > 0:
        sim.explicit_current()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(sim.stream)
        for _ in range(args.explicit_current):
            sim.explicit_current()
        ev1.record(sim.stream)
        ev1.synchronize()
        expl = {"calls": args.explicit_current, "ms_per_call": round(ev0.elapsed_time(ev1) / args.explicit_current, 3)}
    expl_step = None
    if args.explicit_steps > 0:
        sim.close()
        sim = Simulation(wl.dim, wl.n, wl.dx, theta=wl.theta, dt=0.25, lf_E=False, lf_B=False, beta_lim=wl.beta_lim,
                         a_mode=wl.a_mode, comoving=wl.comoving, n_smooth_u=wl.n_smooth_u, fp32=wl.fp32,
                         ns_j=args.ns_j)
        for s in range(wl.nsp):
            p = synth.particles(wl, s, f32=wl.fp32)
            t = {k: torch.from_numpy(v).cuda() for k, v in p.items()}
            del p
            sim.add_species(wl.q[s], wl.m[s], t["cell"], t["off"], t["v"], t["w"])
            del t
            torch.cuda.synchronize()
        sim.set_fields(torch.from_numpy(E).cuda(), torch.from_numpy(B).cuda())
        sim.explicit_step()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(sim.stream)
        for _ in range(args.explicit_steps):
            sim.explicit_step()
        ev1.record(sim.stream)
        ev1.synchronize()
        ms = ev0.elapsed_time(ev1) / args.explicit_steps
        expl_step = {"steps": args.explicit_steps, "dt": 0.25, "ms_per_step": round(ms, 3),
                     "particle_steps_per_s": npart / (ms * 1e-3)}
        log(f"explicit step: {ms:.3f} ms")
    out = {
        "metric": METRIC,
        "value": npart * args.steps / elapsed,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if wl.fp32 else "f64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: {KIND.get(args.workload, wl.name)}, "
                               f"{'x'.join(str(v) for v in wl.n[:wl.dim])} cells, "
                               f"{wl.ppc} ppc/species, m_i/m_e={wl.m[1]:g}, "
                               f"{'FP32' if wl.fp32 else 'FP64'} push/deposit, FP64 GMRES to {args.tol:g}, "
                               f"{'comoving' if wl.comoving else 'lab-frame'} current, "
                               f"{'limited LF' if wl.lf_E or wl.lf_B else 'no LF'}",
                   "cells": wl.ncells, "particles": npart, "precond": args.precond, "ns_j": args.ns_j,
                   "dedner": bool(args.dedner)},
        "push_deposit_particle_steps_per_s": npart / pd_s,
        "gmres_s_per_step": {"plain" if pc == 0 else args.precond: float(np.mean(solve_s)),
                             "nn": nn["nn"]["seconds"] if nn else None},
        "nn_precond": nn,
        "gmres_iterations": float(np.mean(iters)),
        "phase_ms": {k: round(v, 3) for k, v in phase.items()},
        "precond_compare": precond_cmp,
        "explicit_current": expl,
        "explicit_step": expl_step,
        "roofline": roof,
        # the other particle phase against the same peak: algorithmic bytes of
        # both species' push over the phase's event-timed duration (the
        # re-binning count and scan kernels included)
        "push_roofline": {"bound": "hbm", "kernel": f"k_push<{tname}> (x{wl.nsp} species) + re-binning scans",
                          "achieved": round(ab["push"] / tm[0] / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(ab["push"] / tm[0] / 1e9 / HBM_PEAK_GBS, 4),
                          "algorithmic_bytes": ab["push"], "phase_ms": round(tm[0] * 1e3, 4)},
    }
    sim.close()
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample")
        out["cpu_baseline"] = cpu_baseline(wl)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
