#!/usr/bin/env python3
"""Benchmark of the GL-ECSIM step on one MI355X.

One step = the whole hot path on one batch of synthetic particles already
resident in HBM: deposit (mass matrices, current, moments) -> grid pass
(node assembly, smoothed bulk velocity, comoving current, limited LF
coefficients, RHS) -> FP64 GMRES solve to 1e-8 -> field update -> implicit push
with stable re-binning (and the stable re-sort of particles that moved more
than one cell, when there are any).  Prints one JSON line.

Workload (default): the 3D3V reconnection case at HBM scale (256x128x128
cells, 64 macro-particles per cell per species, m_i/m_e = 100, double Harris
sheet with a 0.2c guide flow), FP32 particle path, FP64 field solve.

Legs after the timed steps, each from a fresh load of the same initial state
(so that the driver's --steps does not change what they see):
  nn_precond   learned preconditioner: harvest, train, then plain GMRES and
               CNN-preconditioned FGMRES on the same systems;
  cpu_baseline the FP64 oracle on a bounded sample of the workload, one core
               and all cores (independent sub-boxes in parallel processes).
The JSON line is printed at the end; the exit status is 0 only if every leg
succeeded (a failed leg is named in "errors").
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
BF16_PEAK_TFLOPS = 2500.0
METRIC = "particle-steps/s (push+deposit); GMRES s/step plain vs NN-precond at 1e-8"


# what each synthetic workload stands for
KIND = {"c1": "1D3V shock tube", "c2": "2D3V uniform fast flow", "c3": "2D3V Harris-sheet reconnection",
        "c4": "3D3V shock: flow at -0.15c onto a reflecting wall, inflow at x = L", "c4p": "3D3V colliding-flow shock (periodic)", "c5": "3D3V double-Harris reconnection with a 0.2c guide flow",
        "ff1d": "1D3V uniform fast flow (solar wind)"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(wl, nsp, npart):
    """Algorithmic HBM bytes of the particle phases (the method's compulsory
    traffic, not this library's staging), per launch:
      deposit: each particle's state read once (offsets, weight, velocity:
        (dim + 4) values), and per node the node-averaged B read (3 values)
        and the grid outputs written once: the half-stencil mass matrices
        Mtilde and M0 (2 x nh x 9 values in the particle precision), the
        current (3), charge density per species (nsp), mass-weighted velocity
        (3) and mass (1) in FP64;
      push: each particle's state read and written once, and per node E^{n+theta}
        and the node-averaged B read (6 values), per cell the segment start of
        each species (4 B) -- the re-binning writes nothing beyond the
        particle state it moves;
      step: the two together, the push+deposit pass of one particle-step."""
    N = wl.ncells
    es = 4 if wl.fp32 else 8
    nh = {1: 2, 2: 5, 3: 14}[wl.dim]
    per_p = (wl.dim + 4) * es
    node_dep = 3 * es + 2 * nh * 9 * es + (3 + nsp + 3 + 1) * 8
    dep = npart * per_p + N * node_dep
    push = npart * 2 * per_p + N * (6 * es + 4 * nsp)
    return {"deposit": dep, "push": push, "step": dep + push,
            "per_particle": per_p, "per_node_deposit": node_dep}


TRAFFIC_SOURCES = ("paper_2506_11320_amd/csrc/ge_particles.hip", "paper_2506_11320_amd/csrc/ge_internal.h")


def sources_sha256(files=TRAFFIC_SOURCES):
    """SHA-256 over the kernel's source files (the kernel file and the header
    that fixes its data layouts), in the given order."""
    import hashlib
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()


def measured_traffic(record):
    """HBM bytes per launch of the dominant kernel from the committed counter
    record (profiles/), or None when its sources changed since the counters
    were taken (the record holds their SHA-256)."""
    try:
        rec = json.load(open(os.path.join(ROOT, record)))
        sha = sources_sha256(tuple(rec.get("sources", ())))
    except (OSError, ValueError, TypeError):
        return None
    if not rec.get("sources") or rec.get("sources_sha256") != sha:
        return None
    return float(rec["traffic_bytes"])


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_sample(args):
    """One full oracle step (deposit, comoving current, GMRES to 1e-8, B/E
    update, push) of a periodic box^3 sub-box with the workload's recipe;
    seed offset k makes each process's sub-box independent."""
    wname, box, k = args
    import oracle as O
    import synth
    wl = synth.workloads()[wname]
    sub = synth.small("cpu_sample", dim=3, n=(box, box, box), ppc=wl.ppc, base=wname).replace(seed=wl.seed + 101 * k)
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
    return npart, time.perf_counter() - t0


def _oracle_full_grid(wname):
    """The cpu_baseline leg on the whole grid of a workload: the FP64 oracle,
    on one core, runs the deposit and grid pass of the initial state (lab and
    comoving deposits, bulk velocity and its filter, E_M, J_eff, the LF
    coefficients and the right-hand side), then the field solve by plain
    GMRES(30) from E^n to 1e-8, timed separately.  Takes minutes on the 3D
    workloads."""
    import oracle as O
    import synth
    wl = synth.workloads()[wname]
    G = O.grid(wl.dim, wl.n, wl.dx, bc=wl.bc)
    E, B = synth.fields(wl)
    sp = []
    for s in range(wl.nsp):
        p = synth.particles(wl, s, f32=wl.fp32)
        sp.append(O.Species(wl.q[s], wl.m[s], O.global_positions(G, p["cell"], p["off"].astype(np.float64)),
                            p["v"].astype(np.float64).T, p["w"].astype(np.float64)))
        del p
    npart = sum(x.w.size for x in sp)
    log(f"oracle full solve {wname}: {npart} particles, {O.nnodes(G)} nodes")
    P = O.params(wl.theta, wl.dt)
    t0 = time.perf_counter()
    dep = O.deposit(G, sp, wl.dt, B, wl.comoving, wl.n_smooth_u)
    a_node = O.diffusion_speed(G, dep["u"], wl.a_mode)
    kE = O.kappa_E(G, E, a_node, wl.beta_lim) if wl.lf_E else None
    b = O.rhs(G, P, E, B, dep["J_eff"])
    t1 = time.perf_counter()
    log(f"oracle deposit and grid pass {t1 - t0:.1f} s")
    _, its, rel = O.gmres(G, P, dep["Mt"], kE, b, E, tol=1e-8, maxit=5000, restart=30)
    t2 = time.perf_counter()
    return {"cpu_baseline_full_grid": {"workload": wname, "nodes": O.nnodes(G), "particles": npart,
                                  "deposit_and_grid_pass_s": round(t1 - t0, 2), "gmres_s": round(t2 - t1, 2),
                                  "gmres_iterations": its, "relres": rel, "tol": 1e-8, "cores": 1,
                                  "cpu_model": cpu_model(), "kind": "oracle, single-threaded C, gcc -O2"}}


def cpu_baseline(wname, box, procs, full_grid=False):
    """The FP64 C oracle, as it stands, timed on bounded samples of the same
    workload: one process (one core), then `procs` processes at once on
    independent sub-boxes (all cores, aggregate rate).  full_grid: instead,
    its deposit and GMRES solve on the workload's whole grid, one core."""
    if full_grid:
        return _oracle_full_grid(wname)
    import multiprocessing as mp
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    n1, t1 = _oracle_sample((wname, box, 0))
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(procs) as pool:
        res = pool.map(_oracle_sample, [(wname, box, k + 1) for k in range(procs)])
    tall = time.perf_counter() - t0
    nall = sum(r[0] for r in res)
    return {"value": nall / tall, "unit": "particle-steps/s", "cores": procs, "kind": "oracle",
            "sample": f"1 full FP64 oracle step (deposit, comoving current, GMRES to 1e-8, B/E update, push) of "
                      f"a periodic {box}^3-cell sub-box with the workload's recipe ({n1} particles), one per "
                      f"process, {procs} processes at once ({tall:.1f} s wall); single-threaded C oracle, gcc -O2",
            "single_core": {"value": n1 / t1, "seconds": round(t1, 2), "particles": n1},
            "nproc": os.cpu_count(), "cpu_model": cpu_model()}


def make_sim(wl, args, Simulation, torch, synth):
    sim = Simulation(wl.dim, wl.n, wl.dx, theta=wl.theta, dt=wl.dt, lf_E=wl.lf_E, lf_B=wl.lf_B,
                     beta_lim=wl.beta_lim, a_mode=wl.a_mode, comoving=wl.comoving, n_smooth_u=wl.n_smooth_u,
                     fp32=wl.fp32, ns_j=args.ns_j, dedner=args.dedner, bc=wl.bc)
    counts = []
    for s in range(wl.nsp):
        p = synth.particles(wl, s, f32=wl.fp32)
        t = {k: torch.from_numpy(v).cuda() for k, v in p.items()}
        del p
        sim.add_species(wl.q[s], wl.m[s], t["cell"], t["off"], t["v"], t["w"])
        counts.append(int(t["cell"].numel()))
        del t
        torch.cuda.synchronize()
    E, B = synth.fields(wl)
    sim.set_fields(torch.from_numpy(E).cuda(), torch.from_numpy(B).cuda())
    torch.cuda.synchronize()
    return sim, counts


def per_step_metrics(sim, wl, args, pc, synth, torch):
    """Per-step record of an untimed continuation of the run (one JSON object
    per line): each step is followed by a synchronising read of its phase
    times, diagnostics and move report, so it is kept out of the timed steps."""
    k0 = args.warmup + args.steps
    sim.timings()
    sim.moves()
    with open(args.metrics_jsonl, "w") as f:
        for k in range(args.metrics_steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = sim.step(tol=args.tol, maxit=500, restart=30, precond=pc)
            if wl.walled and wl.bc[1] == 2:
                for s in range(wl.nsp):
                    p = {kk: torch.from_numpy(v).cuda() for kk, v in synth.inflow(wl, s, k0 + k, f32=wl.fp32).items()}
                    sim.inject(s, p["cell"], p["off"], p["v"], p["w"])
            sim.sync()
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            tm = sim.timings()
            d = sim.diagnostics()
            rec = {"step": k0 + k, "workload": wl.name, "wall_ms": round(wall * 1e3, 3),
                   "phase_ms": {"push_rebin": tm[0] * 1e3, "deposit": tm[1] * 1e3, "assemble": tm[2] * 1e3,
                                "grid_rest": tm[3] * 1e3, "update": tm[4] * 1e3, "solve": tm[5] * 1e3},
                   "gmres": {"iterations": r["iterations"], "relres": r["relres"], "converged": r["converged"]},
                   "W_E": d["W_E"], "W_B": d["W_B"], "K": d["K"], "P": d["P"], "gauss": d["gauss"],
                   "particles": [sim.count(s) for s in range(wl.nsp)], "moves": sim.moves()}
            f.write(json.dumps(rec) + "\n")
            f.flush()
            log(f"metrics step {k0 + k}: {r['iterations']} GMRES iterations, W_E {d['W_E']:.4e}, "
                f"gauss {d['gauss']:.3e}")


def cnn_flops_per_node():
    """FLOPs of one application of the 3 -> 32 -> 32 -> 3 network of 3x3x3
    convolutions per grid node (2 per multiply-add)."""
    return 2 * 27 * (3 * 32 + 32 * 32 + 32 * 3)


def nn_compare(wl, args, Simulation, torch, synth):
    """Learned preconditioner from a fresh load of the initial state: harvest
    (residual, correction) pairs from plain solves, train on the GPU, then
    solve each of the next steps both ways from the same state (plain GMRES,
    then CNN-preconditioned FGMRES, both to the same true residual) and push
    with the second answer."""
    from paper_2506_11320_amd import GE_HARVEST_KRYLOV, GE_HARVEST_SOLUTION, GE_PC_CNN
    sim, _ = make_sim(wl, args, Simulation, torch, synth)
    k_inj = [0]

    def inject():
        if wl.walled and wl.bc[1] == 2:
            for s in range(wl.nsp):
                p = {kk: torch.from_numpy(v).cuda() for kk, v in synth.inflow(wl, s, k_inj[0], f32=wl.fp32).items()}
                sim.inject(s, p["cell"], p["off"], p["v"], p["w"])
            k_inj[0] += 1

    try:
        sim.cnn_init(1, max_pairs=args.nn_pairs)
        sim.cnn_harvest({"solution": GE_HARVEST_SOLUTION, "krylov": GE_HARVEST_KRYLOV,
                         "both": GE_HARVEST_SOLUTION | GE_HARVEST_KRYLOV}[args.nn_data])
        for k in range(args.nn_harvest):
            r = sim.step(tol=args.tol, maxit=500, restart=30, precond=0)
            inject()
            log(f"harvest step {k}: {r['iterations']} iterations")
        sim.cnn_harvest(0)
        tr = sim.cnn_train(crop=args.nn_crop, batch=args.nn_batch, iters=args.nn_iters, lr=args.nn_lr, seed=7)
        log(f"trained: {tr}")
        # one application of the network alone (event-timed), for its MFMA rate:
        # the scaled form that the flexible GMRES runs (no RMS reduction, no host
        # round trip), on a vector of RMS 1
        r0 = torch.randn((3, sim.N), dtype=torch.float64, device=sim.device)
        z0 = torch.empty_like(r0)
        sim.cnn_apply_scaled(r0, 1.0, z0)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(sim.stream)
        for _ in range(5):
            sim.cnn_apply_scaled(r0, 1.0, z0)
        ev1.record(sim.stream)
        ev1.synchronize()
        app_s = ev0.elapsed_time(ev1) / 5 * 1e-3
        res = {"plain": [], "nn": []}
        for k in range(args.nn_eval):
            sim.deposit()
            rp = sim.solve(tol=args.tol, maxit=500, restart=30, precond=0)
            rc = sim.solve(tol=args.tol, maxit=500, restart=30, precond=GE_PC_CNN)
            if not (rp["converged"] and rc["converged"]):
                raise RuntimeError(f"eval step {k}: not converged (plain {rp['relres']:.2e}, nn {rc['relres']:.2e})")
            res["plain"].append((rp["seconds"], rp["iterations"], rp["relres"]))
            res["nn"].append((rc["seconds"], rc["iterations"], rc["fallback"], rc["relres"]))
            log(f"eval step {k}: plain {rp['iterations']} it {rp['seconds'] * 1e3:.2f} ms, "
                f"nn {rc['iterations']} it {rc['seconds'] * 1e3:.2f} ms (relres {rc['relres']:.2e})")
            sim.push()
            sim.update_fields()
            inject()
        sim.sync()
    finally:
        sim.close()
    flops = cnn_flops_per_node() * wl.ncells
    return {
        "plain": {"seconds": float(np.mean([a[0] for a in res["plain"]])),
                  "iterations": float(np.mean([a[1] for a in res["plain"]])),
                  "max_relres": float(max(a[2] for a in res["plain"]))},
        "nn": {"seconds": float(np.mean([a[0] for a in res["nn"]])),
               "iterations": float(np.mean([a[1] for a in res["nn"]])),
               "fallbacks": int(sum(a[2] for a in res["nn"])),
               "max_relres": float(max(a[3] for a in res["nn"]))},
        "speedup": float(np.mean([a[0] for a in res["plain"]]) / np.mean([a[0] for a in res["nn"]])),
        "cnn_apply": {"ms": round(app_s * 1e3, 4), "flop": flops,
                      "tflops": round(flops / app_s / 1e12, 1),
                      "mfma_utilisation": round(flops / app_s / 1e12 / BF16_PEAK_TFLOPS, 4),
                      "peak_tflops": BF16_PEAK_TFLOPS, "dtype": "bf16 operands, fp32 accumulation"},
        "train": {"pairs": tr["pairs"], "data": args.nn_data, "steps": tr["steps"], "crop": args.nn_crop,
                  "batch": args.nn_batch, "lr": args.nn_lr,
                  "loss_first": tr["loss_first"], "loss_last": tr["loss_last"], "seconds": tr["seconds"]},
        "harvest_steps": args.nn_harvest, "eval_steps": args.nn_eval,
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
    ap.add_argument("--cpu-box", type=int, default=24, help="edge of the oracle's sub-box in cells")
    ap.add_argument("--cpu-procs", type=int, default=0, help="oracle processes for the all-core rate (0: min(16, nproc))")
    ap.add_argument("--compare-precond", action="store_true", help="also time a Jacobi-preconditioned solve")
    ap.add_argument("--no-nn", action="store_true", help="skip the learned-preconditioner comparison")
    ap.add_argument("--nn-harvest", type=int, default=8, help="plain solves whose (residual, correction) pairs train")
    ap.add_argument("--nn-iters", type=int, default=800, help="training steps")
    ap.add_argument("--nn-crop", type=int, default=16)
    ap.add_argument("--nn-batch", type=int, default=16)
    ap.add_argument("--nn-lr", type=float, default=2e-3)
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
    ap.add_argument("--metrics-jsonl", default="", metavar="PATH",
                    help="after the timed steps, run --metrics-steps more steps (untimed) and write one JSON line "
                         "per step to PATH: phase times, GMRES iterations and residual, FP64 energies, momenta, "
                         "Gauss residual, moves")
    ap.add_argument("--metrics-steps", type=int, default=10)
    ap.add_argument("--cpu-baseline-full-grid", action="store_true",
                    help="only run the CPU-baseline leg on the whole grid of --workload: the FP64 oracle's deposit "
                         "and plain GMRES solve, one core, no GPU; print its record and exit")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of 4 GiB (reference for the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: there is no multi-GPU path (got --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    if args.cpu_baseline_full_grid:
        print(json.dumps(cpu_baseline(args.workload, 0, 1, full_grid=True)), flush=True)
        return

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
    t0 = time.perf_counter()
    sim, counts = make_sim(wl, args, Simulation, torch, synth)
    log(f"setup {time.perf_counter() - t0:.1f} s ({sum(counts)} particles)")
    pc = {"none": 0, "jacobi": 1}[args.precond]
    # an inflow plane: the particles entering in each step, generated and
    # uploaded before the timed region, injected after each step
    inflow = []
    if wl.walled and wl.bc[1] == 2:
        for k in range(args.warmup + args.steps):
            inflow.append([{kk: torch.from_numpy(v).cuda() for kk, v in synth.inflow(wl, s, k, f32=wl.fp32).items()}
                           for s in range(wl.nsp)])
        torch.cuda.synchronize()

    def inject(k):
        for s, p in enumerate(inflow[k] if inflow else []):
            sim.inject(s, p["cell"], p["off"], p["v"], p["w"])

    for k in range(args.warmup):
        r = sim.step(tol=args.tol, maxit=500, restart=30, precond=pc)
        inject(k)
        log(f"warmup step {k}: {r['iterations']} GMRES iterations, relres {r['relres']:.2e}")
    sim.timings()  # reset the per-phase accumulators
    sim.moves()
    iters = []
    solve_s = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        r = sim.step(tol=args.tol, maxit=500, restart=30, precond=pc)
        inject(args.warmup + k)
        iters.append(r["iterations"])
        solve_s.append(r["seconds"])
        if not r["converged"]:
            log(f"step {k}: GMRES did not converge (relres {r['relres']:.2e})")
    sim.sync()  # the last injection joins the species
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tm = sim.timings()
    moves = sim.moves()
    diag = sim.diagnostics()
    log(f"timed {args.steps} steps in {elapsed:.3f} s; moves {moves}")
    npart = sum(counts) if not inflow else sum(sim.count(s) for s in range(wl.nsp))
    ms_step = elapsed / args.steps * 1e3
    phase = {"push_rebin": tm[0] * 1e3, "deposit": tm[1] * 1e3, "assemble": tm[2] * 1e3, "grid_rest": tm[3] * 1e3,
             "update": tm[4] * 1e3, "solve": tm[5] * 1e3, "rebin_scans": tm[6] * 1e3}
    pd_s = tm[0] + tm[1] + tm[2]
    ab = algorithmic_bytes(wl, wl.nsp, npart)
    tname = f"{'float' if wl.fp32 else 'double'},{wl.dim}"
    achieved = ab["deposit"] / tm[1] / 1e9
    roof = {"bound": "hbm", "kernel": f"k_deposit<{tname}>",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic("profiles/c5_deposit_traffic.json")
            if (args.workload == "c5" and wl.fp32) else None,
            "algorithmic_bytes_per_launch": ab["deposit"], "launch_ms": round(tm[1] * 1e3, 4),
            "algorithmic_bytes_per_unit": {"particle": ab["per_particle"], "node": ab["per_node_deposit"]}}
    if roof["traffic"]:
        roof["traffic_over_algorithmic"] = round(roof["traffic"] / ab["deposit"], 3)
    if args.metrics_jsonl:
        per_step_metrics(sim, wl, args, pc, synth, torch)
    precond_cmp = None
    if args.compare_precond:
        pcs = {}
        for name, code in [("plain", 0), ("jacobi", 1)]:
            sim.deposit()
            rep = sim.solve(tol=args.tol, maxit=500, restart=30, precond=code)
            pcs[name] = {"seconds": rep["seconds"], "iterations": rep["iterations"]}
        precond_cmp = pcs
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
    sim.close()
    del sim
    torch.cuda.empty_cache()
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
                   "cells": wl.nphys, "particles": npart, "precond": args.precond, "ns_j": args.ns_j,
                   "x_boundaries": {0: "periodic", 1: "wall", 2: "inflow"}[wl.bc[0]] + "/" +
                                   {0: "periodic", 1: "wall", 2: "inflow"}[wl.bc[1]],
                   "dedner": bool(args.dedner)},
        # the metric's first quantity: particle-steps per second of the
        # particle phases alone (push with re-binning, deposit, node assembly)
        "push_deposit_particle_steps_per_s": npart / pd_s,
        # the same without the re-binning's own kernels (corner packing and
        # segment scans, inside push_rebin); the pushes write the direction
        # runs as they go, so that part of the sort has no separate time
        "push_deposit_particle_steps_per_s_sort_excluded": npart / (pd_s - tm[6]),
        "gmres_s_per_step": {"plain" if pc == 0 else args.precond: float(np.mean(solve_s)), "nn": None},
        "gmres_iterations": float(np.mean(iters)),
        "phase_ms": {k: round(v, 3) for k, v in phase.items()},
        "moves": moves,
        "energy_after": {"W_E": diag["W_E"], "W_B": diag["W_B"], "K": diag["K"]},
        "precond_compare": precond_cmp,
        "explicit_current": expl,
        "roofline": roof,
        # the push phase and the whole particle pass against the same peak,
        # with the algorithmic bytes of algorithmic_bytes()
        "push_roofline": {"bound": "hbm", "kernel": f"k_push<{tname}> (x{wl.nsp} species) + segment scans",
                          "achieved": round(ab["push"] / tm[0] / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(ab["push"] / tm[0] / 1e9 / HBM_PEAK_GBS, 4),
                          "algorithmic_bytes": ab["push"], "phase_ms": round(tm[0] * 1e3, 4)},
        "particle_pass_roofline": {"bound": "hbm", "phases": "push + deposit + node assembly",
                                   "achieved": round(ab["step"] / pd_s / 1e9, 1), "peak": HBM_PEAK_GBS,
                                   "unit": "GB/s", "frac": round(ab["step"] / pd_s / 1e9 / HBM_PEAK_GBS, 4),
                                   "algorithmic_bytes": ab["step"], "ms": round(pd_s * 1e3, 4)},
        "nn_precond": None,
        "explicit_step": None,
        "cpu_baseline": None,
    }
    errors = {}
    if not args.no_nn and wl.dim == 3:
        try:
            nn = nn_compare(wl, args, Simulation, torch, synth)
            out["nn_precond"] = nn
            out["gmres_s_per_step"]["nn"] = nn["nn"]["seconds"]
        except Exception as ex:  # recorded; the exit status reports it
            errors["nn_precond"] = f"{type(ex).__name__}: {ex}"
            log(f"nn leg failed: {errors['nn_precond']}")
        torch.cuda.empty_cache()
    if args.explicit_steps > 0:
        try:
            sim = Simulation(wl.dim, wl.n, wl.dx, theta=wl.theta, dt=0.25, lf_E=False, lf_B=False,
                             beta_lim=wl.beta_lim, a_mode=wl.a_mode, comoving=wl.comoving,
                             n_smooth_u=wl.n_smooth_u, fp32=wl.fp32, ns_j=args.ns_j)
            for s in range(wl.nsp):
                p = synth.particles(wl, s, f32=wl.fp32)
                t = {k: torch.from_numpy(v).cuda() for k, v in p.items()}
                del p
                sim.add_species(wl.q[s], wl.m[s], t["cell"], t["off"], t["v"], t["w"])
                del t
                torch.cuda.synchronize()
            E, B = synth.fields(wl)
            sim.set_fields(torch.from_numpy(E).cuda(), torch.from_numpy(B).cuda())
            sim.explicit_step()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(sim.stream)
            for _ in range(args.explicit_steps):
                sim.explicit_step()
            ev1.record(sim.stream)
            ev1.synchronize()
            ms = ev0.elapsed_time(ev1) / args.explicit_steps
            sim.close()
            out["explicit_step"] = {"steps": args.explicit_steps, "dt": 0.25, "ms_per_step": round(ms, 3),
                                    "particle_steps_per_s": npart / (ms * 1e-3)}
            log(f"explicit step: {ms:.3f} ms")
        except Exception as ex:
            errors["explicit_step"] = f"{type(ex).__name__}: {ex}"
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on samples")
        try:
            procs = args.cpu_procs or min(16, os.cpu_count() or 1)
            out["cpu_baseline"] = cpu_baseline(args.workload if wl.dim == 3 else "c5", args.cpu_box, procs)
        except Exception as ex:
            errors["cpu_baseline"] = f"{type(ex).__name__}: {ex}"
    if errors:
        out["errors"] = errors
    print(json.dumps(out), flush=True)
    if errors:
        sys.exit(1)


if __name__ == "__main__":
    main()
