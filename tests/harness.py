"""Shared helpers of the GPU parity tests: build a GPU context and the oracle
state from the same seeded synthetic inputs, and compare them."""
from __future__ import annotations

import math

import numpy as np

import oracle as O
import synth

try:
    import torch
except Exception:  # pragma: no cover
    torch = None


def relerr(a, b, scale=None) -> float:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    s = np.linalg.norm(b) if scale is None else scale
    d = np.linalg.norm(a - b)
    if s == 0:
        return d
    return d / s


def perturbed_fields(wl, seed=99, amp=0.02):
    """Initial fields plus a seeded smooth-ish perturbation, so that the
    limiter ratios take every branch."""
    E, B = synth.fields(wl)
    rng = np.random.default_rng(seed)
    E = E + amp * rng.standard_normal(E.shape)
    B = B + amp * rng.standard_normal(B.shape)
    return E, B


def species_arrays(wl, f32: bool):
    """Generator output per species (FP32-rounded when f32)."""
    return [synth.particles(wl, s, f32=f32) for s in range(wl.nsp)]


def oracle_species(wl, parts):
    G = O.grid(wl.dim, wl.n, wl.dx, bc=wl.bc)
    out = []
    for s, p in enumerate(parts):
        x = O.global_positions(G, p["cell"], p["off"].astype(np.float64))
        out.append(O.Species(wl.q[s], wl.m[s], x, p["v"].astype(np.float64).T, p["w"].astype(np.float64)))
    return G, out


def make_sim(wl, parts, E, B, **over):
    from paper_2506_11320_amd import Simulation
    kw = dict(theta=wl.theta, dt=wl.dt, lf_E=wl.lf_E, lf_B=wl.lf_B, beta_lim=wl.beta_lim, a_mode=wl.a_mode,
              a_const=1.0, comoving=wl.comoving, n_smooth_u=wl.n_smooth_u, fp32=wl.fp32, bc=wl.bc)
    kw.update(over)
    sim = Simulation(wl.dim, wl.n, wl.dx, **kw)
    dev = sim.device
    for s, p in enumerate(parts):
        t = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in p.items()}
        sim.add_species(wl.q[s], wl.m[s], t["cell"], t["off"], t["v"], t["w"])
    sim.set_fields(torch.from_numpy(np.ascontiguousarray(E)).to(dev), torch.from_numpy(np.ascontiguousarray(B)).to(dev))
    return sim


def half_from_full(M27, dim):
    """Oracle's full 27-offset stencil -> the library's half-stencil layout."""
    return np.stack([M27[O.off27(o)] for o in O.half_offsets(dim)])


def oracle_grid_pass(wl, G, sp, E, B, comoving=None, beta_lim=None, a_mode=None, lf_E=None, lf_B=None,
                     n_smooth_j=0):
    comoving = wl.comoving if comoving is None else comoving
    dep = O.deposit(G, sp, wl.dt, B, comoving, wl.n_smooth_u, n_smooth_j=n_smooth_j)
    a_node = O.diffusion_speed(G, dep["u"], wl.a_mode if a_mode is None else a_mode, 1.0)
    bl = wl.beta_lim if beta_lim is None else beta_lim
    dep["kE"] = O.kappa_E(G, E, a_node, bl) if (wl.lf_E if lf_E is None else lf_E) else None
    dep["kB"] = O.kappa_B(G, B, a_node, bl) if (wl.lf_B if lf_B is None else lf_B) else None
    P = O.params(wl.theta, wl.dt)
    dep["rhs"] = O.rhs(G, P, E, B, dep["J_eff"])
    dep["P"] = P
    # per-species lab currents (normalisation of the J error: they cancel)
    Js = []
    for s in sp:
        a = O.deposit_species(G, s.q, s.m, O.beta_s(s.q, s.m, wl.dt), s.x, s.v, s.w, dep["Bn"])
        Js.append(a["J"])
    dep["J_s"] = Js
    dep["J_scale"] = sum(np.linalg.norm(j) for j in Js)
    return dep


def make_bare_sim(wl, **over):
    """A context with the workload's grid and parameters and no species (for
    ge_restore)."""
    from paper_2506_11320_amd import Simulation
    kw = dict(theta=wl.theta, dt=wl.dt, lf_E=wl.lf_E, lf_B=wl.lf_B, beta_lim=wl.beta_lim, a_mode=wl.a_mode,
              a_const=1.0, comoving=wl.comoving, n_smooth_u=wl.n_smooth_u, fp32=wl.fp32, bc=wl.bc)
    kw.update(over)
    return Simulation(wl.dim, wl.n, wl.dx, **kw)
