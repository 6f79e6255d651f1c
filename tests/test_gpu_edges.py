"""Edge cases of the GPU path against the oracle: empty cells (ragged
occupancy), an empty species, dense FP64 cells, and the error a caller gets
when a particle moves a cell or more in one step (the mover clamps it and
every kernel still finishes normally)."""
import numpy as np
import pytest

import oracle as O
import synth
from tests import harness as H

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _subset(p, keep):
    return {"cell": np.ascontiguousarray(p["cell"][keep]), "off": np.ascontiguousarray(p["off"][:, keep]),
            "v": np.ascontiguousarray(p["v"][:, keep]), "w": np.ascontiguousarray(p["w"][keep])}


def _ragged(wl, fp32):
    """Species 0 without the particles of every third cell (and, in 3D, of a
    whole plane), species 1 with none at all."""
    parts = H.species_arrays(wl, fp32)
    cell = parts[0]["cell"]
    keep = cell % 3 != 1
    if wl.dim == 3:
        keep &= cell // (wl.n[0] * wl.n[1]) != 1
    return [_subset(parts[0], keep), _subset(parts[1], np.zeros(parts[1]["cell"].size, bool))]


CASES = [("1d_fp64", 1, (13, 1, 1), 40, "c1", False), ("2d_fp32", 2, (7, 5, 1), 40, "c3", True),
         ("3d_fp64", 3, (5, 4, 3), 40, "c5", False), ("3d_fp32", 3, (5, 4, 3), 40, "c5", True)]


def _wl(dim, n, ppc, base, fp32):
    wl = synth.small("edges", dim=dim, n=n, ppc=ppc, base=base, fp32=fp32)
    if dim == 1:
        wl = wl.replace(dx=(0.5, 1, 1))
    return wl.replace(lf_E=True, lf_B=True, comoving=True, beta_lim=1.5)


@pytest.mark.parametrize("name,dim,n,ppc,base,fp32", CASES)
def test_empty_cells_and_empty_species(name, dim, n, ppc, base, fp32):
    print(f"[gpu] ragged occupancy {name}", flush=True)
    wl = _wl(dim, n, ppc, base, fp32)
    parts = _ragged(wl, fp32)
    assert parts[1]["cell"].size == 0
    E, B = H.perturbed_fields(wl)
    G, sp = H.oracle_species(wl, parts)
    ref = H.oracle_grid_pass(wl, G, sp, E, B)
    sim = H.make_sim(wl, parts, E, B)
    sim.deposit()
    tol = 1e-5 if fp32 else 1e-10
    assert H.relerr(sim.gather("J_lab").cpu().numpy(), ref["J_lab"]) < tol
    assert H.relerr(sim.gather("Mt").cpu().numpy(), H.half_from_full(ref["Mt"], dim)) < tol
    assert H.relerr(sim.gather("mass").cpu().numpy(), ref["mass"]) < tol
    assert H.relerr(sim.gather("u").cpu().numpy(), ref["u"]) < tol
    assert H.relerr(sim.gather("J_eff").cpu().numpy(), ref["J_eff"]) < tol
    rho = sim.gather("rho").cpu().numpy()
    assert H.relerr(rho[0], ref["rho_s"][0]) < tol and not rho[1].any()
    # one full step: fields and the particles of both species
    r = O.step(G, sp, E, B, dt=wl.dt, theta=wl.theta, comoving=True, lf_E=True, lf_B=True,
               beta_lim=wl.beta_lim, a_mode=wl.a_mode, n_smooth_u=wl.n_smooth_u, tol=1e-13, restart=40)
    sim2 = H.make_sim(wl, parts, E, B)
    assert sim2.step(tol=1e-13, maxit=2000, restart=40)["converged"]
    assert H.relerr(sim2.gather("E").cpu().numpy(), r["E"]) < tol
    assert H.relerr(sim2.gather("B").cpu().numpy(), r["B"]) < tol
    got = {k: v.cpu().numpy() for k, v in sim2.particles(0).items()}
    assert got["cell"].size == parts[0]["cell"].size
    assert np.abs(np.sort(got["v"][0].astype(np.float64)) - np.sort(r["species"][0].v[:, 0])).max() < (
        1e-5 if fp32 else 1e-12)
    assert sim2.particles(1)["cell"].numel() == 0
    sim.close()
    sim2.close()


@pytest.mark.parametrize("dim,n", [(2, (5, 4, 1)), (3, (4, 3, 3))])
def test_dense_cells_fp64(dim, n):
    """More than 128 particles per cell in FP64: the multi-chunk deposit and
    the two-pass push."""
    print(f"[gpu] dense fp64 dim={dim}", flush=True)
    wl = _wl(dim, n, 150, "c2" if dim == 2 else "c5", False)
    parts = H.species_arrays(wl, False)
    E, B = H.perturbed_fields(wl)
    G, sp = H.oracle_species(wl, parts)
    r = O.step(G, sp, E, B, dt=wl.dt, theta=wl.theta, comoving=True, lf_E=True, lf_B=True,
               beta_lim=wl.beta_lim, a_mode=wl.a_mode, n_smooth_u=wl.n_smooth_u, tol=1e-13, restart=40)
    sim = H.make_sim(wl, parts, E, B)
    assert sim.step(tol=1e-13, maxit=2000, restart=40)["converged"]
    assert H.relerr(sim.gather("E").cpu().numpy(), r["E"]) < 1e-10
    assert H.relerr(sim.gather("B").cpu().numpy(), r["B"]) < 1e-10
    for s in range(wl.nsp):
        got = sim.particles(s)["v"].cpu().numpy()
        assert np.abs(np.sort(got[0]) - np.sort(r["species"][s].v[:, 0])).max() < 1e-12
    sim.close()


def test_particle_crossing_cells_is_resorted_and_reported():
    """A particle moving three cells in one step is re-sorted into its cell
    (no error) and counted by ge_moves."""
    print("[gpu] far move report", flush=True)
    wl = _wl(2, (6, 5, 1), 20, "c2", False)
    parts = H.species_arrays(wl, False)
    parts[0]["v"][0, 7] = 3.0 * wl.dx[0] / wl.dt  # three cells in one step
    E, B = H.perturbed_fields(wl)
    sim = H.make_sim(wl, parts, E, B)
    sim.step(tol=1e-10, maxit=500, restart=30)
    mv = sim.moves()
    assert mv["far_moves"][0] == 1 and mv["far_moves"][1] == 0 and mv["resorts"] == 1
    assert 2.5 < mv["max_move"][0] < 3.5
    got = sim.particles(0)
    assert got["cell"].numel() == parts[0]["cell"].size
    assert bool((got["cell"][1:] >= got["cell"][:-1]).all())
    sim.close()


@pytest.mark.parametrize("name,dim,n,ppc,base,fp32", CASES)
def test_explicit_step_with_empty_cells_and_species(name, dim, n, ppc, base, fp32):
    """The explicit step (two light particle passes, Boris push, leapfrog) on
    ragged occupancy with an empty species, against the oracle."""
    print(f"[gpu] explicit ragged {name}", flush=True)
    wl = _wl(dim, n, ppc, base, fp32).replace(dt=0.2)
    parts = _ragged(wl, fp32)
    E, B = H.perturbed_fields(wl)
    G, sp = H.oracle_species(wl, parts)
    r = O.explicit_step(G, sp, E, B, dt=wl.dt, comoving=True, n_smooth_u=wl.n_smooth_u)
    sim = H.make_sim(wl, parts, E, B)
    sim.explicit_step()
    tol = 1e-5 if fp32 else 1e-10
    assert H.relerr(sim.gather("E").cpu().numpy(), r["E"]) < tol
    assert H.relerr(sim.gather("B").cpu().numpy(), r["B"]) < tol
    assert H.relerr(sim.gather("J_eff").cpu().numpy(), r["J"]) < tol
    assert sim.particles(1)["cell"].numel() == 0
    sim.close()


def test_phase_timings_of_a_step():
    """ge_timings: every timed phase of a step is positive, the re-binning's
    own kernels (slot 6) are part of the push phase (slot 0), and the call
    resets the accumulators."""
    print("[gpu] phase timings", flush=True)
    wl = _wl(3, (6, 5, 4), 20, "c5", True)
    parts = H.species_arrays(wl, True)
    E, B = H.perturbed_fields(wl)
    sim = H.make_sim(wl, parts, E, B)
    for _ in range(2):
        sim.step(tol=1e-8, maxit=500, restart=30)
    t = sim.timings()
    assert t[7] == 2
    assert all(v > 0 for v in t[:7]), t
    assert t[6] < t[0], t
    assert sim.timings() == [0.0] * 8
    sim.close()
