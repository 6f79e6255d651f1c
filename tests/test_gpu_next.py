"""Parity of the HIP path with the FP64 oracle for the current smoothing
(Sec. 3.2, ns_j filter passes on the comoving-frame current) and the
divergence cleaning of B (Sec. 2.3, cell-centred scalar psi), on seeded
synthetic inputs; tolerances as in test_gpu_parity (1e-10 FP64, 1e-5 FP32)."""
import math

import numpy as np
import pytest

import oracle as O
import synth
from tests import harness as H

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [
    ("1d_fp64", 1, (13, 1, 1), 70, "c1", False),
    ("2d_fp32", 2, (7, 5, 1), 70, "c3", True),
    ("3d_fp64", 3, (5, 3, 3), 70, "c5", False),
    ("3d_fp32", 3, (5, 4, 3), 70, "c5", True),
]


def _wl(dim, n, ppc, base, fp32, **kw):
    wl = synth.small("next", dim=dim, n=n, ppc=ppc, base=base, fp32=fp32)
    if dim == 1:
        wl = wl.replace(dx=(0.5, 1, 1))
    return wl.replace(lf_E=True, lf_B=True, beta_lim=1.5, **kw)


def _tol(fp32):
    return 1e-5 if fp32 else 1e-10


@pytest.mark.parametrize("comoving", [True, False])
@pytest.mark.parametrize("ns_j", [1, 3])
@pytest.mark.parametrize("name,dim,n,ppc,base,fp32", CASES)
def test_smoothed_current_matches_oracle(name, dim, n, ppc, base, fp32, ns_j, comoving):
    print(f"[gpu] smoothed current {name} ns_j={ns_j} comoving={comoving}", flush=True)
    wl = _wl(dim, n, ppc, base, fp32, comoving=comoving)
    parts = H.species_arrays(wl, fp32)
    E, B = H.perturbed_fields(wl)
    G, sp = H.oracle_species(wl, parts)
    ref = H.oracle_grid_pass(wl, G, sp, E, B, n_smooth_j=ns_j)
    sim = H.make_sim(wl, parts, E, B, ns_j=ns_j)
    sim.deposit()
    tol = _tol(fp32)
    assert H.relerr(sim.gather("J_eff").cpu().numpy(), ref["J_eff"], ref["J_scale"]) < tol
    assert H.relerr(sim.gather("rhs").cpu().numpy(), ref["rhs"]) < tol
    # the smoothing changed the current (the test is not vacuous)
    raw = H.oracle_grid_pass(wl, G, sp, E, B, n_smooth_j=0)
    assert H.relerr(ref["J_eff"], raw["J_eff"], ref["J_scale"]) > 100 * tol
    sim.close()


@pytest.mark.parametrize("name,dim,n,ppc,base,fp32", CASES)
def test_cleaning_update_matches_oracle(name, dim, n, ppc, base, fp32):
    print(f"[gpu] divergence cleaning {name}", flush=True)
    wl = _wl(dim, n, ppc, base, fp32)
    parts = H.species_arrays(wl, fp32)
    E, B = H.perturbed_fields(wl)
    G, sp = H.oracle_species(wl, parts)
    ref = H.oracle_grid_pass(wl, G, sp, E, B)
    sim = H.make_sim(wl, parts, E, B, dedner=True, ch_frac=0.8, dedner_damp=0.1)
    sim.deposit()
    rng = np.random.default_rng(23)
    Eth = E + 0.05 * rng.standard_normal(E.shape)
    psi0 = 0.3 * rng.standard_normal(O.nnodes(G))
    sim.set("Eth", torch.from_numpy(Eth))
    sim.set("psi", torch.from_numpy(psi0))
    sim.update_fields()
    ch = O.cleaning_speed(G, wl.dt, 0.8)
    psi_ref = O.dedner_psi(G, wl.dt, psi0, B, ch, 0.1)
    B_ref = O.update_B(G, ref["P"], B, Eth, ref["kB"]) - wl.dt * O.grad_cc(G, psi_ref)
    assert H.relerr(sim.gather("psi").cpu().numpy(), psi_ref) < 1e-12
    assert H.relerr(sim.gather("B").cpu().numpy(), B_ref) < _tol(fp32)
    sim.close()


def test_full_step_with_smoothing_and_cleaning_c1():
    """One full step of the 1D shock tube (C1 at full size) with ns_j = 2 and
    the cleaning on: E, B, psi and the particles against the oracle's step."""
    print("[gpu] full step c1 + smoothing + cleaning", flush=True)
    wl = synth.workloads()["c1"].replace(lf_E=True, lf_B=True, comoving=True)
    parts = H.species_arrays(wl, False)
    E, B = synth.fields(wl)
    rng = np.random.default_rng(31)
    B = B + 0.01 * rng.standard_normal(B.shape)  # a divergent part for the cleaning to act on
    G, sp = H.oracle_species(wl, parts)
    r = O.step(G, sp, E, B, dt=wl.dt, theta=wl.theta, comoving=True, lf_E=True, lf_B=True,
               beta_lim=wl.beta_lim, a_mode=wl.a_mode, tol=1e-13, restart=40, n_smooth_j=2, dedner=True)
    sim = H.make_sim(wl, parts, E, B, ns_j=2, dedner=True)
    rep = sim.step(tol=1e-13, maxit=2000, restart=40)
    assert rep["converged"]
    assert H.relerr(sim.gather("E").cpu().numpy(), r["E"]) < 1e-10
    assert H.relerr(sim.gather("B").cpu().numpy(), r["B"]) < 1e-10
    assert H.relerr(sim.gather("psi").cpu().numpy(), r["psi"]) < 1e-10
    assert np.linalg.norm(r["psi"]) > 0
    for s in range(wl.nsp):
        got = {k: v.cpu().numpy() for k, v in sim.particles(s).items()}
        assert np.abs(np.sort(got["v"][0]) - np.sort(r["species"][s].v[:, 0])).max() < 1e-12
    sim.close()


def test_cleaning_off_leaves_psi_at_zero():
    wl = _wl(2, (6, 5, 1), 20, "c2", False)
    parts = H.species_arrays(wl, False)
    E, B = H.perturbed_fields(wl)
    sim = H.make_sim(wl, parts, E, B)
    sim.step(tol=1e-10, maxit=500, restart=30)
    assert np.array_equal(sim.gather("psi").cpu().numpy(), np.zeros(sim.N))
    sim.close()
