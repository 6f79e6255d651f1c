"""The explicit-PIC current (Sec. 3.1, explicit form) on the GPU path against
the oracle, on seeded synthetic inputs (1e-10 FP64, 1e-5 FP32 relative), and
the state rule that the implicit solve needs a new deposit afterwards."""
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


def _wl(dim, n, ppc, base, fp32):
    wl = synth.small("expl", dim=dim, n=n, ppc=ppc, base=base, fp32=fp32)
    return wl.replace(dx=(0.5, 1, 1)) if dim == 1 else wl


@pytest.mark.parametrize("ns_j", [0, 2])
@pytest.mark.parametrize("comoving", [True, False])
@pytest.mark.parametrize("name,dim,n,ppc,base,fp32", CASES)
def test_explicit_current_matches_oracle(name, dim, n, ppc, base, fp32, comoving, ns_j):
    print(f"[gpu] explicit current {name} comoving={comoving} ns_j={ns_j}", flush=True)
    wl = _wl(dim, n, ppc, base, fp32)
    parts = H.species_arrays(wl, fp32)
    E, B = H.perturbed_fields(wl)
    G, sp = H.oracle_species(wl, parts)
    ref = O.explicit_current(G, sp, comoving, n_smooth_u=wl.n_smooth_u, n_smooth_j=ns_j)
    sim = H.make_sim(wl, parts, E, B, comoving=comoving, ns_j=ns_j)
    J = sim.explicit_current().cpu().numpy()
    assert H.relerr(J, ref) < (1e-5 if fp32 else 1e-10)
    assert np.array_equal(sim.gather("J_eff").cpu().numpy(), J)
    sim.close()


def test_explicit_current_then_implicit_step_needs_a_new_deposit():
    print("[gpu] explicit current state rule", flush=True)
    from paper_2506_11320_amd import GlecsimError
    wl = _wl(2, (6, 5, 1), 30, "c2", False)
    parts = H.species_arrays(wl, False)
    E, B = H.perturbed_fields(wl)
    sim = H.make_sim(wl, parts, E, B)
    sim.explicit_current()
    with pytest.raises(GlecsimError):
        sim.solve(tol=1e-10)
    # a full step afterwards is the same as on a fresh context
    sim.step(tol=1e-12, maxit=500, restart=30)
    ref = H.make_sim(wl, parts, E, B)
    ref.step(tol=1e-12, maxit=500, restart=30)
    for f in ("E", "B"):
        assert np.array_equal(sim.gather(f).cpu().numpy(), ref.gather(f).cpu().numpy())
    sim.close()
    ref.close()


@pytest.mark.parametrize("comoving", [True, False])
@pytest.mark.parametrize("name,dim,n,ppc,base,fp32", CASES)
def test_explicit_step_matches_oracle(name, dim, n, ppc, base, fp32, comoving):
    """Three explicit PIC steps (Boris push, explicit-form current, leapfrog
    fields) against the oracle's explicit_step; dt = 0.2 keeps c dt below
    dx / sqrt(dim)."""
    print(f"[gpu] explicit step {name} comoving={comoving}", flush=True)
    wl = _wl(dim, n, ppc, base, fp32).replace(dt=0.2)
    parts = H.species_arrays(wl, fp32)
    E, B = H.perturbed_fields(wl)
    G, sp = H.oracle_species(wl, parts)
    sim = H.make_sim(wl, parts, E, B, comoving=comoving, ns_j=1)
    Eo, Bo = E, B
    for _ in range(3):
        r = O.explicit_step(G, sp, Eo, Bo, dt=wl.dt, comoving=comoving, n_smooth_u=wl.n_smooth_u, n_smooth_j=1)
        sp, Eo, Bo = r["species"], r["E"], r["B"]
        sim.explicit_step()
    tol = 1e-5 if fp32 else 1e-10
    assert H.relerr(sim.gather("E").cpu().numpy(), Eo) < tol
    assert H.relerr(sim.gather("B").cpu().numpy(), Bo) < tol
    for s in range(wl.nsp):
        got = sim.particles(s)["v"].cpu().numpy().astype(np.float64)
        for d in range(3):
            ref = np.sort(sp[s].v[:, d])
            assert np.abs(np.sort(got[d]) - ref).max() < (1e-5 if fp32 else 1e-12) * max(1.0, np.abs(ref).max())
    sim.close()


def test_explicit_light_wave_on_gpu():
    """The leapfrog's discrete eigenmode in vacuum (one weightless particle per
    cell): E_y = cos(k x_i - w M dt) after M steps, with
    sin(w dt/2) = (c dt/dx) sin(k dx/2)."""
    print("[gpu] explicit light wave", flush=True)
    from paper_2506_11320_amd import Simulation
    n, dx, dt, M = 32, 0.1, 0.07, 40
    xn = np.arange(n) * dx
    xc = xn + 0.5 * dx
    k = 2 * np.pi * 3 / (n * dx)
    w = 2.0 / dt * np.arcsin(dt / dx * np.sin(k * dx / 2))
    E = np.zeros((3, n)); E[1] = np.cos(k * xn)
    B = np.zeros((3, n)); B[2] = np.cos(k * xc - 0.5 * w * dt) + 0.5 * dt * (np.roll(E[1], -1) - E[1]) / dx
    sim = Simulation(1, (n, 1, 1), (dx, 1, 1), theta=0.5, dt=dt, comoving=False, n_smooth_u=0)
    dev = sim.device
    off = torch.zeros((3, n), dtype=torch.float64, device=dev)
    off[0] = 0.5
    sim.add_species(-1.0, 1.0, torch.arange(n, dtype=torch.int32, device=dev), off,
                    torch.zeros((3, n), dtype=torch.float64, device=dev), torch.zeros(n, dtype=torch.float64, device=dev))
    sim.set_fields(torch.from_numpy(E).to(dev), torch.from_numpy(B).to(dev))
    for _ in range(M):
        sim.explicit_step()
    Eg = sim.gather("E").cpu().numpy()
    assert np.max(np.abs(Eg[1] - np.cos(k * xn - w * M * dt))) < 1e-11
    sim.close()


def _explicit_drift_gpu(comoving, ns_j, steps):
    wl = synth.workloads()["ff1d"].replace(dt=0.5)
    parts = H.species_arrays(wl, False)
    E, B = synth.fields(wl)
    sim = H.make_sim(wl, parts, E, B, comoving=comoving, ns_j=ns_j)
    P0 = sum(p[0] for p in sim.diagnostics()["P"])
    drift = 0.0
    for _ in range(steps):
        sim.explicit_step()
        drift = max(drift, abs(sum(p[0] for p in sim.diagnostics()["P"]) - P0) / abs(P0))
    sim.close()
    return drift


def test_comoving_current_stabilises_an_explicit_fast_flow_on_gpu():
    """The Sec. 4.2 fast flow with the explicit step on the GPU path: the
    comoving current keeps the momentum drift more than ten times below the
    lab-frame current's (as on the oracle)."""
    print("[gpu] explicit fast flow", flush=True)
    lab0, cm0 = _explicit_drift_gpu(False, 0, 120), _explicit_drift_gpu(True, 0, 120)
    lab1, cm1 = _explicit_drift_gpu(False, 1, 400), _explicit_drift_gpu(True, 1, 400)
    print(f"  max |dP/P|: 120 steps lab {lab0:.3e} comoving {cm0:.3e}; 400 steps with one smoothing pass "
          f"lab {lab1:.3e} comoving {cm1:.3e}", flush=True)
    assert cm0 < 0.1 * lab0 and cm1 < 0.1 * lab1
