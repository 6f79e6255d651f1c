"""Parity of the HIP path (through the C ABI) with the FP64 oracle, element by
element, on seeded synthetic inputs of small grids that span several
workgroups, a ragged tail of cells and cells holding more than one 64-particle
chunk.  Tolerances (normwise relative, currents normalised by the sum of the
species' current norms because they cancel between species): 1e-10 for the
FP64 path, 1e-5 for the FP32 deposit/push path."""
import math

import numpy as np
import pytest

import oracle as O
import synth
from tests import harness as H

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [
    # name, dim, n, ppc, base workload, fp32
    ("1d_fp64", 1, (13, 1, 1), 70, "c1", False),
    ("2d_fp64", 2, (7, 5, 1), 70, "c2", False),
    ("2d_fp32", 2, (7, 5, 1), 70, "c3", True),
    ("3d_fp64", 3, (5, 3, 3), 70, "c5", False),
    ("3d_fp32", 3, (5, 3, 3), 70, "c5", True),
    # more than 128 particles per cell: the two-pass push and 3-chunk deposit
    ("3d_fp32_dense", 3, (4, 3, 3), 150, "c5", True),
    # the paper's baseline particle count (Table 1: 1600 per cell per species),
    # 25 chunks per species and cell in FP32
    ("2d_fp32_1600ppc", 2, (4, 3, 1), 1600, "c3", True),
]


def _wl(dim, n, ppc, base, fp32, **kw):
    wl = synth.small("parity", dim=dim, n=n, ppc=ppc, base=base, fp32=fp32)
    if dim == 1:
        wl = wl.replace(dx=(0.5, 1, 1))
    return wl.replace(lf_E=True, lf_B=True, comoving=True, beta_lim=1.5, **kw)


def _tol(fp32):
    return 1e-5 if fp32 else 1e-10


@pytest.mark.parametrize("name,dim,n,ppc,base,fp32", CASES)
def test_deposit_and_grid_pass(name, dim, n, ppc, base, fp32):
    print(f"[gpu] deposit parity {name}", flush=True)
    _check_deposit_and_grid_pass(_wl(dim, n, ppc, base, fp32), dim, fp32)


@pytest.mark.parametrize("fp32", [False, True])
def test_deposit_with_four_species(fp32):
    """Four species (the most the library holds): species 0 and 1 take the
    deposit's prefetched path, species 2 and 3 the general one (every particle
    located through the cell's run table); 150 particles per cell and species
    give three 64-particle chunks each (compensated chunk sums in FP32)."""
    print(f"[gpu] deposit parity, four species, fp32={fp32}", flush=True)
    wl = synth.small("four_species", dim=3, n=(6, 5, 4), ppc=150, fp32=fp32, base="c5")
    wl = wl.replace(q=(-1.0, 1.0, 1.0, -1.0), m=(1.0, 100.0, 16.0, 1.0), vth=(wl.vth[0], wl.vth[1], 0.02, 0.08),
                    dsheet=(wl.dsheet[0], wl.dsheet[1], 0.0, 0.0))
    assert wl.nsp == 4
    _check_deposit_and_grid_pass(wl, 3, fp32)


def _check_deposit_and_grid_pass(wl, dim, fp32):
    parts = H.species_arrays(wl, fp32)
    E, B = H.perturbed_fields(wl)
    G, sp = H.oracle_species(wl, parts)
    ref = H.oracle_grid_pass(wl, G, sp, E, B)
    sim = H.make_sim(wl, parts, E, B)
    sim.deposit()
    g = {k: sim.gather(k).cpu().numpy() for k in ["Bn", "J_lab", "J_eff", "rho", "mm", "mass", "u", "EM", "Mt",
                                                  "M0", "kappa_E", "kappa_B", "rhs"]}
    tol = _tol(fp32)
    errs = {"J_lab": H.relerr(g["J_lab"], ref["J_lab"], ref["J_scale"]),
            "Mt": H.relerr(g["Mt"], H.half_from_full(ref["Mt"], dim)),
            "M0": H.relerr(g["M0"], H.half_from_full(ref["M0"], dim)),
            "J_eff": H.relerr(g["J_eff"], ref["J_eff"], ref["J_scale"])}
    print("  errors " + " ".join(f"{k} {v:.2e}" for k, v in errs.items()), flush=True)
    assert H.relerr(g["Bn"], ref["Bn"]) < 1e-14
    assert H.relerr(g["J_lab"], ref["J_lab"], ref["J_scale"]) < tol
    assert H.relerr(g["Mt"], H.half_from_full(ref["Mt"], dim)) < tol
    assert H.relerr(g["M0"], H.half_from_full(ref["M0"], dim)) < tol
    for s in range(wl.nsp):
        assert H.relerr(g["rho"][s], ref["rho_s"][s]) < tol
    assert H.relerr(g["mm"], ref["mm"]) < tol
    assert H.relerr(g["mass"], ref["mass"]) < tol
    assert H.relerr(g["u"], ref["u"]) < tol
    assert H.relerr(g["EM"], ref["EM"]) < tol
    # comoving current: GPU form J_lab - (M0 u + Mt E_M)/dV vs the oracle's
    # literal second deposit with u(x_p)
    assert H.relerr(g["J_eff"], ref["J_eff"], ref["J_scale"]) < tol
    assert H.relerr(g["kappa_E"], ref["kE"]) < tol
    assert H.relerr(g["kappa_B"], ref["kB"]) < tol
    assert H.relerr(g["rhs"], ref["rhs"]) < tol
    sim.close()


@pytest.mark.parametrize("name,dim,n,ppc,base,fp32", CASES)
def test_operator_and_solve(name, dim, n, ppc, base, fp32):
    print(f"[gpu] operator/solve parity {name}", flush=True)
    wl = _wl(dim, n, ppc, base, fp32)
    parts = H.species_arrays(wl, fp32)
    E, B = H.perturbed_fields(wl)
    G, sp = H.oracle_species(wl, parts)
    ref = H.oracle_grid_pass(wl, G, sp, E, B)
    sim = H.make_sim(wl, parts, E, B)
    sim.deposit()
    rng = np.random.default_rng(5)
    x = rng.standard_normal((3, G_N(G)))
    y = sim.apply_operator(torch.from_numpy(x).cuda()).cpu().numpy()
    y_ref = O.apply_A(G, ref["P"], ref["Mt"], ref["kE"], x)
    assert H.relerr(y, y_ref) < _tol(fp32)
    # solve to 1e-12 and compare with the oracle's dense direct solve
    rep = sim.solve(tol=1e-12, maxit=2000, restart=40)
    assert rep["converged"] and rep["relres"] <= 1e-12
    Eth = sim.gather("Eth").cpu().numpy()
    A = O.dense_A(G, ref["P"], ref["Mt"], ref["kE"])
    x_lu = O.dense_solve(A, ref["rhs"].ravel()).reshape(3, -1)
    assert H.relerr(Eth, x_lu) < (1e-5 if fp32 else 1e-10)
    # Jacobi-preconditioned GMRES reaches the same solution
    rep2 = sim.solve(tol=1e-12, maxit=2000, restart=40, precond=1)
    assert rep2["converged"]
    assert H.relerr(sim.gather("Eth").cpu().numpy(), x_lu) < (1e-5 if fp32 else 1e-10)
    sim.close()


def G_N(G):
    return O.nnodes(G)


@pytest.mark.parametrize("name,dim,n,ppc,base,fp32", CASES)
def test_push_and_stable_rebinning(name, dim, n, ppc, base, fp32):
    """Mover parity and the re-binning: the GPU order after the push is the
    stable sort by new cell of the previous order (checked bit-exactly for
    FP64 against numpy's stable argsort of the oracle's new cells)."""
    print(f"[gpu] push parity {name}", flush=True)
    wl = _wl(dim, n, ppc, base, fp32)
    parts = H.species_arrays(wl, fp32)
    # tag every particle with its index through the weight (the push only
    # carries w); integers up to 2^24 are exact in FP32
    for p in parts:
        p["w"] = (np.arange(p["w"].size) + 1).astype(p["w"].dtype)
    E, B = H.perturbed_fields(wl)
    rng = np.random.default_rng(11)
    Eth = E + 0.05 * rng.standard_normal(E.shape)
    G, sp = H.oracle_species(wl, parts)
    sim = H.make_sim(wl, parts, E, B)
    sim.deposit()
    sim.set("Eth", torch.from_numpy(Eth))
    sim.push()
    sim.sync()
    Bn = O.node_avg(G, B)
    L = np.array([wl.n[d] * wl.dx[d] for d in range(wl.dim)])
    for s in range(wl.nsp):
        got = {k: v.cpu().numpy() for k, v in sim.particles(s).items()}
        ids = np.rint(got["w"]).astype(np.int64) - 1
        assert np.array_equal(np.sort(ids), np.arange(ids.size))
        xo, vo = O.push_species(G, O.beta_s(wl.q[s], wl.m[s], wl.dt), wl.dt, sp[s].x, sp[s].v, Eth, Bn)
        # positions: periodic distance, velocities
        xg = O.global_positions(G, got["cell"], got["off"].astype(np.float64))
        dxp = (xg[:, :wl.dim] - xo[ids, :wl.dim] + 0.5 * L) % L - 0.5 * L
        scale = np.array(wl.dx[:wl.dim])
        assert np.abs(dxp / scale).max() < (2e-6 if fp32 else 1e-12)
        vscale = np.abs(vo).max()
        assert np.abs(got["v"].T.astype(np.float64) - vo[ids]).max() / vscale < (1e-5 if fp32 else 1e-12)
        # sort invariants at any size: cells non-decreasing, stable within a cell
        assert np.all(np.diff(got["cell"]) >= 0)
        same = np.diff(got["cell"]) == 0
        assert np.all(np.diff(ids)[same] > 0)
        if not fp32:
            cell_o = np.zeros(ids.size, np.int64)
            mul = 1
            for d in range(wl.dim):
                cell_o += (np.floor(xo[:, d] / wl.dx[d]).astype(np.int64) % wl.n[d]) * mul
                mul *= wl.n[d]
            order = O.stable_cell_order(cell_o)
            assert np.array_equal(ids, order)
            assert np.array_equal(got["cell"], cell_o[order])
    sim.close()


@pytest.mark.parametrize("name,dim,n,ppc,base,fp32", CASES)
def test_field_update(name, dim, n, ppc, base, fp32):
    print(f"[gpu] field update parity {name}", flush=True)
    wl = _wl(dim, n, ppc, base, fp32)
    parts = H.species_arrays(wl, fp32)
    E, B = H.perturbed_fields(wl)
    G, sp = H.oracle_species(wl, parts)
    ref = H.oracle_grid_pass(wl, G, sp, E, B)
    sim = H.make_sim(wl, parts, E, B)
    sim.deposit()
    rng = np.random.default_rng(17)
    Eth = E + 0.05 * rng.standard_normal(E.shape)
    sim.set("Eth", torch.from_numpy(Eth))
    sim.update_fields()
    Bg = sim.gather("B").cpu().numpy()
    Eg = sim.gather("E").cpu().numpy()
    B_ref = O.update_B(G, ref["P"], B, Eth, ref["kB"])
    E_ref = O.update_E(wl.theta, E, Eth)
    assert H.relerr(Bg, B_ref) < _tol(fp32)
    assert H.relerr(Eg, E_ref) < 1e-14
    sim.close()


@pytest.mark.parametrize("fp32", [False, True])
def test_deposit_is_deterministic(fp32):
    print(f"[gpu] determinism fp32={fp32}", flush=True)
    wl = _wl(3, (5, 3, 3), 70, "c5", fp32)
    parts = H.species_arrays(wl, fp32)
    E, B = H.perturbed_fields(wl)
    outs = []
    for _ in range(2):
        sim = H.make_sim(wl, parts, E, B)
        sim.deposit()
        outs.append({k: sim.gather(k).cpu().numpy() for k in ["Mt", "M0", "J_lab", "J_eff", "rhs"]})
        sim.close()
    for k in outs[0]:
        assert np.array_equal(outs[0][k], outs[1][k]), k


def test_cold_flow_comoving_equals_lab_on_gpu():
    print("[gpu] cold flow comoving", flush=True)
    wl = synth.workloads()["c2"].replace(n=(6, 5, 1), ppc=70, paired=True, vth=(0.0, 0.0))
    parts = H.species_arrays(wl, False)
    E, B = synth.fields(wl)
    sim = H.make_sim(wl, parts, E, B, comoving=True)
    sim.deposit()
    Jlab = sim.gather("J_lab").cpu().numpy()
    Jeff = sim.gather("J_eff").cpu().numpy()
    rho = sim.gather("rho").cpu().numpy()
    G, sp = H.oracle_species(wl, parts)
    ref = H.oracle_grid_pass(wl, G, sp, E, B, comoving=True)
    assert np.abs(rho.sum(axis=0)).max() < 1e-15
    assert np.linalg.norm(Jeff - Jlab) <= 1e-13 * ref["J_scale"]
    sim.close()


@pytest.mark.parametrize("dim,n", [(1, (16, 1, 1)), (2, (6, 5, 1)), (3, (4, 3, 3))])
def test_energy_conservation_over_steps(dim, n):
    """theta = 1/2, lab frame, no LF: W_E + W_B + K is conserved per step to
    the solver tolerance (ECSIM energy theorem), on the GPU path end to end."""
    print(f"[gpu] energy theorem dim={dim}", flush=True)
    base = {1: "c1", 2: "c2", 3: "c5"}[dim]
    wl = synth.small("energy", dim=dim, n=n, ppc=20, base=base).replace(theta=0.5)
    if dim == 1:
        wl = wl.replace(dx=(0.5, 1, 1))
    parts = H.species_arrays(wl, False)
    E, B = H.perturbed_fields(wl, amp=0.01)
    sim = H.make_sim(wl, parts, E, B, comoving=False, lf_E=False, lf_B=False)
    d0 = sim.diagnostics()
    W0 = d0["W_E"] + d0["W_B"] + sum(d0["K"])
    for _ in range(4):
        sim.step(tol=1e-13, maxit=2000, restart=40)
        d = sim.diagnostics()
        W = d["W_E"] + d["W_B"] + sum(d["K"])
        assert abs(W - W0) / W0 < 1e-11
    sim.close()


def test_full_step_matches_oracle_c1():
    """One full step of the 1D shock tube (C1 at its full size) from identical
    inputs: E^{n+1}, B^{n+1} and the particles."""
    print("[gpu] full step c1", flush=True)
    wl = synth.workloads()["c1"].replace(lf_E=True, lf_B=True, comoving=True)
    parts = H.species_arrays(wl, False)
    E, B = synth.fields(wl)
    G, sp = H.oracle_species(wl, parts)
    r = O.step(G, sp, E, B, dt=wl.dt, theta=wl.theta, comoving=True, lf_E=True, lf_B=True,
               beta_lim=wl.beta_lim, a_mode=wl.a_mode, tol=1e-13, restart=40)
    sim = H.make_sim(wl, parts, E, B)
    rep = sim.step(tol=1e-13, maxit=2000, restart=40)
    assert rep["converged"]
    assert H.relerr(sim.gather("E").cpu().numpy(), r["E"]) < 1e-10
    assert H.relerr(sim.gather("B").cpu().numpy(), r["B"]) < 1e-10
    L = wl.n[0] * wl.dx[0]
    for s in range(wl.nsp):
        got = {k: v.cpu().numpy() for k, v in sim.particles(s).items()}
        xo = r["species"][s].x
        cell_o = (np.floor(xo[:, 0] / wl.dx[0]).astype(np.int64)) % wl.n[0]
        order = O.stable_cell_order(cell_o)
        assert np.array_equal(got["cell"], cell_o[order])
        xg = (got["cell"] + got["off"][0]) * wl.dx[0]
        d = (xg - xo[order, 0] + 0.5 * L) % L - 0.5 * L
        assert np.abs(d).max() < 1e-12
        assert np.abs(got["v"].T - r["species"][s].v[order]).max() < 1e-12
    sim.close()


@pytest.mark.parametrize("name,dim,n,ppc,base,fp32", CASES)
def test_diagnostics_match_oracle(name, dim, n, ppc, base, fp32):
    """The FP64 reductions of ge_diagnostics against the oracle on the same
    state: W_E, W_B (fields), K_s and P_s (particles, the FP32 path's records
    widened exactly), and the Gauss residual with the charge density of the
    deposit (1e-10 in FP64, 1e-5 with the FP32 deposit)."""
    print(f"[gpu] diagnostics parity {name}", flush=True)
    wl = _wl(dim, n, ppc, base, fp32)
    parts = H.species_arrays(wl, fp32)
    E, B = H.perturbed_fields(wl)
    G, sp = H.oracle_species(wl, parts)
    dep = O.deposit(G, sp, wl.dt, B, wl.comoving, wl.n_smooth_u)
    ref = O.diagnostics(G, sp, E, B, rho_s=dep["rho_s"])
    sim = H.make_sim(wl, parts, E, B)
    sim.deposit()
    got = sim.diagnostics()
    assert abs(got["W_E"] - ref["W_E"]) <= 1e-12 * ref["W_E"]
    assert abs(got["W_B"] - ref["W_B"]) <= 1e-12 * ref["W_B"]
    for s in range(wl.nsp):
        assert abs(got["K"][s] - ref["K"][s]) <= 1e-12 * ref["K"][s]
        pscale = sp[s].m * np.sum(sp[s].w * np.linalg.norm(sp[s].v, axis=1))
        assert np.abs(np.array(got["P"][s]) - ref["P"][s]).max() <= 1e-12 * pscale
    assert ref["gauss"] > 0
    assert abs(got["gauss"] - ref["gauss"]) <= (1e-5 if fp32 else 1e-10) * ref["gauss"]
    sim.close()
