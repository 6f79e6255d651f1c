"""The walled x axis on the GPU (through the C ABI) against the oracle: a
reflecting, conducting wall at x = 0 with a wall or an inflow plane at x = L.
Element by element on small grids: the operator (boundary planes included),
full steps with specular reflection, losses through the inflow plane and
injected particles (particles compared in the library's cell order: the
stable sort by cell of the oracle's previous order, injected ones after the
others in their cell), and the diagnostics with half-weight boundary planes.
Tolerances as in the periodic parity tests: 1e-10 (FP64), 1e-5 (FP32)."""
import numpy as np
import pytest

import oracle as O
import synth
from tests import harness as H

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [
    # name, dim, n (physical cells), ppc, fp32, bc
    ("1d_fp64_inflow", 1, (12, 1, 1), 40, False, (1, 2)),
    ("2d_fp64_walls", 2, (7, 5, 1), 30, False, (1, 1)),
    ("3d_fp64_inflow", 3, (6, 4, 3), 20, False, (1, 2)),
    ("3d_fp32_inflow", 3, (6, 4, 3), 20, True, (1, 2)),
    ("3d_fp64_walls", 3, (6, 4, 3), 20, False, (1, 1)),
    ("2d_fp32_inflow", 2, (7, 5, 1), 30, True, (1, 2)),
]


def _wl(dim, n, ppc, fp32, bc):
    wl = synth.workloads()["c4"].replace(name="walls", dim=dim, n=n[:dim] + (1,) * (3 - dim),
                                         dx=(0.5, 0.5, 0.5)[:dim] + (1.0,) * (3 - dim), ppc=ppc, fp32=fp32, bc=bc)
    return wl.replace(lf_E=True, lf_B=True, comoving=True, beta_lim=1.5)


def _fields(wl, seed=99, amp=0.02):
    """Initial fields plus a perturbation that keeps the boundary values:
    tangential E zero on the wall planes, E and the ghost's B at the upstream
    values on an inflow plane."""
    E, B = synth.fields(wl)
    rng = np.random.default_rng(seed)
    i = np.arange(wl.ncells) % wl.nstore[0]
    nx = wl.n[0]
    dE = amp * rng.standard_normal(E.shape)
    dE[1:, i == 0] = 0.0
    dE[:, i == nx] = 0.0 if wl.bc[1] == 2 else dE[:, i == nx]
    if wl.bc[1] == 1:
        dE[1:, i == nx] = 0.0
    dB = amp * rng.standard_normal(B.shape)
    dB[:, i == nx] = 0.0
    return E + dE, B + dB


def _parts(wl, fp32, seed=5):
    """The generator's particles; some near each end get a fast x velocity so
    that they reflect or leave."""
    parts = H.species_arrays(wl, fp32)
    rng = np.random.default_rng(seed)
    for p in parts:
        ix = p["cell"] % wl.nstore[0]
        n = ix.size
        lo = (ix == 0) & (rng.random(n) < 0.5)
        hi = (ix == wl.n[0] - 1) & (rng.random(n) < 0.5)
        p["v"][0, lo] = (-0.7 * wl.dx[0] / wl.dt)
        p["v"][0, hi] = (0.8 * wl.dx[0] / wl.dt)
    return parts


def _canonical(G, wl, sp):
    """The oracle's particles in the library's order: stable sort by cell of
    the oracle's array order."""
    out = []
    for s in sp:
        cell = np.zeros(s.w.size, np.int64)
        mul = 1
        for d in range(wl.dim):
            cell += (np.floor(s.x[:, d] / wl.dx[d]).astype(np.int64) % G.n[d]) * mul
            mul *= G.n[d]
        o = O.stable_cell_order(cell)
        out.append((cell[o], s.x[o], s.v[o], s.w[o]))
    return out


@pytest.mark.parametrize("name,dim,n,ppc,fp32,bc", CASES)
def test_walled_operator_matches_oracle(name, dim, n, ppc, fp32, bc):
    print(f"[gpu] walled operator {name}", flush=True)
    wl = _wl(dim, n, ppc, fp32, bc)
    parts = _parts(wl, fp32)
    E, B = _fields(wl)
    G, sp = H.oracle_species(wl, parts)
    ref = H.oracle_grid_pass(wl, G, sp, E, B)
    sim = H.make_sim(wl, parts, E, B)
    sim.deposit()
    tol = 1e-5 if fp32 else 1e-10
    for k in ["Bn", "kappa_E", "kappa_B", "rhs"]:
        got = sim.gather(k).cpu().numpy()
        want = {"Bn": ref["Bn"], "kappa_E": ref["kE"], "kappa_B": ref["kB"], "rhs": ref["rhs"]}[k]
        assert H.relerr(got, want) < (1e-14 if k == "Bn" else tol), k
    assert H.relerr(sim.gather("J_eff").cpu().numpy(), ref["J_eff"], ref["J_scale"]) < tol
    x = np.random.default_rng(5).standard_normal((3, G_N(G)))
    y = sim.apply_operator(torch.from_numpy(x).cuda()).cpu().numpy()
    y_ref = O.apply_A(G, ref["P"], ref["Mt"], ref["kE"], x)
    assert H.relerr(y, y_ref) < tol
    rep = sim.solve(tol=1e-13, maxit=4000, restart=40)
    assert rep["converged"]
    A = O.dense_A(G, ref["P"], ref["Mt"], ref["kE"])
    x_lu = O.dense_solve(A, ref["rhs"].ravel()).reshape(3, -1)
    assert H.relerr(sim.gather("Eth").cpu().numpy(), x_lu) < tol
    rep = sim.solve(tol=1e-13, maxit=4000, restart=40, precond=1)  # Jacobi
    assert rep["converged"]
    sim.close()


def G_N(G):
    return O.nnodes(G)


@pytest.mark.parametrize("name,dim,n,ppc,fp32,bc", CASES)
def test_walled_steps_match_oracle(name, dim, n, ppc, fp32, bc):
    """Three steps with reflection, losses and (on an inflow plane) injection
    after each step, against the oracle's steps fed the same injected
    particles."""
    print(f"[gpu] walled steps {name}", flush=True)
    wl = _wl(dim, n, ppc, fp32, bc)
    parts = _parts(wl, fp32)
    E, B = _fields(wl)
    G, sp = H.oracle_species(wl, parts)
    sim = H.make_sim(wl, parts, E, B)
    tol = 1e-5 if fp32 else 1e-10
    ptol = 2e-6 if fp32 else 1e-12
    gone = 0
    for k in range(3):
        inj = [synth.inflow(wl, s, k, f32=fp32) for s in range(wl.nsp)] if bc[1] == 2 else [None] * wl.nsp
        inj_or = []
        for s, p in enumerate(inj):
            if p is None or p["cell"].size == 0:
                inj_or.append(None)
                continue
            x = O.global_positions(G, p["cell"], p["off"].astype(np.float64))
            inj_or.append((x, p["v"].astype(np.float64).T, p["w"].astype(np.float64)))
        r = O.step(G, sp, E, B, dt=wl.dt, theta=wl.theta, comoving=True, lf_E=True, lf_B=True,
                   beta_lim=wl.beta_lim, a_mode=wl.a_mode, solve="dense", inject=inj_or)
        sim.step(tol=1e-13, maxit=4000, restart=40)
        for s, p in enumerate(inj):
            if p is not None and p["cell"].size:
                t = {kk: torch.from_numpy(np.ascontiguousarray(v)).cuda() for kk, v in p.items()}
                sim.inject(s, t["cell"], t["off"], t["v"], t["w"])
        assert H.relerr(sim.gather("E").cpu().numpy(), r["E"]) < tol
        assert H.relerr(sim.gather("B").cpu().numpy(), r["B"]) < tol
        mv = sim.moves()
        assert all(g >= 0 for g in mv["gone"])
        gone += sum(mv["gone"])
        can = _canonical(G, wl, r["species"])
        for s in range(wl.nsp):
            got = {kk: v.cpu().numpy() for kk, v in sim.particles(s).items()}
            cell, x, v, w = can[s]
            assert got["cell"].size == cell.size, (k, s)
            assert np.array_equal(got["cell"], cell)
            xg = O.global_positions(G, got["cell"], got["off"].astype(np.float64))
            assert np.abs((xg - x)[:, :dim] / np.array(wl.dx[:dim])).max() < ptol
            assert np.abs(got["v"].T.astype(np.float64) - v).max() / np.abs(v).max() < (1e-5 if fp32 else 1e-12)
            assert np.abs(got["w"].astype(np.float64) - w).max() <= 1e-7 * np.abs(w).max()
            assert np.all(xg[:, 0] >= 0) and np.all(xg[:, 0] < wl.n[0] * wl.dx[0])
        # the next step starts from the library's order (cell order)
        E, B = r["E"], r["B"]
        sp = [O.Species(q.q, q.m, x, v, w) for q, (_, x, v, w) in zip(r["species"], can)]
        # the wall field condition on the GPU
        i = np.arange(wl.ncells) % wl.nstore[0]
        Eg = sim.gather("E").cpu().numpy()
        assert np.abs(Eg[1:, i == 0]).max() == 0.0
    # the fast particles next to x = L leave through an inflow plane, and are
    # reflected by a wall there
    if bc[1] == 2:
        assert gone > 0
    else:
        assert gone == 0
    d = sim.diagnostics()
    dep = O.deposit(G, sp, wl.dt, B, True, wl.n_smooth_u)
    ref = O.diagnostics(G, sp, E, B)
    assert abs(d["W_E"] - ref["W_E"]) <= tol * ref["W_E"]
    assert abs(d["W_B"] - ref["W_B"]) <= tol * ref["W_B"]
    sim.close()


def test_losses_and_injection_are_counted():
    print("[gpu] walled: loss and injection counts", flush=True)
    wl = _wl(3, (6, 4, 3), 20, False, (1, 2))
    parts = _parts(wl, False)
    E, B = _fields(wl)
    sim = H.make_sim(wl, parts, E, B)
    n0 = [sim.count(s) for s in range(wl.nsp)]
    sim.step(tol=1e-10, maxit=2000, restart=30)
    mv = sim.moves()
    assert all(g > 0 for g in mv["gone"]), mv
    n1 = [sim.count(s) for s in range(wl.nsp)]
    assert [a - b for a, b in zip(n0, n1)] == mv["gone"]
    # injection without a push in between: merged at the next settle
    p = synth.inflow(wl, 0, 0)
    t = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in p.items()}
    sim.inject(0, t["cell"], t["off"], t["v"], t["w"])
    got = sim.particles(0)
    assert got["cell"].numel() == n1[0] + p["cell"].size
    assert bool((got["cell"][1:] >= got["cell"][:-1]).all())
    assert sim.moves()["injected"][0] == p["cell"].size
    # a ghost cell is refused
    from paper_2506_11320_amd import GlecsimError
    bad = t["cell"].clone()
    bad[0] = wl.n[0]  # x index n = the ghost column
    sim.inject(0, bad, t["off"], t["v"], t["w"])
    with pytest.raises(GlecsimError):
        sim.sync()
    sim.close()


def test_far_moves_next_to_walls():
    """Moves of up to 2.5 cells per step on a walled grid: reflection on the
    wall, losses through the inflow plane and the stable re-sort of the far
    movers together, against the oracle's mover (FP64, bit-exact order)."""
    print("[gpu] walled: far movers", flush=True)
    wl = _wl(3, (8, 6, 5), 20, False, (1, 2))
    parts = _parts(wl, False)
    rng = np.random.default_rng(23)
    cells_per_v = wl.dt / np.array(wl.dx[:3])
    for p in parts:
        n = p["w"].size
        pick = rng.random(n) < 0.3
        d = rng.standard_normal((3, n))
        d /= np.linalg.norm(d, axis=0)
        v = d * rng.uniform(0.5, 2.5, n) / cells_per_v[:, None]
        p["v"][:, pick] = v[:, pick]
        p["w"] = (np.arange(n) + 1).astype(p["w"].dtype)  # the index rides in the weight
    E, B = _fields(wl)
    Eth = E + 0.01 * rng.standard_normal(E.shape)
    G, sp = H.oracle_species(wl, parts)
    sim = H.make_sim(wl, parts, E, B)
    sim.deposit()
    sim.set("Eth", torch.from_numpy(Eth))
    sim.push()
    sim.sync()
    mv = sim.moves()
    assert max(mv["far_moves"]) > 0 and max(mv["max_move"]) > 1.5, mv
    Bn = O.node_avg(G, B)
    for s in range(wl.nsp):
        xo, vo, keep = O.push_species(G, O.beta_s(wl.q[s], wl.m[s], wl.dt), wl.dt, sp[s].x, sp[s].v, Eth, Bn,
                                      with_keep=True)
        assert mv["gone"][s] == int((~keep).sum())
        kept = np.nonzero(keep)[0]
        cell_o = np.zeros(kept.size, np.int64)
        mul = 1
        for d in range(3):
            cell_o += np.floor(xo[kept, d] / wl.dx[d]).astype(np.int64) % G.n[d] * mul
            mul *= G.n[d]
        order = kept[O.stable_cell_order(cell_o)]
        got = {k: v.cpu().numpy() for k, v in sim.particles(s).items()}
        ids = np.rint(got["w"]).astype(np.int64) - 1
        assert np.array_equal(ids, order)
        xg = O.global_positions(G, got["cell"], got["off"].astype(np.float64))
        assert np.abs((xg - xo[ids]) / np.array(wl.dx)).max() < 1e-12
        assert np.abs(got["v"].T - vo[ids]).max() / np.abs(vo).max() < 1e-12
        assert np.all(xg[:, 0] >= 0) and np.all(xg[:, 0] < wl.n[0] * wl.dx[0])
    sim.close()


def test_walled_checkpoint_resumes_bitwise(tmp_path):
    """A walled run with injection, checkpointed after two steps and resumed
    in a fresh context, continues bit for bit like the uninterrupted run."""
    print("[gpu] walled: checkpoint and resume", flush=True)
    wl = _wl(3, (6, 4, 3), 20, True, (1, 2))
    parts = _parts(wl, True)
    E, B = _fields(wl)

    def inject(sim, k):
        for s in range(wl.nsp):
            p = synth.inflow(wl, s, k, f32=True)
            if p["cell"].size:
                t = {kk: torch.from_numpy(np.ascontiguousarray(v)).cuda() for kk, v in p.items()}
                sim.inject(s, t["cell"], t["off"], t["v"], t["w"])

    a = H.make_sim(wl, parts, E, B)
    for k in range(2):
        a.step(tol=1e-10, maxit=2000, restart=40)
        inject(a, k)
    path = str(tmp_path / "walled.ckpt")
    a.checkpoint(path)
    b = H.make_bare_sim(wl)
    b.restore(path)
    for k in range(2, 4):
        for sim in (a, b):
            sim.step(tol=1e-10, maxit=2000, restart=40)
            inject(sim, k)
    for key in ("E", "B"):
        assert torch.equal(a.gather(key), b.gather(key)), key
    for s in range(wl.nsp):
        pa, pb = a.particles(s), b.particles(s)
        for key in pa:
            assert torch.equal(pa[key], pb[key]), (s, key)
    a.close()
    b.close()
