"""Parity at the full size of the 3D reconnection workload (256x128x128 cells,
64 particles per cell per species, FP32 particle path), in the launch
configuration the benchmark times, and of the 3D shock (128x64x64 cells, 27
particles per cell; against a wall with an inflow plane, and its periodic
colliding-flow variant) for the grid quantities.

The FP64 oracle cannot run the whole grid in seconds, so it checks sampled
outputs it can compute on its own:
  * deposit and grid pass at sampled nodes: the oracle runs the same recipe on
    a 24^3-cell periodic patch centred on the node, built from the
    generator's counter-based particles of those cells and the same initial
    fields.  Every quantity at the centre node depends on cells within 9 of
    it (the 5 filter passes of u reach 7 nodes, the limiter 2 more), so the
    patch's own wrap-around never reaches it;
  * the field operator at the same nodes, on a synthetic field;
  * the implicit push of sampled particles, traced through the re-binning by
    an identifier carried in the weight (the push only copies w);
and checks properties that hold at any size on every output: the converged
solve's true residual, and the re-binned order (cells non-decreasing, stable
within a cell, a permutation of the input).  Tolerances as in the small FP32
parity cases: 1e-5 relative (currents relative to the sum of the species'
current magnitudes at the node, since they cancel), positions 2e-6 cells."""
import math

import numpy as np
import pytest

import oracle as O
import synth
from tests import harness as H

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

PATCH = 24
C = PATCH // 2
NODES = [(7, 32, 5), (200, 64, 100), (131, 97, 64)]  # in a current sheet, between sheets, elsewhere
NODES_C4 = [(64, 32, 32), (3, 60, 7), (100, 17, 50)]  # at the flows' meeting plane, near the wrap, elsewhere


def _workload(name="c5"):
    return synth.workloads()[name]


def _sim(wl, id_weights=False, keep=None):
    """The benchmark's context and particles; with id_weights, w carries the
    particle's index as the bit pattern of a normal float.  keep: {s: idx}
    particles whose initial state is returned."""
    from paper_2506_11320_amd import Simulation
    sim = Simulation(wl.dim, wl.n, wl.dx, theta=wl.theta, dt=wl.dt, lf_E=wl.lf_E, lf_B=wl.lf_B,
                     beta_lim=wl.beta_lim, a_mode=wl.a_mode, comoving=wl.comoving, n_smooth_u=wl.n_smooth_u,
                     fp32=wl.fp32, bc=wl.bc)
    kept = {}
    for s in range(wl.nsp):
        p = synth.particles(wl, s, f32=wl.fp32)
        if keep is not None:
            idx = keep[s]
            kept[s] = {"cell": p["cell"][idx].copy(), "off": p["off"][:, idx].copy(), "v": p["v"][:, idx].copy()}
        t = {k: torch.from_numpy(v).cuda() for k, v in p.items()}
        n = p["w"].size
        del p
        if id_weights:
            t["w"] = (torch.arange(n, dtype=torch.int32, device="cuda") + 0x00800000).view(torch.float32)
        sim.add_species(wl.q[s], wl.m[s], t["cell"], t["off"], t["v"], t["w"])
        del t
        torch.cuda.synchronize()
        print(f"  species {s} loaded", flush=True)
    return sim, kept


def _patch(wl, E, B, node):
    """Oracle state of the periodic PATCH^3 patch centred on node (the patch's
    node C sits on it)."""
    nx, ny, nz = wl.n
    o = [node[d] - C for d in range(3)]
    Gp = O.grid(3, (PATCH, PATCH, PATCH), wl.dx)
    a = np.arange(PATCH)
    fx, fy, fz = [(o[d] + a) % wl.n[d] for d in range(3)]
    full = (fx[None, None, :] + nx * (fy[None, :, None] + ny * fz[:, None, None])).ravel()  # patch index -> full
    Ep, Bp = E[:, full], B[:, full]
    sp = []
    for s in range(wl.nsp):
        cells, offs, vs, ws = [], [], [], []
        for kz in range(PATCH):
            for ky in range(PATCH):
                row = nx * (fy[ky] + ny * fz[kz])
                xs = fx
                # contiguous runs of the row in the full grid
                start = 0
                for i in range(1, PATCH + 1):
                    if i == PATCH or xs[i] != xs[i - 1] + 1:
                        p = synth.particles(wl, s, row + xs[start], row + xs[i - 1] + 1, f32=wl.fp32)
                        gx = p["cell"] - row
                        px = (gx - o[0]) % nx
                        cells.append(px + PATCH * (ky + PATCH * kz))
                        offs.append(p["off"])
                        vs.append(p["v"])
                        ws.append(p["w"])
                        start = i
        cell = np.concatenate(cells)
        off = np.concatenate(offs, axis=1).astype(np.float64)
        x = O.global_positions(Gp, cell, off)
        sp.append(O.Species(wl.q[s], wl.m[s], x, np.concatenate(vs, axis=1).astype(np.float64).T,
                            np.concatenate(ws).astype(np.float64)))
    ref = H.oracle_grid_pass(wl.replace(n=(PATCH, PATCH, PATCH)), Gp, sp, Ep, Bp)
    # species currents at the centre node, the scale of the (cancelling) total
    cidx = C + PATCH * (C + PATCH * C)
    ref["J_scale_node"] = sum(np.linalg.norm(j[:, cidx]) for j in ref["J_s"])
    ref["cidx"] = cidx
    ref["G"] = Gp
    ref["full"] = full
    return ref


def _rel(a, b, scale=None):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    s = np.linalg.norm(b) if scale is None else scale
    return np.linalg.norm(a - b) / s


def _probe_field(wl):
    """Synthetic smooth field at the nodes for the operator check."""
    nx, ny, nz = wl.n
    E, _ = synth.fields(wl)
    i = np.arange(nx)[None, None, :]
    j = np.arange(ny)[None, :, None]
    k = np.arange(nz)[:, None, None]
    ph = 2 * math.pi * (3 * i / nx + 2 * j / ny + k / nz)
    x = E.copy()
    x[0] += 0.01 * np.sin(ph).ravel()
    x[1] += 0.02 * np.cos(ph + 0.3).ravel()
    x[2] += 0.015 * np.sin(2 * ph + 1.0).ravel()
    return x


@pytest.mark.parametrize("name,nodes", [("c5", NODES), ("c4p", NODES_C4)])
def test_grid_quantities_operator_and_solve_at_full_size(name, nodes):
    wl = _workload(name)
    print(f"[gpu] full-size {name} deposit/operator/solve", flush=True)
    E, B = synth.fields(wl)
    sim, _ = _sim(wl)
    sim.set_fields(torch.from_numpy(E).cuda(), torch.from_numpy(B).cuda())
    sim.deposit()
    gidx = torch.tensor([n[0] + wl.n[0] * (n[1] + wl.n[1] * n[2]) for n in nodes], device="cuda")
    got = {}
    for k in ["J_lab", "J_eff", "rho", "mm", "mass", "u", "EM", "Mt", "M0", "kappa_E", "rhs"]:
        g = sim.gather(k)
        got[k] = g.index_select(g.dim() - 1, gidx).cpu().numpy()
        del g
    xprobe = _probe_field(wl)
    Ax = sim.apply_operator(torch.from_numpy(xprobe).cuda())
    got["Ax"] = Ax.index_select(1, gidx).cpu().numpy()
    del Ax
    torch.cuda.synchronize()
    for q, node in enumerate(nodes):
        print(f"  node {node}: oracle patch", flush=True)
        ref = _patch(wl, E, B, node)
        c = ref["cidx"]
        tol = 1e-5
        errs = {
            "J_lab": _rel(got["J_lab"][:, q], ref["J_lab"][:, c], ref["J_scale_node"]),
            "Mt": _rel(got["Mt"][:, :, q], H.half_from_full(ref["Mt"], 3)[:, :, c]),
            "M0": _rel(got["M0"][:, :, q], H.half_from_full(ref["M0"], 3)[:, :, c]),
            "mass": _rel(got["mass"][q], ref["mass"][c]),
            "mm": _rel(got["mm"][:, q], ref["mm"][:, c]),
            "u": _rel(got["u"][:, q], ref["u"][:, c]),
            # E_M = -u x B can cancel: scale by |u||B|
            "EM": _rel(got["EM"][:, q], ref["EM"][:, c], np.linalg.norm(ref["u"][:, c]) * np.linalg.norm(ref["Bn"][:, c])),
            "J_eff": _rel(got["J_eff"][:, q], ref["J_eff"][:, c], ref["J_scale_node"]),
            # kappa = (1 - phi) a / 2 vanishes where the limiter saturates: scale by a / 2 = |u| / 2
            "kappa_E": _rel(got["kappa_E"][:, :, q], ref["kE"][:, :, c], 0.5 * np.linalg.norm(ref["u"][:, c])),
            "rhs": _rel(got["rhs"][:, q], ref["rhs"][:, c]),
        }
        for s in range(wl.nsp):
            errs[f"rho{s}"] = _rel(got["rho"][s, q], ref["rho_s"][s][c])
        xp = xprobe[:, ref["full"]]
        Ax_ref = O.apply_A(ref["G"], ref["P"], ref["Mt"], ref["kE"], xp)
        errs["Ax"] = _rel(got["Ax"][:, q], Ax_ref[:, c])
        print("   " + ", ".join(f"{k} {v:.1e}" for k, v in errs.items()), flush=True)
        for k, v in errs.items():
            assert v < tol, (node, k, v)
    # the converged field meets the residual bound through the operator itself
    rep = sim.solve(tol=1e-8, maxit=500, restart=30)
    assert rep["converged"] and rep["relres"] <= 1e-8
    b = sim.gather("rhs")
    r = b - sim.apply_operator(sim.gather("Eth"))
    rel = (torch.linalg.vector_norm(r) / torch.linalg.vector_norm(b)).item()
    print(f"  solve: {rep['iterations']} iterations, true relres {rel:.2e}", flush=True)
    assert rel <= 1.01e-8
    sim.close()


def test_c5_push_and_rebinning_at_full_size():
    wl = _workload()
    print("[gpu] full-size C5 push/re-binning", flush=True)
    rng = np.random.default_rng(2024)
    npart = wl.ncells * wl.ppc
    keep = {s: np.sort(rng.choice(npart, size=3000, replace=False)) for s in range(wl.nsp)}
    E, B = synth.fields(wl)
    sim, kept = _sim(wl, id_weights=True, keep=keep)
    sim.set_fields(torch.from_numpy(E).cuda(), torch.from_numpy(B).cuda())
    sim.deposit()  # node-averaged B for the mover (the tagged weights make the moments meaningless)
    Eth = E + 0.02 * rng.standard_normal(E.shape)
    sim.set("Eth", torch.from_numpy(Eth))
    sim.push()
    sim.sync()
    G = O.grid(3, wl.n, wl.dx)
    Bn = O.node_avg(G, B)
    L = np.array([wl.n[d] * wl.dx[d] for d in range(3)])
    for s in range(wl.nsp):
        p = sim.particles(s)
        n = p["cell"].numel()
        assert n == npart
        ids = p["w"].view(torch.int32).long() - 0x00800000
        cell = p["cell"]
        # re-binned order: cells non-decreasing, stable within a cell, a permutation
        assert bool((cell[1:] >= cell[:-1]).all())
        same = cell[1:] == cell[:-1]
        assert bool(((ids[1:] > ids[:-1]) | ~same).all())
        assert int(ids.min()) == 0 and int(ids.max()) == n - 1
        inv = torch.full((n,), -1, dtype=torch.int64, device="cuda")
        inv[ids] = torch.arange(n, device="cuda")
        assert bool((inv >= 0).all())
        pos = inv[torch.from_numpy(keep[s]).cuda()]
        gc = cell[pos].cpu().numpy()
        goff = p["off"][:, pos].cpu().numpy().astype(np.float64)
        gv = p["v"][:, pos].cpu().numpy().astype(np.float64)
        del p, ids, cell, inv, same
        k0 = kept[s]
        x0 = O.global_positions(G, k0["cell"], k0["off"].astype(np.float64))
        xo, vo = O.push_species(G, O.beta_s(wl.q[s], wl.m[s], wl.dt), wl.dt, x0, k0["v"].astype(np.float64).T,
                                Eth, Bn)
        xg = O.global_positions(G, gc, goff)
        dxp = (xg - xo + 0.5 * L) % L - 0.5 * L
        ex = np.abs(dxp / np.array(wl.dx)).max()
        ev = np.abs(gv.T - vo).max() / np.abs(vo).max()
        print(f"  species {s}: position err {ex:.1e} cells, velocity err {ev:.1e}", flush=True)
        assert ex < 2e-6 and ev < 1e-5
    sim.close()


# walled shock: a node on the wall plane, one near the wall, one in the interior
NODES_C4W = [(0, 40, 9), (3, 5, 60), (64, 32, 32)]
PX = 24  # x extent of the walled patch (walls at both of its ends)


def _patch_walled(wl, E, B, node):
    """Oracle state of a patch of the walled grid around node: y and z as in
    _patch (periodic, PATCH wide, centred); along x either cells [0, PX) with
    walls at both ends (nodes within 12 of the wall: the patch's far wall is
    beyond the 9-node reach of every quantity at the node), or a periodic
    PATCH-wide window centred on the node (interior nodes, whose reach never
    meets a wall)."""
    nxs, ny, nz = wl.nstore
    near = node[0] <= 12
    a = np.arange(PATCH)
    fy, fz = [(node[d] - C + a) % wl.n[d] for d in (1, 2)]
    if near:
        xs = np.arange(PX + 1)  # storage x of the patch: nodes 0..PX, cells 0..PX-1, ghost PX
        Gp = O.grid(3, (PX, PATCH, PATCH), wl.dx, bc=(O.BC_WALL, O.BC_WALL))
        cidx = node[0] + (PX + 1) * (C + PATCH * C)
        pwl = wl.replace(n=(PX, PATCH, PATCH), bc=(O.BC_WALL, O.BC_WALL))
        cell_x = np.arange(PX)
    else:
        xs = (node[0] - C + a)
        Gp = O.grid(3, (PATCH, PATCH, PATCH), wl.dx)
        cidx = C + PATCH * (C + PATCH * C)
        pwl = wl.replace(n=(PATCH, PATCH, PATCH), bc=(0, 0))
        cell_x = xs
    nxp = xs.size
    full = (xs[None, None, :] + nxs * (fy[None, :, None] + ny * fz[:, None, None])).ravel()
    Ep, Bp = E[:, full], B[:, full]
    sp = []
    for s in range(wl.nsp):
        cells, offs, vs, ws = [], [], [], []
        for kz in range(PATCH):
            for ky in range(PATCH):
                row = nxs * (fy[ky] + ny * fz[kz])
                p = synth.particles(wl, s, row + int(cell_x[0]), row + int(cell_x[-1]) + 1, f32=wl.fp32)
                px = p["cell"] - row - int(cell_x[0])
                cells.append(px + nxp * (ky + PATCH * kz))
                offs.append(p["off"])
                vs.append(p["v"])
                ws.append(p["w"])
        cell = np.concatenate(cells)
        x = O.global_positions(Gp, cell, np.concatenate(offs, axis=1).astype(np.float64))
        sp.append(O.Species(wl.q[s], wl.m[s], x, np.concatenate(vs, axis=1).astype(np.float64).T,
                            np.concatenate(ws).astype(np.float64)))
    ref = H.oracle_grid_pass(pwl, Gp, sp, Ep, Bp)
    ref["J_scale_node"] = sum(np.linalg.norm(j[:, cidx]) for j in ref["J_s"])
    ref["cidx"], ref["G"], ref["full"] = cidx, Gp, full
    return ref


def test_walled_shock_grid_quantities_and_operator_at_full_size():
    wl = _workload("c4")
    assert wl.walled
    print("[gpu] full-size walled c4 deposit/operator/solve", flush=True)
    E, B = synth.fields(wl)
    sim, _ = _sim(wl)
    sim.set_fields(torch.from_numpy(E).cuda(), torch.from_numpy(B).cuda())
    sim.deposit()
    nxs, ny, nz = wl.nstore
    gidx = torch.tensor([n[0] + nxs * (n[1] + ny * n[2]) for n in NODES_C4W], device="cuda")
    got = {}
    for k in ["J_lab", "J_eff", "rho", "mm", "mass", "u", "EM", "Mt", "M0", "kappa_E", "rhs"]:
        g = sim.gather(k)
        got[k] = g.index_select(g.dim() - 1, gidx).cpu().numpy()
        del g
    # a smooth probe field on the storage grid for the operator
    i = np.arange(nxs)[None, None, :]
    j = np.arange(ny)[None, :, None]
    k = np.arange(nz)[:, None, None]
    ph = 2 * math.pi * (3 * i / nxs + 2 * j / ny + k / nz)
    xprobe = E.copy()
    xprobe[0] += 0.01 * np.sin(ph).ravel()
    xprobe[1] += 0.02 * np.cos(ph + 0.3).ravel()
    xprobe[2] += 0.015 * np.sin(2 * ph + 1.0).ravel()
    Ax = sim.apply_operator(torch.from_numpy(xprobe).cuda())
    got["Ax"] = Ax.index_select(1, gidx).cpu().numpy()
    del Ax
    torch.cuda.synchronize()
    for q, node in enumerate(NODES_C4W):
        print(f"  node {node}: oracle patch", flush=True)
        ref = _patch_walled(wl, E, B, node)
        c = ref["cidx"]
        un = np.linalg.norm(ref["u"][:, c])
        errs = {
            "J_lab": _rel(got["J_lab"][:, q], ref["J_lab"][:, c], ref["J_scale_node"]),
            "Mt": _rel(got["Mt"][:, :, q], H.half_from_full(ref["Mt"], 3)[:, :, c]),
            "M0": _rel(got["M0"][:, :, q], H.half_from_full(ref["M0"], 3)[:, :, c]),
            "mass": _rel(got["mass"][q], ref["mass"][c]),
            "mm": _rel(got["mm"][:, q], ref["mm"][:, c]),
            "u": _rel(got["u"][:, q], ref["u"][:, c]),
            "EM": _rel(got["EM"][:, q], ref["EM"][:, c], un * np.linalg.norm(ref["Bn"][:, c])),
            "J_eff": _rel(got["J_eff"][:, q], ref["J_eff"][:, c], ref["J_scale_node"]),
            "kappa_E": _rel(got["kappa_E"][:, :, q], ref["kE"][:, :, c], 0.5 * un),
            "rhs": _rel(got["rhs"][:, q], ref["rhs"][:, c]),
        }
        for s in range(wl.nsp):
            errs[f"rho{s}"] = _rel(got["rho"][s, q], ref["rho_s"][s][c])
        Ax_ref = O.apply_A(ref["G"], ref["P"], ref["Mt"], ref["kE"], xprobe[:, ref["full"]])
        errs["Ax"] = _rel(got["Ax"][:, q], Ax_ref[:, c])
        print("   " + ", ".join(f"{k} {v:.1e}" for k, v in errs.items()), flush=True)
        for k, v in errs.items():
            assert v < 1e-5, (node, k, v)
    rep = sim.solve(tol=1e-8, maxit=500, restart=30)
    assert rep["converged"] and rep["relres"] <= 1e-8
    b = sim.gather("rhs")
    r = b - sim.apply_operator(sim.gather("Eth"))
    rel = (torch.linalg.vector_norm(r) / torch.linalg.vector_norm(b)).item()
    print(f"  solve: {rep['iterations']} iterations, true relres {rel:.2e}", flush=True)
    assert rel <= 1.01e-8
    sim.close()
