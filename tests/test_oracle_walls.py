"""Pins of the oracle's walled x axis (a conducting, reflecting wall at x = 0,
a wall or an inflow plane at x = L), none of which compares the oracle with
itself:
  * a walled vacuum field step equals the periodic step (pinned elsewhere) on
    the mirror-doubled domain, restricted to the walled half: the wall is the
    mirror plane (tangential E and normal B odd, normal E and tangential B
    even);
  * the vacuum field energy with half weights on the wall planes is
    conserved at theta = 1/2 (the energy theorem of the doubled domain);
  * specular reflection in closed form, |v| conserved, and removal through
    the inflow plane;
  * the wall field condition (tangential E = 0 on the wall, E held on the
    inflow plane, the ghost cell keeps the upstream B) after a plasma step."""
import math

import numpy as np
import pytest

import oracle as O
import synth

RNG = np.random.default_rng(41)


def _idx(n):
    N = int(np.prod(n))
    return np.stack(np.unravel_index(np.arange(N), tuple(n)[::-1])[::-1])


def _walled_fields(G, dim, rng):
    """Random E (nodes) and B (cells) on a walled grid with E_t = 0 on both
    wall planes (the ghost cell column holds zeros)."""
    N = O.nnodes(G)
    n = [G.n[d] for d in range(3)]
    i = _idx(n)[0]
    E = rng.standard_normal((3, N))
    E[1:, (i == 0) | (i == n[0] - 1)] = 0.0
    B = rng.standard_normal((3, N))
    B[:, i == n[0] - 1] = 0.0
    return E, B


def _double(G, Gd, E, B):
    """Mirror-doubled periodic fields: nodes 0..nx copied, nodes nx+1..2nx-1
    mirrored about node nx; cells 0..nx-1 copied, cells nx..2nx-1 mirrored."""
    nx = G.n[0] - 1
    nw = [G.n[d] for d in range(3)]
    nd = [Gd.n[d] for d in range(3)]
    Nd = O.nnodes(Gd)
    Ed, Bd = np.zeros((3, Nd)), np.zeros((3, Nd))
    id_ = _idx(nd)
    for g in range(Nd):
        i, j, k = id_[:, g]
        if i <= nx:
            gw = i + nw[0] * (j + nw[1] * k)
            Ed[:, g] = E[:, gw]
        else:
            gw = (2 * nx - i) + nw[0] * (j + nw[1] * k)
            Ed[:, g] = E[:, gw] * np.array([1, -1, -1])
        if i < nx:
            gw = i + nw[0] * (j + nw[1] * k)
            Bd[:, g] = B[:, gw]
        else:
            gw = (2 * nx - 1 - i) + nw[0] * (j + nw[1] * k)
            Bd[:, g] = B[:, gw] * np.array([-1, 1, 1])
    return Ed, Bd


def _vacuum_step(G, P, E, B):
    b = O.rhs(G, P, E, B, np.zeros_like(E))
    Eth = O.dense_solve(O.dense_A(G, P, None, None), b.ravel()).reshape(E.shape)
    return O.update_E(P.theta, E, Eth), O.update_B(G, P, B, Eth, None)


@pytest.mark.parametrize("dim,n", [(1, (6, 1, 1)), (2, (5, 3, 1)), (3, (4, 3, 3))])
@pytest.mark.parametrize("theta", [0.5, 0.6])
def test_walled_vacuum_step_is_the_mirrored_periodic_step(dim, n, theta):
    dx = (0.5, 0.4, 0.3)
    G = O.grid(dim, n, dx, bc=(O.BC_WALL, O.BC_WALL))
    Gd = O.grid(dim, (2 * n[0],) + tuple(n[1:]), dx)
    E, B = _walled_fields(G, dim, RNG)
    Ed, Bd = _double(G, Gd, E, B)
    P = O.params(theta, 0.45)
    nx = n[0]
    i = _idx([G.n[d] for d in range(3)])[0]
    idd = _idx([Gd.n[d] for d in range(3)])[0]
    for _ in range(3):
        E, B = _vacuum_step(G, P, E, B)
        Ed, Bd = _vacuum_step(Gd, P, Ed, Bd)
        np.testing.assert_allclose(E, Ed[:, idd <= nx], rtol=0, atol=1e-12 * np.abs(Ed).max())
        np.testing.assert_allclose(B[:, i < nx], Bd[:, idd < nx], rtol=0, atol=1e-12 * np.abs(Bd).max())
    # the doubled solution keeps the mirror symmetry (tangential E = 0 on the planes)
    assert np.abs(Ed[1:, (idd == 0) | (idd == nx)]).max() < 1e-12 * np.abs(Ed).max()


def test_walled_vacuum_energy_is_conserved():
    G = O.grid(3, (5, 4, 3), (0.5, 0.4, 0.3), bc=(O.BC_WALL, O.BC_WALL))
    E, B = _walled_fields(G, 3, RNG)
    P = O.params(0.5, 0.3)
    W0 = O.diagnostics(G, [], E, B)
    W0 = W0["W_E"] + W0["W_B"]
    for _ in range(5):
        E, B = _vacuum_step(G, P, E, B)
        W = O.diagnostics(G, [], E, B)
        assert abs(W["W_E"] + W["W_B"] - W0) < 1e-12 * W0
    # a full weight on the wall planes would not be conserved
    wfull = lambda E: (E ** 2).sum() * O.cellvol(G) / (8 * math.pi)
    E0, B0 = _walled_fields(G, 3, np.random.default_rng(5))
    E1, B1 = _vacuum_step(G, P, E0, B0)
    Wb = lambda B: (B[:, O.physical_cells(G)] ** 2).sum() * O.cellvol(G) / (8 * math.pi)
    assert abs(wfull(E1) + Wb(B1) - wfull(E0) - Wb(B0)) > 1e-6 * (wfull(E0) + Wb(B0))


@pytest.mark.parametrize("hi", [O.BC_WALL, O.BC_INFLOW])
def test_specular_reflection_and_inflow_removal(hi):
    """E = B = 0: the mover is free flight; a particle crossing x = 0 comes
    back mirrored with v_x reversed (|v| kept); at x = L it is mirrored by a
    wall or removed by an inflow plane."""
    nx, dx, dt = 6, 0.5, 0.5
    G = O.grid(3, (nx, 3, 3), (dx, 0.5, 0.5), bc=(O.BC_WALL, hi))
    N = O.nnodes(G)
    Z = np.zeros((3, N))
    L = nx * dx
    x = np.array([[0.10, 0.3, 0.7], [L - 0.05, 1.0, 0.2], [1.3, 0.4, 0.4], [0.02, 0.1, 0.1]])
    v = np.array([[-0.6, 0.2, 0.1], [0.4, -0.3, 0.05], [0.1, 0.1, 0.1], [-0.01, 0.0, 0.0]])
    xn, vn, keep = O.push_species(G, -0.25, dt, x, v, Z, Z, with_keep=True)
    np.testing.assert_allclose(np.linalg.norm(vn, axis=1), np.linalg.norm(v, axis=1), rtol=1e-15)
    # particle 0: 0.10 - 0.30 = -0.20 -> 0.20, v_x reversed
    assert xn[0, 0] == pytest.approx(0.20, abs=1e-15) and vn[0, 0] == pytest.approx(0.6)
    np.testing.assert_allclose(vn[0, 1:], v[0, 1:])
    # particle 2 flies freely; particle 3 stays inside
    np.testing.assert_allclose(xn[2], x[2] + dt * v[2], atol=1e-15)
    assert xn[3, 0] == pytest.approx(0.02 - 0.005) and keep[3]
    # particle 1 crosses x = L
    if hi == O.BC_WALL:
        assert keep.all()
        assert xn[1, 0] == pytest.approx(2 * L - (L - 0.05 + 0.2)) and vn[1, 0] == pytest.approx(-0.4)
    else:
        assert not keep[1] and keep[[0, 2, 3]].all()


def test_wall_field_condition_after_a_plasma_step():
    """A walled plasma (wall at x = 0, inflow at x = L), comoving current and
    limited LF on: after a step the tangential E on the wall plane is zero,
    E on the inflow plane and the ghost cell's B are the upstream values, and
    particles that crossed the inflow plane are gone."""
    nx, ny, nz = 6, 4, 3
    wl = synth.small("walls", dim=3, n=(nx, ny, nz), ppc=12, base="c5", fp32=False)
    G = O.grid(3, (nx, ny, nz), wl.dx, bc=(O.BC_WALL, O.BC_INFLOW))
    N = O.nnodes(G)
    i = _idx([G.n[d] for d in range(3)])[0]
    rng = np.random.default_rng(3)
    sp = []
    for s in range(2):
        n = nx * ny * nz * wl.ppc
        x = rng.random((n, 3)) * np.array([nx * wl.dx[0], ny * wl.dx[1], nz * wl.dx[2]])
        v = rng.normal(0, wl.vth[s], (n, 3)) + np.array([-0.15, 0.0, 0.0])
        v[:, 0] += np.where(x[:, 0] > (nx - 1) * wl.dx[0], 0.6, 0.0)  # some leave through x = L
        sp.append(O.Species(wl.q[s], wl.m[s], x, v, np.full(n, 0.01)))
    Eup = np.array([0.0, 0.0, 0.02])
    Bup = np.array([0.13, 0.075, 0.0])
    E = np.tile(Eup[:, None], (1, N))
    E[1:, i == 0] = 0.0
    B = np.tile(Bup[:, None], (1, N)) + 0.01 * rng.standard_normal((3, N))
    B[:, i == nx] = Bup[:, None]
    r = O.step(G, sp, E, B, dt=wl.dt, theta=0.5, comoving=True, lf_E=True, lf_B=True, beta_lim=1.5, a_mode=1,
               solve="dense")
    assert np.abs(r["E"][1:, i == 0]).max() < 1e-13
    assert np.abs(r["Eth"][1:, i == 0]).max() < 1e-13
    np.testing.assert_allclose(r["E"][:, i == nx], E[:, i == nx], atol=1e-13)
    np.testing.assert_array_equal(r["B"][:, i == nx], B[:, i == nx])
    for s in range(2):
        assert 0 < (~r["kept"][s]).sum() < sp[s].w.size
        assert np.all(r["species"][s].x[:, 0] >= 0) and np.all(r["species"][s].x[:, 0] < nx * wl.dx[0])
