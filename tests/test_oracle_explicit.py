"""Pins of the oracle's explicit-PIC current (Sec. 3.1, explicit form):
brute force on a tiny 1D mesh written here from the definitions (linear
weights, mass-weighted bulk velocity, the filter of Sec. 2.4), the cold
uniform flow, and invariance of the comoving current under a uniform boost."""
import numpy as np
import pytest

import oracle as O


def _species(G, rng, n, q, m, vshift=(0.0, 0.0, 0.0), vth=0.1):
    lo = np.zeros(3)
    hi = np.array([G.n[d] * G.dx[d] if d < G.dim else 0.0 for d in range(3)])
    x = lo + rng.random((n, 3)) * hi
    v = vth * rng.standard_normal((n, 3)) + np.asarray(vshift)
    w = 0.5 + rng.random(n)
    return O.Species(q, m, x, v, w)


def _brute_1d(nx, dx, species, comoving, n_smooth_u):
    """Nodes at i dx, periodic, linear weights; u = sum m w v W / sum m w W
    filtered n_smooth_u times (phi = 0.5, strides 1, 2, ...); then
    J_i = (1/dx) sum q w (v - u(x_p)) W_i(x_p)."""
    def weights(x):
        s = x / dx
        i0 = int(np.floor(s)) % nx
        f = s - np.floor(s)
        return [(i0, 1.0 - f), ((i0 + 1) % nx, f)]

    mm = np.zeros((3, nx)); mass = np.zeros(nx)
    for sp in species:
        for p in range(len(sp.w)):
            for i, W in weights(sp.x[p, 0]):
                mm[:, i] += sp.m * sp.w[p] * sp.v[p] * W
                mass[i] += sp.m * sp.w[p] * W
    u = np.where(mass > 0, mm / np.where(mass > 0, mass, 1.0), 0.0)
    for k in range(n_smooth_u):
        d = 1 if k % 2 == 0 else 2
        u = 0.5 * u + 0.25 * (np.roll(u, d, axis=1) + np.roll(u, -d, axis=1))
    J = np.zeros((3, nx))
    for sp in species:
        for p in range(len(sp.w)):
            ws = weights(sp.x[p, 0])
            up = sum(W * u[:, i] for i, W in ws) if comoving else 0.0
            for i, W in ws:
                J[:, i] += sp.q * sp.w[p] * (sp.v[p] - up) * W / dx
    return J


@pytest.mark.parametrize("comoving", [True, False])
@pytest.mark.parametrize("n_smooth_u", [0, 1, 5])
def test_explicit_current_matches_brute_force_1d(comoving, n_smooth_u):
    nx, dx = 9, 0.7
    G = O.grid(1, (nx, 1, 1), (dx, 1, 1))
    rng = np.random.default_rng(5 + n_smooth_u)
    sp = [_species(G, rng, 40, -1.0, 1.0, (0.3, 0.0, -0.1)), _species(G, rng, 30, 1.0, 25.0, (0.2, 0.1, 0.0))]
    J = O.explicit_current(G, sp, comoving, n_smooth_u=n_smooth_u)
    ref = _brute_1d(nx, dx, sp, comoving, n_smooth_u)
    assert np.max(np.abs(J - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("dim,n", [(1, (12, 1, 1)), (2, (5, 4, 1)), (3, (4, 3, 3))])
def test_cold_uniform_flow_has_no_comoving_current(dim, n):
    # every particle moves with V, so u = V at every node and v - u(x_p) = 0
    G = O.grid(dim, n, (0.5, 0.5, 0.5))
    rng = np.random.default_rng(dim)
    V = np.array([0.3, -0.2, 0.1])
    sp = [_species(G, rng, 300, -1.0, 1.0, V, vth=0.0), _species(G, rng, 300, 1.0, 100.0, V, vth=0.0)]
    Jc = O.explicit_current(G, sp, True)
    Jl = O.explicit_current(G, sp, False)
    assert np.max(np.abs(Jc)) < 1e-12 * np.max(np.abs(Jl))
    assert np.max(np.abs(Jl)) > 0.1


@pytest.mark.parametrize("dim,n", [(1, (10, 1, 1)), (2, (5, 4, 1)), (3, (4, 3, 3))])
def test_comoving_current_is_invariant_under_a_uniform_boost(dim, n):
    # v -> v + V shifts u by V at every node (all nodes carry mass), so
    # v - u(x_p) is unchanged; the lab current changes by rho V
    G = O.grid(dim, n, (0.5, 0.5, 0.5))
    rng = np.random.default_rng(10 + dim)
    sp = [_species(G, rng, 400, -1.0, 1.0), _species(G, rng, 300, 1.0, 25.0)]
    V = np.array([0.4, 0.0, -0.3])
    boosted = [O.Species(s.q, s.m, s.x, s.v + V, s.w) for s in sp]
    for ns_j in (0, 1):
        a = O.explicit_current(G, sp, True, n_smooth_j=ns_j)
        b = O.explicit_current(G, boosted, True, n_smooth_j=ns_j)
        assert np.max(np.abs(a - b)) < 1e-12 * max(1.0, np.max(np.abs(a)))
    la = O.explicit_current(G, sp, False)
    lb = O.explicit_current(G, boosted, False)
    rhoV = O.explicit_current(G, [O.Species(s.q, s.m, s.x, np.tile(V, (len(s.w), 1)), s.w) for s in sp], False)
    assert np.max(np.abs((lb - la) - rhoV)) < 1e-12 * np.max(np.abs(rhoV))
    assert np.max(np.abs(rhoV)) > 1e-3


def _boris(v, E, B, beta):
    """Boris (1970): half electric kick, rotation by t = beta B with
    s = 2 t / (1 + t^2), half kick; beta = q dt / (2 m)."""
    vm = v + beta * E
    t = beta * B
    s = 2.0 * t / (1.0 + (t * t).sum(axis=1, keepdims=True))
    vp = vm + np.cross(vm + np.cross(vm, t), s)
    return vp + beta * E


def test_mover_with_En_is_the_boris_push():
    """The implicit-midpoint rotation of the mover (Sec. 3.1) with E^n is the
    Boris push: both formulations agree to rounding on random inputs."""
    G = O.grid(1, (4, 1, 1), (1.0, 1, 1))
    rng = np.random.default_rng(3)
    n = 50
    x = np.zeros((n, 3)); x[:, 0] = 1.5  # middle of a cell: the gathers are plain averages
    v = 0.3 * rng.standard_normal((n, 3))
    Ec = rng.standard_normal((3, 1)) * np.ones((3, 4))
    Bc = rng.standard_normal((3, 1)) * np.ones((3, 4))
    for beta in (0.05, 0.7, -1.3):
        _, vn = O.push_species(G, beta, 0.5, x, v, Ec, Bc)
        ref = _boris(v, np.tile(Ec[:, 0], (n, 1)), np.tile(Bc[:, 0], (n, 1)), beta)
        assert np.max(np.abs(vn - ref)) < 1e-13


def test_explicit_fields_follow_the_discrete_light_wave():
    """Vacuum (one weightless particle per cell): E_y = cos(k x_i), and B_z at
    cell centres half a step ahead, form the leapfrog's discrete eigenmode, with
    sin(w dt/2) = (c dt/dx) sin(k dx/2) (Yee 1966).  After M steps
    E_y = cos(k x_i - w M dt) to rounding."""
    n, dx, dt, M = 32, 0.1, 0.07, 40
    G = O.grid(1, (n, 1, 1), (dx, 1, 1))
    xn = np.arange(n) * dx
    xc = xn + 0.5 * dx
    k = 2 * np.pi * 3 / (n * dx)
    w = 2.0 / dt * np.arcsin(dt / dx * np.sin(k * dx / 2))
    E = np.zeros((3, n)); E[1] = np.cos(k * xn)
    Bh = np.cos(k * xc - 0.5 * w * dt)                       # B^{1/2}
    DE = (np.roll(E[1], -1) - E[1]) / dx                      # (E_{i+1} - E_i)/dx at cell i + 1/2
    B = np.zeros((3, n)); B[2] = Bh + 0.5 * dt * DE           # B^0 = B^{1/2} + (dt/2) dE/dx
    sp = [O.Species(-1.0, 1.0, np.stack([xc, np.zeros(n), np.zeros(n)], axis=1), np.zeros((n, 3)), np.zeros(n))]
    for _ in range(M):
        r = O.explicit_step(G, sp, E, B, dt=dt, comoving=False)
        sp, E, B = r["species"], r["E"], r["B"]
    assert np.max(np.abs(E[1] - np.cos(k * xn - w * M * dt))) < 1e-11
    assert np.max(np.abs(E[0])) == 0 and np.max(np.abs(E[2])) == 0


def explicit_fast_flow_drift(comoving, ns_j, steps, dt=0.5):
    """Largest |dP_x / P_x| of the total particle momentum over an explicit run
    of the Sec. 4.2 fast flow (dt = 0.5 keeps c dt below dx)."""
    import synth
    from tests import harness as H
    wl = synth.workloads()["ff1d"]
    parts = H.species_arrays(wl, False)
    E, B = synth.fields(wl)
    G, sp = H.oracle_species(wl, parts)
    P0 = sum(s.m * (s.w * s.v[:, 0]).sum() for s in sp)
    drift = 0.0
    for _ in range(steps):
        r = O.explicit_step(G, sp, E, B, dt=dt, comoving=comoving, n_smooth_u=wl.n_smooth_u, n_smooth_j=ns_j)
        sp, E, B = r["species"], r["E"], r["B"]
        drift = max(drift, abs(sum(s.m * (s.w * s.v[:, 0]).sum() for s in sp) - P0) / abs(P0))
    return drift


def test_comoving_current_stabilises_an_explicit_fast_flow():
    """Sec. 3.1 says the comoving current carries over to explicit PIC codes.
    In the explicit step the lab-frame current lets the uniform fast flow's
    momentum drift (and without smoothing the run goes unstable soon after 120
    steps); the comoving current keeps it more than ten times smaller, with or
    without one smoothing pass."""
    assert explicit_fast_flow_drift(True, 0, 120) < 0.1 * explicit_fast_flow_drift(False, 0, 120)
    assert explicit_fast_flow_drift(True, 1, 400) < 0.1 * explicit_fast_flow_drift(False, 1, 400)
