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
