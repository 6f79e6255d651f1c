"""Pins of the oracle's current smoothing (Sec. 3.2) and divergence cleaning
(Sec. 2.3): closed forms of single Fourier modes, brute-force loops on tiny
meshes, adjointness, conservation and the exact decay of the damping."""
import math

import numpy as np
import pytest

import oracle as O


def _grid(dim, n, dx=(0.5, 0.25, 0.4)):
    return O.grid(dim, n, dx)


@pytest.mark.parametrize("dim,n", [(1, (11, 1, 1)), (2, (6, 5, 1)), (3, (4, 5, 6))])
def test_smoothing_keeps_constants_and_sums(dim, n):
    G = _grid(dim, n)
    N = O.nnodes(G)
    rng = np.random.default_rng(dim)
    J = rng.standard_normal((3, N))
    S = O.smooth_current(G, J, 3)
    assert np.allclose(S.sum(axis=1), J.sum(axis=1), rtol=0, atol=1e-12)
    c = np.ones((3, N)) * np.array([[1.5], [-2.0], [0.25]])
    assert np.array_equal(O.smooth_current(G, c, 2), c)
    assert np.array_equal(O.smooth_current(G, J, 0), J)


def test_smoothing_fourier_factor_and_nyquist():
    # one pass of the stride-1 filter multiplies a mode along x by
    # phi + (1 - phi) cos(k dx) (the paper's filter with phi = 0.5, d = 1)
    nx = 16
    G = _grid(1, (nx, 1, 1))
    i = np.arange(nx)
    for m in (1, 3, 5):
        k = 2 * math.pi * m / nx
        J = np.stack([np.cos(k * i), np.sin(k * i), np.cos(k * i + 0.3)])
        S = O.smooth_current(G, J, 1)
        assert np.max(np.abs(S - (0.5 + 0.5 * math.cos(k)) * J)) < 1e-14
    nyq = np.stack([(-1.0) ** i] * 3)
    assert np.max(np.abs(O.smooth_current(G, nyq, 1))) == 0.0
    # three passes: the factor cubed
    k = 2 * math.pi * 3 / nx
    J = np.stack([np.cos(k * i)] * 3)
    assert np.max(np.abs(O.smooth_current(G, J, 3) - (0.5 + 0.5 * math.cos(k)) ** 3 * J)) < 1e-14


def _div_loops(G, B):
    nx, ny, nz = G.n[0], G.n[1], G.n[2]
    out = np.zeros(nx * ny * nz)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                c = i + nx * (j + ny * k)
                s = 0.0
                idx = [(i, j, k)]
                for d in range(G.dim):
                    p = [i, j, k]; m = [i, j, k]
                    p[d] = (p[d] + 1) % G.n[d]; m[d] = (m[d] - 1) % G.n[d]
                    cp = p[0] + nx * (p[1] + ny * p[2]); cm = m[0] + nx * (m[1] + ny * m[2])
                    s += (B[d, cp] - B[d, cm]) / (2 * G.dx[d])
                out[c] = s
    return out


@pytest.mark.parametrize("dim,n", [(1, (7, 1, 1)), (2, (5, 4, 1)), (3, (3, 4, 5))])
def test_div_matches_loops_and_grad_is_its_negative_adjoint(dim, n):
    G = _grid(dim, n)
    N = O.nnodes(G)
    rng = np.random.default_rng(10 + dim)
    B = rng.standard_normal((3, N))
    psi = rng.standard_normal(N)
    assert np.max(np.abs(O.div_cc(G, B) - _div_loops(G, B))) < 1e-12
    lhs = float(np.dot(psi, O.div_cc(G, B)))
    rhs = -float(np.sum(O.grad_cc(G, psi) * B))
    assert abs(lhs - rhs) < 1e-11 * (abs(lhs) + 1)
    # inactive axes carry no gradient
    g = O.grad_cc(G, psi)
    assert np.all(g[dim:] == 0)


def test_div_and_grad_of_a_mode_closed_form():
    nx, ny, nz = 12, 8, 6
    G = _grid(3, (nx, ny, nz))
    N = nx * ny * nz
    i = np.arange(N) % nx
    j = (np.arange(N) // nx) % ny
    kx, ky = 2 * math.pi * 2 / nx, 2 * math.pi / ny
    B = np.zeros((3, N))
    B[0] = np.sin(kx * i)
    B[1] = np.cos(ky * j)
    want = np.cos(kx * i) * math.sin(kx) / G.dx[0] - np.sin(ky * j) * math.sin(ky) / G.dx[1]
    assert np.max(np.abs(O.div_cc(G, B) - want)) < 1e-12
    g = O.grad_cc(G, np.sin(kx * i))
    assert np.max(np.abs(g[0] - np.cos(kx * i) * math.sin(kx) / G.dx[0])) < 1e-12
    assert np.max(np.abs(g[1:])) == 0.0


def test_cleaning_scalar_decays_exactly_when_b_is_solenoidal():
    G = _grid(3, (5, 4, 6))
    N = O.nnodes(G)
    rng = np.random.default_rng(3)
    psi = rng.standard_normal(N)
    B = np.ones((3, N)) * np.array([[0.3], [-1.0], [2.0]])  # uniform: no divergence
    out = O.dedner_psi(G, 0.2, psi, B, ch=1.7, damp=0.1)
    assert np.max(np.abs(out - psi * math.exp(-0.1))) < 1e-15
    # a single divergent mode from rest: psi = -dt ch^2 div B e^{-damp}
    nx = 5
    i = np.arange(N) % nx
    k = 2 * math.pi / nx
    Bm = np.zeros((3, N))
    Bm[0] = np.sin(k * i)
    dt, ch = 0.2, 1.7
    out = O.dedner_psi(G, dt, np.zeros(N), Bm, ch=ch, damp=0.1)
    want = -dt * ch * ch * np.cos(k * i) * math.sin(k) / G.dx[0] * math.exp(-0.1)
    assert np.max(np.abs(out - want)) < 1e-12
    assert O.cleaning_speed(G, 0.2, 0.8) == pytest.approx(0.8 * 0.25 / 0.2)


def test_cleaning_iteration_removes_divergence():
    # psi and B advanced by the cleaning terms alone (no curl E): the
    # divergence of a random field falls steadily at c_h = 0.8 dx/dt
    G = O.grid(3, (8, 8, 8), (1.0, 1.0, 1.0))
    N = O.nnodes(G)
    rng = np.random.default_rng(5)
    B = rng.standard_normal((3, N))
    dt = 0.1
    ch = O.cleaning_speed(G, dt, 0.8)
    psi = np.zeros(N)
    d0 = np.linalg.norm(O.div_cc(G, B))
    for _ in range(60):
        psi = O.dedner_psi(G, dt, psi, B, ch, 0.1)
        B = B - dt * O.grad_cc(G, psi)
    assert np.linalg.norm(O.div_cc(G, B)) < 0.05 * d0
