"""Pins of the FP64 oracle to what the paper and the mathematics fix.

Each test checks the oracle against a closed form, an invariant, a special
case that reduces to a textbook result, or brute force on a tiny input, so
that a dropped term, a wrong sign, a wrong index or a transposed operand in
the oracle fails at least one of them.  None of these tests uses the GPU.
"""
import math

import numpy as np
import pytest

import oracle as O
import synth

RNG = np.random.default_rng(12345)


# ------------------------------------------------------------- limiter (Sec. 2.2)
def test_limiter_special_cases():
    # beta = 1 is minmod: phi = max(0, min(r, 1))
    for r in [-2.0, -0.1, 0.0, 0.3, 0.999, 1.0, 1.7, 5.0]:
        assert O.limiter(r, 1.0, 1.0) == pytest.approx(max(0.0, min(r, 1.0)), abs=1e-15)
    # beta = 2 is van Leer's MC limiter: max(0, min(2r, (1+r)/2, 2))
    for r, want in [(-1.0, 0.0), (0.2, 0.4), (0.5, 0.75), (1.0, 1.0), (3.0, 2.0), (10.0, 2.0)]:
        assert O.limiter(r, 1.0, 2.0) == pytest.approx(want, abs=1e-15)
    # "beta = 0" is the unlimited first-order scheme: phi == 0
    for r in [-3.0, 0.0, 0.5, 1.0, 4.0]:
        assert O.limiter(r, 1.0, 0.0) == 0.0
    # smooth (r = 1) gives the second-order scheme for every beta in [1, 2]
    for b in [1.0, 1.25, 1.5, 2.0]:
        assert O.limiter(1.0, 1.0, b) == 1.0
    # ratios with a vanishing denominator
    assert O.limiter(0.0, 0.0, 1.5) == 1.0
    assert O.limiter(2.0, 0.0, 1.5) == 1.5
    assert O.limiter(-2.0, 0.0, 1.5) == 0.0


def _tv(u):
    return np.abs(np.diff(np.concatenate([u, u[:1]]))).sum()


@pytest.mark.parametrize("beta", [0.0, 1.0, 1.5, 2.0])
@pytest.mark.parametrize("nu", [0.2, 0.4, 0.5])
@pytest.mark.parametrize("profile", ["step", "tophat"])
def test_llf_limited_scheme_is_tvd(beta, nu, profile):
    """Harten's lemma bound: TVD and no new extrema for nu <= 2/(2+beta)."""
    if nu > 2.0 / (2.0 + beta) + 1e-12:
        pytest.skip("outside the proven TVD range")
    n = 100
    x = np.arange(n)
    u0 = (x >= 50).astype(float) if profile == "step" else ((x >= 30) & (x < 60)).astype(float)
    u = u0.copy()
    tv = _tv(u)
    for _ in range(60):
        u = O.advect(u, nu, beta, 1)
        assert _tv(u) <= tv + 1e-13
        assert u.min() >= -1e-14 and u.max() <= 1.0 + 1e-14
        tv = _tv(u)


def test_ftcs_is_not_tvd_negative_control():
    n = 100
    u = ((np.arange(n) >= 30) & (np.arange(n) < 60)).astype(float)
    tv0 = _tv(u)
    u = O.advect(u, 0.4, 1.0, 10, phi_override=1.0)
    assert _tv(u) > tv0 + 1e-3


def test_lf_with_phi_zero_is_upwind_and_exact_at_cfl_one():
    """phi = 0, a = c: the LLF flux is the upwind flux; at nu = 1 it shifts
    the profile by exactly one cell per step."""
    u0 = RNG.random(40)
    u = O.advect(u0, 1.0, 0.0, 7)
    np.testing.assert_allclose(u, np.roll(u0, 7), atol=1e-15)
    u = O.advect(u0, 0.3, 0.0, 1)
    np.testing.assert_allclose(u, u0 - 0.3 * (u0 - np.roll(u0, 1)), atol=1e-15)


# ------------------------------------------------------------- alpha and mover (Sec. 3.1)
def test_alpha_is_inverse_of_implicit_rotation_and_comoving_identity():
    for _ in range(50):
        beta = RNG.normal() * 2
        B = RNG.normal(size=3)
        u = RNG.normal(size=3)
        al = O.alpha(beta, B)
        # (I - beta [. x B]) alpha = I
        cross = np.array([[0, B[2], -B[1]], [-B[2], 0, B[0]], [B[1], -B[0], 0]])  # w -> w x B
        np.testing.assert_allclose((np.eye(3) - beta * cross) @ al, np.eye(3), atol=1e-13)
        # the paper's identity alpha (u + beta E_M) = u with E_M = -u x B
        EM = -np.cross(u, B)
        np.testing.assert_allclose(al @ (u + beta * EM), u, atol=1e-13)


def _one_particle_grid():
    G = O.grid(3, (4, 4, 4), (0.5, 0.5, 0.5))
    return G, O.nnodes(G)


def test_mover_gyration_closed_form():
    """E = 0, uniform B: |v| is conserved and the velocity rotates by
    2 atan(|beta B|) per step (implicit midpoint = Cayley transform)."""
    G, N = _one_particle_grid()
    B0 = np.array([0.0, 0.0, 0.7])
    Bn = np.repeat(B0[:, None], N, axis=1)
    E = np.zeros((3, N))
    beta = O.beta_s(-1.0, 1.0, 0.5)
    x = np.array([[0.3, 0.7, 1.1]])
    v = np.array([[0.2, 0.0, 0.05]])
    xn, vn = O.push_species(G, beta, 0.5, x, v, E, Bn)
    assert np.linalg.norm(vn) == pytest.approx(np.linalg.norm(v), rel=1e-14)
    ang = math.atan2(vn[0, 1], vn[0, 0]) - math.atan2(v[0, 1], v[0, 0])
    ang = (ang + math.pi) % (2 * math.pi) - math.pi
    assert abs(ang) == pytest.approx(2 * math.atan(abs(beta) * 0.7), rel=1e-13)
    assert vn[0, 2] == pytest.approx(0.05, abs=1e-15)
    np.testing.assert_allclose(xn, (x + 0.5 * vn) % 2.0, atol=1e-15)


def test_mover_exb_fixed_point_and_free_acceleration():
    G, N = _one_particle_grid()
    B0 = np.array([0.1, -0.3, 0.5])
    E0 = np.cross(np.array([0.2, 0.4, 0.1]), B0)  # E perpendicular to B
    vexb = np.cross(E0, B0) / (B0 @ B0)
    Bn = np.repeat(B0[:, None], N, axis=1)
    En = np.repeat(E0[:, None], N, axis=1)
    beta = O.beta_s(1.0, 25.0, 0.5)
    x = np.array([[1.2, 0.1, 0.9]])
    _, vn = O.push_species(G, beta, 0.5, x, vexb[None, :], En, Bn)
    np.testing.assert_allclose(vn[0], vexb, atol=1e-15)
    # uniform E, no B: v^{n+1} = v^n + 2 beta E
    _, vn = O.push_species(G, beta, 0.5, x, np.array([[0.1, 0.2, 0.3]]), En, np.zeros((3, N)))
    np.testing.assert_allclose(vn[0], np.array([0.1, 0.2, 0.3]) + 2 * beta * E0, atol=1e-15)


# ------------------------------------------------------------- shape and deposit (Sec. 3.1)
@pytest.mark.parametrize("dim", [1, 2, 3])
def test_shape_partition_of_unity_and_brute_force_deposit(dim):
    n = (5, 4, 3)
    dx = (0.5, 0.7, 0.3)
    G = O.grid(dim, n, dx)
    N = O.nnodes(G)
    L = np.array([n[d] * dx[d] if d < dim else 1.0 for d in range(3)])
    npart = 9
    x = RNG.random((npart, 3)) * L
    x[:, dim:] = 0.0
    v = RNG.normal(size=(npart, 3)) * 0.1
    w = RNG.random(npart) + 0.5
    Bc = RNG.normal(size=(3, N)) * 0.3
    Bn = O.node_avg(G, Bc)
    q, m, dt = -1.0, 1.0, 0.5
    beta = O.beta_s(q, m, dt)
    a = O.deposit_species(G, q, m, beta, x, v, w, Bn)
    dV = O.cellvol(G)
    # brute force, one particle at a time, from the definitions
    J = np.zeros((3, N)); rho = np.zeros(N); M = np.zeros((27, 9, N))
    sum_qalpha_v = np.zeros(3)
    for p in range(npart):
        nodes, W = O.shape(G, x[p])
        assert W.sum() == pytest.approx(1.0, abs=1e-15)
        assert np.all(W >= 0)
        Bp = (Bn[:, nodes] * W).sum(axis=1)
        al = O.alpha(beta, Bp)
        qp = q * w[p]
        sum_qalpha_v += qp * al @ v[p]
        for ia, ga in enumerate(nodes):
            J[:, ga] += qp * (al @ v[p]) * W[ia] / dV
            rho[ga] += qp * W[ia] / dV
            ia_c = np.unravel_index(ia, (2, 2, 2)[:dim], order="F")
            for ib, gb in enumerate(nodes):
                ib_c = np.unravel_index(ib, (2, 2, 2)[:dim], order="F")
                o = [0, 0, 0]
                for d in range(dim):
                    o[d] = int(ib_c[d]) - int(ia_c[d])
                M[O.off27(o), :, ga] += qp * al.ravel() * W[ia] * W[ib]
    np.testing.assert_allclose(a["J"], J, atol=1e-14)
    np.testing.assert_allclose(a["rho"], rho, atol=1e-14)
    np.testing.assert_allclose(a["M"], M, atol=1e-14)
    # charge and current sums
    assert (a["rho"].sum() * dV) == pytest.approx(q * w.sum(), rel=1e-14)
    np.testing.assert_allclose(a["J"].sum(axis=1) * dV, sum_qalpha_v, rtol=1e-12, atol=1e-15)


def _shifted(G, g, o):
    ic = []
    rem = g
    for d in range(G.dim):
        ic.append(rem % G.n[d]); rem //= G.n[d]
    out = 0
    for d in reversed(range(G.dim)):
        out = out * G.n[d] + (ic[d] + o[d]) % G.n[d]
    return out


def test_mass_matrix_symmetry_and_total():
    wl = synth.small("pin", dim=3, n=(4, 3, 5), ppc=5)
    G = O.grid(3, wl.n, wl.dx)
    N = O.nnodes(G)
    p = synth.particles(wl, 0)
    x = O.global_positions(G, p["cell"], p["off"])
    v = p["v"].T
    Bc = RNG.normal(size=(3, N)) * 0.4
    Bn = O.node_avg(G, Bc)
    beta = O.beta_s(-1.0, 1.0, 0.5)
    a = O.deposit_species(G, -1.0, 1.0, beta, x, v, p["w"], Bn)
    M = a["M"]
    for o in O.half_offsets(3):
        neg = tuple(-c for c in o)
        for g in range(N):
            h = _shifted(G, g, o)
            np.testing.assert_allclose(M[O.off27(neg), :, h], M[O.off27(o), :, g], rtol=1e-13, atol=1e-18)
    # sum over all node pairs = sum_p q_p alpha_p
    tot = np.zeros(9)
    for i in range(p["w"].size):
        nodes, W = O.shape(G, x[i])
        Bp = (Bn[:, nodes] * W).sum(axis=1)
        tot += -1.0 * p["w"][i] * O.alpha(beta, Bp).ravel()
    np.testing.assert_allclose(M.sum(axis=(0, 2)), tot, rtol=1e-12)


def test_cold_uniform_flow_comoving_equals_lab():
    """Cold (v = u everywhere), paired e/i loading, uniform B: the net charge
    at every node is zero, so the comoving current equals the lab current
    (Sec. 3.1, the decomposition of J), and in general J_lab - J_eff = u rho."""
    wl = synth.workloads()["c2"].replace(n=(6, 5, 1), ppc=6, paired=True, vth=(0.0, 0.0))
    G = O.grid(2, wl.n, wl.dx)
    N = O.nnodes(G)
    E, Bc = synth.fields(wl)
    sp = []
    for s in range(2):
        p = synth.particles(wl, s)
        sp.append(O.Species(wl.q[s], wl.m[s], O.global_positions(G, p["cell"], p["off"]), p["v"].T, p["w"]))
    dep = O.deposit(G, sp, wl.dt, Bc, comoving=True)
    scale = np.abs(dep["J_lab"]).max() + sum(np.abs(O.deposit_species(G, s.q, s.m, O.beta_s(s.q, s.m, wl.dt),
                                                                      s.x, s.v, s.w, dep["Bn"])["J"]).max()
                                             for s in sp)
    np.testing.assert_allclose(dep["J_eff"], dep["J_lab"], atol=1e-14 * scale)
    rho = sum(dep["rho_s"])
    np.testing.assert_allclose(rho, 0.0, atol=1e-15)
    # unpaired: J_lab - J_eff = u rho_node with uniform u
    wl2 = wl.replace(paired=False)
    sp2 = []
    for s in range(2):
        p = synth.particles(wl2, s)
        sp2.append(O.Species(wl.q[s], wl.m[s], O.global_positions(G, p["cell"], p["off"]), p["v"].T, p["w"]))
    dep2 = O.deposit(G, sp2, wl.dt, Bc, comoving=True)
    rho2 = sum(dep2["rho_s"])
    u = np.array(wl.u0)[:, None]
    np.testing.assert_allclose(dep2["J_lab"] - dep2["J_eff"], u * rho2[None, :], atol=1e-13 * scale)


# ------------------------------------------------------------- grid operators (Sec. 2.1)
@pytest.mark.parametrize("dim", [1, 2, 3])
def test_curl_adjointness_and_div_curl(dim):
    G = O.grid(dim, (5, 4, 3), (0.4, 0.6, 0.9))
    N = O.nnodes(G)
    E = RNG.normal(size=(3, N)); B = RNG.normal(size=(3, N))
    lhs = (O.curl_nc(G, E) * B).sum()
    rhs = (E * O.curl_cn(G, B)).sum()
    assert lhs == pytest.approx(rhs, rel=1e-12, abs=1e-12)
    assert np.abs(O.div_nc(G, O.curl_cn(G, B))).max() < 1e-12


def test_1d_vacuum_operator_is_the_printed_tridiagonal_system():
    """In 1D vacuum the E_y system and B_z update reduce to the paper's
    eq. (e-1d) and eq. (1d-b)."""
    n, dx, dt, th, c = 12, 0.1, 0.07, 0.6, 1.3
    G = O.grid(1, (n, 1, 1), (dx, 1, 1))
    P = O.params(th, dt, c)
    E = RNG.normal(size=(3, n)); B = RNG.normal(size=(3, n))
    k = (c * th * dt / dx) ** 2
    y = O.apply_A(G, P, None, None, E)
    Ey = E[1]
    want = Ey - k * (np.roll(Ey, -1) - 2 * Ey + np.roll(Ey, 1))
    np.testing.assert_allclose(y[1], want, atol=1e-13)
    np.testing.assert_allclose(y[0], E[0], atol=1e-15)  # no x curl-curl in 1D
    # RHS: E_y - (c theta dt/dx)(B_z,right - B_z,left), node g between cells g-1 and g
    b = O.rhs(G, P, E, B, np.zeros((3, n)))
    np.testing.assert_allclose(b[1], Ey - c * th * dt / dx * (B[2] - np.roll(B[2], 1)), atol=1e-13)
    # eq. (1d-b): B_z,i^{n+1} = B_z,i - (c dt/dx)(E_y at node i+1 - E_y at node i)
    Bn1 = O.update_B(G, P, B, E)
    np.testing.assert_allclose(Bn1[2], B[2] - c * dt / dx * (np.roll(Ey, -1) - Ey), atol=1e-13)


def test_diffusion_fourier_mode_with_unlimited_lf():
    """beta = 0 (phi = 0): kappa = a/2 and D acts on sin(kx) with the
    eigenvalue -(a/dx)(1 - cos k dx); its sign is dissipative."""
    n, dx, a = 32, 0.25, 0.8
    G = O.grid(1, (n, 1, 1), (dx, 1, 1))
    x = (np.arange(n) + 0.5) * dx
    for mode in [1, 3, 7]:
        kx = 2 * math.pi * mode / (n * dx)
        Bc = np.zeros((3, n)); Bc[2] = np.sin(kx * x); Bc[0] = np.cos(kx * x)
        kap = O.kappa_B(G, Bc, np.full(n, a), 0.0)
        np.testing.assert_allclose(kap[0, 2], a / 2, atol=1e-15)
        DB = O.diffusion(G, kap, Bc)
        lam = -(a / dx) * (1 - math.cos(kx * dx))
        np.testing.assert_allclose(DB[2], lam * Bc[2], atol=1e-13)
        np.testing.assert_allclose(DB[0], lam * Bc[0], atol=1e-13)


def test_kappa_on_a_step_takes_the_limiter_values():
    """For a step the ratio r is 0 at the jump (first order, kappa = a/2),
    1 in flat regions (phi = 1: no diffusion) and +inf just past the jump."""
    n = 10
    G = O.grid(1, (n, 1, 1), (1.0, 1, 1))
    B = np.zeros((3, n)); B[1, 5:] = 1.0
    a = 0.6
    for beta in [1.0, 1.5]:
        k = O.kappa_B(G, B, np.full(n, a), beta)[0, 1]
        assert k[4] == pytest.approx(a / 2)          # face between cells 4 and 5: r = 0
        assert k[2] == 0.0 and k[7] == 0.0            # flat: r = 0/0 -> phi = 1
        assert k[5] == pytest.approx((1 - beta) * a / 2)  # r = +inf -> phi = beta
        assert k[9] == pytest.approx(a / 2)          # periodic wrap face 9|0 (1 -> 0): r = 0
    # linear profile: r = 1 -> phi = 1 -> kappa = 0 (second order recovered)
    E = np.zeros((3, n)); E[0] = np.arange(n) * 2.0
    kE = O.kappa_E(G, E, np.full(n, a), 1.0)
    assert np.all(kE[0, 0, 1:n - 2] == 0.0)


def test_filter_fourier_closed_form():
    """One filter pass of stride d multiplies a mode by phi + (1-phi) cos(k d dx)."""
    n, dx = 24, 0.3
    G = O.grid(2, (n, 6, 1), (dx, 0.2, 1))
    N = O.nnodes(G)
    ix = np.arange(N) % n
    for d in [1, 2]:
        for mode in [1, 2, 5]:
            k = 2 * math.pi * mode / (n * dx)
            f = np.zeros((3, N)); f[1] = np.cos(k * ix * dx)
            out = O.filter_axis(G, f, 0.5, d, 0)
            np.testing.assert_allclose(out[1], (0.5 + 0.5 * math.cos(k * d * dx)) * f[1], atol=1e-14)
    f = np.full((3, N), 2.5)
    np.testing.assert_allclose(O.smooth(G, f, 5), 2.5, atol=1e-14)


# ------------------------------------------------------------- solver and step
def _tiny_plasma(dim, n, ppc, seed=7):
    wl = synth.small("tiny", dim=dim, n=n, ppc=ppc, base="c2" if dim < 3 else "c5").replace(seed=seed)
    if dim == 1:
        wl = wl.replace(dx=(0.5, 1, 1))
    G = O.grid(dim, wl.n, wl.dx)
    E, Bc = synth.fields(wl)
    E = E + RNG.normal(size=E.shape) * 1e-3
    sp = []
    for s in range(wl.nsp):
        p = synth.particles(wl, s)
        sp.append(O.Species(wl.q[s], wl.m[s], O.global_positions(G, p["cell"], p["off"]), p["v"].T, p["w"]))
    return wl, G, E, Bc, sp


@pytest.mark.parametrize("dim,n", [(1, (6, 1, 1)), (2, (4, 3, 1)), (3, (3, 3, 3))])
def test_gmres_matches_dense_direct_solve(dim, n):
    wl, G, E, Bc, sp = _tiny_plasma(dim, n, 4)
    P = O.params(0.6, wl.dt)
    dep = O.deposit(G, sp, wl.dt, Bc, comoving=True)
    a_node = O.diffusion_speed(G, dep["u"], 1)
    kE = O.kappa_E(G, E, a_node, 1.5)
    b = O.rhs(G, P, E, Bc, dep["J_eff"])
    A = O.dense_A(G, P, dep["Mt"], kE)
    # the dense matrix reproduces the matrix-free operator
    xr = RNG.normal(size=E.shape)
    np.testing.assert_allclose(A @ xr.ravel(), O.apply_A(G, P, dep["Mt"], kE, xr).ravel(), atol=1e-13)
    # I + curl-curl is symmetric (curl_CN is the adjoint of curl_NC); the
    # mass term's symmetric part is positive semidefinite (q_s beta_s > 0 and
    # the symmetric part of alpha is (I + beta^2 B B)/(1 + beta^2 B^2))
    A_cc = O.dense_A(G, P, None, None)
    np.testing.assert_allclose(A_cc, A_cc.T, atol=1e-13)
    A_m = O.dense_A(G, P, dep["Mt"], None) - A_cc
    assert np.linalg.eigvalsh(0.5 * (A_m + A_m.T)).min() > -1e-13
    x_lu = O.dense_solve(A, b.ravel())
    x_gm, its, rel = O.gmres(G, P, dep["Mt"], kE, b, E, tol=1e-13, restart=10)
    assert its > 0 and rel <= 1e-13
    cond = np.linalg.cond(A)
    np.testing.assert_allclose(x_gm.ravel(), x_lu, atol=10 * cond * 1e-13 * np.abs(x_lu).max())


@pytest.mark.parametrize("dim,n", [(1, (8, 1, 1)), (2, (4, 4, 1)), (3, (3, 3, 3))])
def test_energy_theorem(dim, n):
    """theta = 1/2, no LF, lab-frame current: W_E + W_B + sum K_s is
    conserved per step up to the solver tolerance (ECSIM)."""
    wl, G, E, Bc, sp = _tiny_plasma(dim, n, 6)
    d0 = O.diagnostics(G, sp, E, Bc)
    W0 = d0["W_E"] + d0["W_B"] + sum(d0["K"])
    errs = []
    for tol in [1e-9, 1e-13]:
        r = O.step(G, sp, E, Bc, dt=wl.dt, theta=0.5, comoving=False, lf_E=False, lf_B=False, tol=tol, restart=40)
        d1 = O.diagnostics(G, r["species"], r["E"], r["B"])
        W1 = d1["W_E"] + d1["W_B"] + sum(d1["K"])
        errs.append(abs(W1 - W0) / W0)
    assert errs[1] < 1e-11
    # with LF diffusion on the field energy is not conserved (it dissipates)
    r = O.step(G, sp, E, Bc, dt=wl.dt, theta=0.5, comoving=False, lf_E=True, lf_B=True, beta_lim=0.0,
               a_mode=1, tol=1e-13)
    d1 = O.diagnostics(G, r["species"], r["E"], r["B"])
    assert d1["W_E"] + d1["W_B"] + sum(d1["K"]) < W0 * (1 - 1e-9)


def test_energy_theorem_fails_with_the_printed_mass_coefficient():
    """Negative control for the reading of the mass-term coefficient: the
    printed 4 pi/(c dV) breaks energy conservation; 4 pi theta dt/dV keeps it."""
    wl, G, E, Bc, sp = _tiny_plasma(2, (4, 4, 1), 6)
    P = O.params(0.5, wl.dt)
    dep = O.deposit(G, sp, wl.dt, Bc, comoving=False)
    b = O.rhs(G, P, E, Bc, dep["J_eff"])
    d0 = O.diagnostics(G, sp, E, Bc)
    W0 = d0["W_E"] + d0["W_B"] + sum(d0["K"])
    res = {}
    for name, scale in [("derived", 1.0), ("printed", 1.0 / (P.theta * P.dt))]:
        Eth, _, _ = O.gmres(G, P, dep["Mt"] * scale, None, b, E, tol=1e-13)
        Bn1 = O.update_B(G, P, Bc, Eth)
        En1 = O.update_E(0.5, E, Eth)
        sp1 = [O.Species(s.q, s.m, *O.push_species(G, O.beta_s(s.q, s.m, wl.dt), wl.dt, s.x, s.v, Eth, dep["Bn"]),
                         s.w) for s in sp]
        d1 = O.diagnostics(G, sp1, En1, Bn1)
        res[name] = abs(d1["W_E"] + d1["W_B"] + sum(d1["K"]) - W0) / W0
    assert res["derived"] < 1e-11
    assert res["printed"] > 1e-6


def test_gauss_identity_without_lf():
    """div_NC (E^{n+1} - E^n) = -4 pi dt div_NC Jbar exactly (LF off), with
    Jbar = J_eff + (1/dV) Mtilde E^{n+theta}; div_NC curl_CN = 0."""
    wl, G, E, Bc, sp = _tiny_plasma(3, (3, 4, 3), 5)
    r = O.step(G, sp, E, Bc, dt=wl.dt, theta=0.55, comoving=True, lf_E=False, lf_B=False, solve="dense")
    dep = r["dep"]
    Jbar = dep["J_eff"] + O.mass_apply(G, dep["Mt"], r["Eth"]) / O.cellvol(G)
    lhs = O.div_nc(G, r["E"] - E)
    rhs = -4 * math.pi * wl.dt * O.div_nc(G, Jbar)
    np.testing.assert_allclose(lhs, rhs, atol=1e-12 * np.abs(rhs).max())


def _light_wave(lf, beta, cfl=0.4, nsteps=25):
    n, dx = 80, 0.01
    G = O.grid(1, (n, 1, 1), (dx, 1, 1))
    dt = cfl * dx
    xn = -0.4 + np.arange(n) * dx
    xc = xn + 0.5 * dx
    E = np.zeros((3, n)); B = np.zeros((3, n))
    E[1] = (np.abs(xn) < 0.2).astype(float)
    B[2] = (np.abs(xc) < 0.2).astype(float)
    P = O.params(0.5, dt)
    a = np.full(n, 1.0)
    for _ in range(nsteps):
        kE = O.kappa_E(G, E, a, beta) if lf else None
        kB = O.kappa_B(G, B, a, beta) if lf else None
        b = O.rhs(G, P, E, B, np.zeros((3, n)))
        Eth, _, _ = O.gmres(G, P, None, kE, b, E, tol=1e-13)
        B = O.update_B(G, P, B, Eth, kB)
        E = O.update_E(0.5, E, Eth)
    t = nsteps * dt
    exact = (np.abs(((xn - t + 0.4) % 0.8) - 0.4) < 0.2).astype(float)
    return E[1], B[2], exact


def _overshoot(f):
    return max(f.max() - 1.0, -f.min(), 0.0)


def test_light_wave_lf_suppresses_oscillations():
    """Sec. 4.1 (top-hat light wave, CFL 0.4, t = 0.1): without LF diffusion
    the solution oscillates by tens of percent; the LF term (a = c) cuts the
    over/undershoot by a large factor, the unlimited form (beta = 0) keeps B
    inside [0, 1], and the limiter gives a sharper front than beta = 0.
    (The figure is not available, so amplitudes are not pinned beyond this.)"""
    Ey, Bz, exact = _light_wave(False, 1.0)
    base = min(_overshoot(Ey), _overshoot(Bz))
    assert base > 0.2
    errs = {}
    for beta in [0.0, 1.0, 1.5]:
        Ey, Bz, exact = _light_wave(True, beta)
        assert _overshoot(Ey) < base / 3 and _overshoot(Bz) < base / 10
        errs[beta] = np.abs(Ey - exact).sum()
        if beta == 0.0:
            assert _overshoot(Bz) < 1e-3
    assert errs[1.0] < errs[0.0] and errs[1.5] < errs[0.0]


def test_light_wave_energy_conserved_without_lf():
    n, dx = 80, 0.01
    G = O.grid(1, (n, 1, 1), (dx, 1, 1))
    E = np.zeros((3, n)); B = np.zeros((3, n))
    E[1, 20:60] = 1.0; B[2, 20:60] = 1.0
    P = O.params(0.5, 0.004)
    W0 = (E ** 2).sum() + (B ** 2).sum()
    for _ in range(10):
        b = O.rhs(G, P, E, B, np.zeros((3, n)))
        Eth, _, _ = O.gmres(G, P, None, None, b, E, tol=1e-14)
        B = O.update_B(G, P, B, Eth)
        E = O.update_E(0.5, E, Eth)
    assert abs((E ** 2).sum() + (B ** 2).sum() - W0) / W0 < 1e-12


def test_half_offset_enumeration():
    assert len(O.half_offsets(3)) == 14
    assert len(O.half_offsets(2)) == 5
    assert len(O.half_offsets(1)) == 2
    seen = set()
    for o in O.half_offsets(3):
        assert tuple(-c for c in o) not in seen or o == (0, 0, 0)
        seen.add(o)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_node_average_is_exact_on_linear_fields(dim):
    """The node average of a cell-centred field (the B interpolated to the
    particles) reproduces a linear field exactly at the node: the 2^dim cells
    around node g have centres x_g +- dx/2 per axis.  Nodes whose cells wrap
    around the periodic boundary are left out.  A wrong cell offset (cells
    g..g+1 instead of g-1..g) would give the field at x_g + dx: the check
    tells the two apart."""
    n = (7, 6, 5)[:dim] + (1,) * (3 - dim)
    dx = (0.5, 0.4, 0.3)[:dim] + (1.0,) * (3 - dim)
    G = O.grid(dim, n, dx)
    N = O.nnodes(G)
    idx = np.stack(np.unravel_index(np.arange(N), n[::-1])[::-1])  # (i, j, k) per linear index
    xc = (idx + 0.5) * np.array(dx)[:, None]
    xn = idx * np.array(dx)[:, None]
    coef = np.array([[0.3, 1.7, -0.6, 0.25], [-1.1, 0.4, 2.2, -0.9], [0.05, -2.0, 0.7, 1.3]])

    def lin(x):
        return np.stack([c[0] + sum(c[1 + d] * x[d] for d in range(dim)) for c in coef])

    Bn = O.node_avg(G, lin(xc))
    inner = np.all(idx[:dim] >= 1, axis=0)
    assert inner.sum() > 0
    np.testing.assert_allclose(Bn[:, inner], lin(xn)[:, inner], rtol=0, atol=1e-13)
    shifted = lin(xn + np.array(dx)[:, None] * (np.arange(3) < dim)[:, None])
    assert np.abs(Bn[:, inner] - shifted[:, inner]).max() > 0.1
    # a uniform field stays uniform
    U = np.array([0.2, -0.7, 1.9])[:, None] * np.ones((3, N))
    np.testing.assert_allclose(O.node_avg(G, U), U, rtol=1e-15, atol=0)


@pytest.mark.parametrize("species_split", [1, 2])
def test_gauss_residual_vanishes_for_a_discrete_poisson_mode(species_split):
    """Closed form of the discrete Gauss residual: for E_x = A sin(kx x)
    cos(ky y) at the nodes, div_NC E at the cell centre is
    (2A/dx) sin(kx dx/2) cos(kx x_c) cos(ky y_c) cos(ky dy/2) (face means), and
    the cell mean of the node charge rho = R cos(kx x) cos(ky y) is
    R cos(kx x_c) cos(kx dx/2) cos(ky y_c) cos(ky dy/2); so with
    R = A tan(kx dx/2) / (2 pi dx) the residual is zero to rounding, while
    the continuum amplitude R = A kx / (4 pi) leaves a residual of the size of
    the discretisation error.  The charge may be split over species."""
    n, dx = (8, 6, 5), (0.5, 0.4, 0.3)
    G = O.grid(3, n, dx)
    N = O.nnodes(G)
    idx = np.stack(np.unravel_index(np.arange(N), n[::-1])[::-1])
    x, y = idx[0] * dx[0], idx[1] * dx[1]
    kx, ky = 2 * math.pi * 2 / (n[0] * dx[0]), 2 * math.pi / (n[1] * dx[1])
    A = 0.37
    E = np.zeros((3, N))
    E[0] = A * np.sin(kx * x) * np.cos(ky * y)
    R = A * math.tan(0.5 * kx * dx[0]) / (2 * math.pi * dx[0])
    rho = R * np.cos(kx * x) * np.cos(ky * y)
    rho_s = [rho / species_split] * species_split
    assert O.gauss_residual(G, E, rho_s) < 1e-13
    rho_c = (A * kx / (4 * math.pi)) * np.cos(kx * x) * np.cos(ky * y)
    r_cont = O.gauss_residual(G, E, [rho_c])
    assert 1e-3 < r_cont < 0.5
    # and the residual is relative to the charge, not to E
    assert abs(O.gauss_residual(G, 10 * E, [10 * rho]) - O.gauss_residual(G, E, [rho])) < 1e-13


def test_picard_limiter_step():
    """The one-step Picard option of the E limiter (Sec. 2.2: the ratio uses
    the unknown E^{n+theta}): its E^{n+theta} solves the system whose limiter
    is taken from the lagged solution; with beta = 0 the limiter is the
    constant phi = 0, so the option changes nothing; and with the limiter
    active it changes the answer."""
    wl, G, E, Bc, sp = _tiny_plasma(3, (4, 3, 3), 6)
    E = E + 0.05 * np.random.default_rng(3).standard_normal(E.shape)
    kw = dict(dt=wl.dt, theta=0.5, comoving=True, lf_E=True, lf_B=True, a_mode=0, solve="dense")
    lag = O.step(G, sp, E, Bc, beta_lim=1.5, **kw)
    pic = O.step(G, sp, E, Bc, beta_lim=1.5, limiter_lag="picard1", **kw)
    kE1 = O.kappa_E(G, lag["Eth"], pic["a_node"], 1.5)
    np.testing.assert_array_equal(pic["kE"], kE1)
    P = O.params(0.5, wl.dt)
    res = O.apply_A(G, P, pic["dep"]["Mt"], kE1, pic["Eth"]) - pic["b"]
    assert np.linalg.norm(res) <= 1e-12 * np.linalg.norm(pic["b"])
    assert np.abs(pic["Eth"] - lag["Eth"]).max() > 1e-8 * np.abs(lag["Eth"]).max()
    lag0 = O.step(G, sp, E, Bc, beta_lim=0.0, **kw)
    pic0 = O.step(G, sp, E, Bc, beta_lim=0.0, limiter_lag="picard1", **kw)
    np.testing.assert_allclose(pic0["Eth"], lag0["Eth"], rtol=0, atol=1e-13 * np.abs(lag0["Eth"]).max())
