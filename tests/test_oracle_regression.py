"""The paper's 1D experiments on the oracle (Sec. 4.1 top-hat light wave,
Sec. 4.2 uniform fast flow): the qualitative claims of the text, and the
closed form of the explicit magnetic diffusion that decides the CFL-2 case."""
import numpy as np
import pytest

import oracle as O
import synth
from tests import harness as H


def _overshoot(f):
    return max(f.max() - 1.0, -f.min(), 0.0)


def _light_wave(lf_E, lf_B, beta, cfl, nsteps, n=80, dx=0.01, ns_e=0):
    G = O.grid(1, (n, 1, 1), (dx, 1, 1))
    xn = -0.4 + np.arange(n) * dx
    xc = xn + 0.5 * dx
    E = np.zeros((3, n)); B = np.zeros((3, n))
    E[1] = (np.abs(xn) < 0.2).astype(float)
    B[2] = (np.abs(xc) < 0.2).astype(float)
    P = O.params(0.5, cfl * dx)
    a = np.full(n, 1.0)
    for _ in range(nsteps):
        kE = O.kappa_E(G, E, a, beta) if lf_E else None
        kB = O.kappa_B(G, B, a, beta) if lf_B else None
        b = O.rhs(G, P, E, B, np.zeros((3, n)))
        Eth, _, _ = O.gmres(G, P, None, kE, b, E, tol=1e-13)
        B = O.update_B(G, P, B, Eth, kB)
        E = O.update_E(0.5, E, Eth)
        if ns_e:
            E = O.smooth(G, E, ns_e)
    return E, B


def _l1_error(E, B, cfl, nsteps, n=80, dx=0.01):
    t = nsteps * cfl * dx
    xn = -0.4 + np.arange(n) * dx
    xc = xn + 0.5 * dx
    ex = lambda x: (np.abs(((x - t + 0.4) % 0.8) - 0.4) < 0.2).astype(float)
    return dx * np.abs(E[1] - ex(xn)).sum(), dx * np.abs(B[2] - ex(xc)).sum()


@pytest.mark.parametrize("cfl", [0.4, 1.0, 2.0])
def test_explicit_B_diffusion_grid_mode_factor(cfl):
    """Eq. (flux-b) with E = 0 on the grid-scale mode B_z = (-1)^i: the MC
    limiter returns 0 (the slope ratio is -1), so one update multiplies the
    mode by 1 - 2 a dt/dx.  With a = c the factor is -3 at CFL 2: the explicit
    term alone amplifies the mode, and the light wave at CFL 2 with the
    magnetic diffusion on grows."""
    n, dx = 16, 0.01
    G = O.grid(1, (n, 1, 1), (dx, 1, 1))
    P = O.params(0.5, cfl * dx)
    B = np.zeros((3, n)); B[2] = (-1.0) ** np.arange(n)
    kB = O.kappa_B(G, B, np.full(n, 1.0), 1.0)
    out = O.update_B(G, P, B, np.zeros((3, n)), kB)
    assert np.allclose(out[2], (1.0 - 2.0 * cfl) * B[2], rtol=0, atol=1e-14)
    assert np.allclose(out[:2], 0.0)


def test_light_wave_claims():
    """Sec. 4.1 at CFL 0.4: the diffusion removes most of the over/undershoot
    of the centred scheme, and the limiter (beta = 1) gives a sharper front
    (smaller L1 error) than the first-order diffusion (beta = 0)."""
    n, dx, cfl, steps = 80, 0.01, 0.4, 25
    E0, B0 = _light_wave(False, False, 1.0, cfl, steps)
    base = min(_overshoot(E0[1]), _overshoot(B0[2]))
    assert base > 0.2
    xn = -0.4 + np.arange(n) * dx
    t = steps * cfl * dx
    exact = (np.abs(((xn - t + 0.4) % 0.8) - 0.4) < 0.2).astype(float)
    errs = {}
    for beta in (0.0, 1.0):
        E, B = _light_wave(True, True, beta, cfl, steps)
        assert _overshoot(E[1]) < base / 3 and _overshoot(B[2]) < base / 10
        errs[beta] = np.abs(E[1] - exact).sum()
    assert errs[1.0] < errs[0.0]


def test_light_wave_cfl2():
    """At CFL 2 the implicit diffusion in the field solve still reduces the
    oscillation amplitude of E and B, while adding the explicit magnetic
    diffusion with a = c makes the run grow (factor 1 - 2 a dt/dx = -3 on the
    grid-scale mode)."""
    E, B = _light_wave(False, False, 1.0, 2.0, 5)
    Ee, Be = _light_wave(True, False, 1.0, 2.0, 5)
    Eb, Bb = _light_wave(True, True, 1.0, 2.0, 5)
    assert _overshoot(Ee[1]) < _overshoot(E[1]) and _overshoot(Be[2]) < _overshoot(B[2])
    assert _overshoot(Bb[2]) > 10.0


def fast_flow_drift(comoving, ns_j, steps):
    """Largest |P_x(t) - P_x(0)| / |P_x(0)| of the total particle momentum over
    the run of the Sec. 4.2 fast flow (uniform, so P is conserved exactly)."""
    wl = synth.workloads()["ff1d"]
    parts = H.species_arrays(wl, False)
    E, B = synth.fields(wl)
    G, sp = H.oracle_species(wl, parts)
    P0 = sum(s.m * (s.w * s.v[:, 0]).sum() for s in sp)
    drift = 0.0
    for _ in range(steps):
        r = O.step(G, sp, E, B, dt=wl.dt, theta=wl.theta, comoving=comoving, lf_E=wl.lf_E, lf_B=wl.lf_B,
                   beta_lim=wl.beta_lim, a_mode=wl.a_mode, tol=1e-10, restart=40, n_smooth_j=ns_j)
        sp, E, B = r["species"], r["E"], r["B"]
        P = sum(s.m * (s.w * s.v[:, 0]).sum() for s in sp)
        drift = max(drift, abs(P - P0) / abs(P0))
    return drift


def test_fast_flow_momentum_claim():
    """Sec. 4.2: the comoving-frame current with one smoothing pass keeps the
    total momentum of the uniform fast flow far better than the lab-frame
    current, with or without smoothing."""
    d_lab = fast_flow_drift(False, 0, 200)
    d_lab_s = fast_flow_drift(False, 1, 200)
    d_cm = fast_flow_drift(True, 1, 200)
    assert d_cm < 0.05 * min(d_lab, d_lab_s)


def test_light_wave_E_filter_claims():
    """Sec. 4.1 at t = 0.4 (100 steps, CFL 0.4) with E smoothed by the filter
    instead of the LF term (LF kept on B): one pass (d = 1) gives an error
    comparable to the unlimited LF diffusion (beta = 0); three passes
    (d = 1, 2, 1) smear the front far more; the limited LF diffusion is more
    accurate than either.  The text's overshoot for three passes is not
    reproduced (the filter weights are all positive, and none appears here)."""
    cfl, steps = 0.4, 100
    l1 = {}
    for key, kw in (("lf0", dict(lf_E=True, lf_B=True, beta=0.0)), ("lf1", dict(lf_E=True, lf_B=True, beta=1.0)),
                    ("f1", dict(lf_E=False, lf_B=True, beta=1.0, ns_e=1)),
                    ("f3", dict(lf_E=False, lf_B=True, beta=1.0, ns_e=3))):
        E, B = _light_wave(kw.pop("lf_E"), kw.pop("lf_B"), kw.pop("beta"), cfl, steps, **kw)
        l1[key] = _l1_error(E, B, cfl, steps)
    for i in range(2):
        assert 0.6 < l1["f1"][i] / l1["lf0"][i] < 1.4
        assert l1["f3"][i] > 1.8 * l1["f1"][i]
        assert l1["lf1"][i] < 0.7 * min(l1["f1"][i], l1["lf0"][i])
