"""GPU tests of the learned preconditioner through the C ABI.

Parity bar: the BF16/FP32 GPU network against the FP64 reference fed the
same BF16-rounded inputs, weights and activations (oracle/cnn.py with
quant=True).  With dyadic inputs and weights (every sum exact in FP32) the
forward pass must agree bit for bit.  With random inputs the FP32
accumulation order alone gives ~1e-7, but a BF16 rounding that this order
flips (probability ~1e-4 per activation) moves one activation by one BF16 ulp
(2^-8 relative) and spreads through the next layers: the normwise bar is
1e-3 for the forward pass and 3e-3 for the weight gradient.  Against the
unrounded FP64 network the error is the BF16 error itself, <= 2e-2.  The preconditioned
solve is judged like every solve: true relative residual <= tol, and the
same field as plain GMRES."""
import numpy as np
import pytest

import synth
from oracle import cnn as C
from tests import harness as H

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _ctx(n):
    from paper_2506_11320_amd import Simulation
    return Simulation(3, n, (0.5, 0.5, 0.5), theta=0.5, dt=0.5)


def _rand_w(rng, scale=1.0):
    parts = []
    for ci, co in C.LAYERS:
        parts.append(rng.standard_normal(27 * ci * co) * scale * np.sqrt(2.0 / (27 * ci)))
    return np.concatenate(parts).astype(np.float32)


def _layer_errs(g, ref):
    offs = [0, 27 * 3 * 32, 27 * 3 * 32 + 27 * 32 * 32, C.NW]
    return [H.relerr(g[offs[l]:offs[l + 1]], ref[offs[l]:offs[l + 1]]) for l in range(3)]


# (12, 10, 9): 1080 nodes = 67.5 MFMA tiles (ragged); (3, 4, 5): the smallest periodic box
@pytest.mark.parametrize("n", [(12, 10, 9), (3, 4, 5), (16, 16, 16)])
def test_forward_matches_oracle(n):
    print(f"[gpu] cnn forward {n}", flush=True)
    N = n[0] * n[1] * n[2]
    sim = _ctx(n)
    sim.cnn_init(7)
    rng = np.random.default_rng(11)
    w = _rand_w(rng)
    sim.cnn_set_weights(w)
    assert np.array_equal(sim.cnn_weights(), w)
    r = rng.standard_normal((3, N)) * 3e-3
    z = sim.cnn_apply(torch.from_numpy(r).to(sim.device)).cpu().numpy()
    ref = C.forward_apply(w.astype(np.float64), r, n, quant=True)
    e = H.relerr(z, ref)
    print(f"  rel err vs BF16-rounded FP64 reference {e:.2e}", flush=True)
    assert e <= 1e-3
    assert H.relerr(z, C.forward_apply(w.astype(np.float64), r, n)) <= 2e-2
    # bit-identical on a second application
    z2 = sim.cnn_apply(torch.from_numpy(r).to(sim.device)).cpu().numpy()
    assert np.array_equal(z, z2)
    sim.close()


def test_scaled_application():
    """ge_cnn_apply_scaled(r, s) = N(s r) / s: against the BF16-rounded FP64
    reference on the input scaled by 1/RMS (what ge_cnn_apply does), exactly
    twice as large for (2 r, s / 2) (the network's input is then bit-identical
    and its output divided by an exactly halved scale), and a non-positive or
    non-finite scale is refused."""
    print("[gpu] cnn scaled application (12, 10, 9)", flush=True)
    from paper_2506_11320_amd import GlecsimError
    n = (12, 10, 9)
    N = n[0] * n[1] * n[2]
    sim = _ctx(n)
    sim.cnn_init(7)
    rng = np.random.default_rng(12)
    w = _rand_w(rng)
    sim.cnn_set_weights(w)
    r = rng.standard_normal((3, N)) * 3e-3
    s = 1.0 / np.sqrt(np.mean(r * r))
    rt = torch.from_numpy(r).to(sim.device)
    z1 = sim.cnn_apply_scaled(rt, s).cpu().numpy()
    ref = C.forward_apply(w.astype(np.float64), r, n, quant=True)
    assert H.relerr(z1, ref) <= 1e-3
    assert H.relerr(z1, sim.cnn_apply(rt).cpu().numpy()) <= 1e-3
    z2 = sim.cnn_apply_scaled(2.0 * rt, s / 2.0).cpu().numpy()
    assert np.array_equal(z2, 2.0 * z1)
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(GlecsimError):
            sim.cnn_apply_scaled(rt, bad)
    sim.close()


def test_forward_on_a_walled_grid():
    """On a grid with a wall at x = 0 and an inflow plane at x = L the network
    runs on the domain periodic along x over the node planes 0 .. nxp - 1 (the
    inflow plane, all of whose components are held, is left out), and the
    output equals the input on the held components: the tangential ones on the
    wall plane and all three on the inflow plane."""
    from paper_2506_11320_amd import Simulation
    print("[gpu] cnn forward on a walled grid", flush=True)
    n = (12, 10, 9)  # physical cells along x; the grid stores 13 node planes
    sim = Simulation(3, n, (0.5, 0.5, 0.5), theta=0.5, dt=0.5, bc=(1, 2))  # wall, inflow
    nxs = n[0] + 1
    N = nxs * n[1] * n[2]
    sim.cnn_init(7)
    rng = np.random.default_rng(13)
    w = _rand_w(rng)
    sim.cnn_set_weights(w)
    r = rng.standard_normal((3, N)) * 3e-3
    z = sim.cnn_apply(torch.from_numpy(r).to(sim.device)).cpu().numpy()
    rg = r.reshape(3, n[2], n[1], nxs)
    zg = z.reshape(3, n[2], n[1], nxs)
    assert np.array_equal(zg[1:, :, :, 0], rg[1:, :, :, 0])
    assert np.array_equal(zg[:, :, :, n[0]], rg[:, :, :, n[0]])
    # the rest: the network on the reduced periodic domain, with the GPU's
    # normalisation (the RMS of the whole input)
    inner = np.ascontiguousarray(rg[..., :n[0]]).reshape(3, -1)
    rms = np.sqrt(np.mean(r * r))
    ref = C.forward_grid(w.astype(np.float64), inner, n, 1.0 / rms, quant=True).reshape(3, n[2], n[1], n[0])
    got = zg[..., :n[0]].copy()
    got[1:, :, :, 0] = 0.0
    ref[1:, :, :, 0] = 0.0
    e = H.relerr(got, ref)
    print(f"  rel err vs BF16-rounded FP64 reference {e:.2e}", flush=True)
    assert e <= 1e-3
    sim.close()


def _dyadic_w(rng):
    """Sparse weights in {0, +-1/2, +-1/4}: every partial sum of the network
    on +-1 inputs is a short dyadic number, exact in FP32."""
    w = rng.choice([0.5, -0.5, 0.25, -0.25], size=C.NW) * (rng.random(C.NW) < 0.06)
    return w.astype(np.float32)


@pytest.mark.parametrize("n", [(12, 10, 9), (16, 16, 16)])
def test_forward_bit_exact_on_dyadic_data(n):
    print(f"[gpu] cnn dyadic forward {n}", flush=True)
    N = n[0] * n[1] * n[2]
    sim = _ctx(n)
    sim.cnn_init(7)
    rng = np.random.default_rng(21)
    w = _dyadic_w(rng)
    sim.cnn_set_weights(w)
    r = rng.choice([-1.0, 1.0], size=(3, N))  # RMS exactly 1: no rescaling rounding
    z = sim.cnn_apply(torch.from_numpy(r).to(sim.device)).cpu().numpy()
    ref = C.forward_apply(w.astype(np.float64), r, n, quant=True)
    assert np.abs(ref).max() > 0
    assert np.array_equal(z, ref), np.abs(z - ref).max()
    sim.close()


def test_gradient_on_dyadic_data():
    """Forward exact, so the loss agrees to FP32 summation order; the
    backward sums are inexact in FP32 and may flip a BF16 rounding."""
    print("[gpu] cnn dyadic loss/grad", flush=True)
    sim = _ctx((8, 8, 8))
    sim.cnn_init(5)
    rng = np.random.default_rng(31)
    w = _dyadic_w(rng)
    sim.cnn_set_weights(w)
    B, k = 4, 5
    x = rng.choice([-1.0, 0.0, 1.0], size=(B, (k + 6) ** 3, 3)).astype(np.float32)
    e = rng.choice([-0.5, 0.0, 0.5], size=(B, k ** 3, 3)).astype(np.float32)
    L, g = sim.cnn_loss_grad(torch.from_numpy(x), torch.from_numpy(e))
    Lr, gr = C.loss_grad(w.astype(np.float64), x.astype(np.float64), e.astype(np.float64), quant=True)
    errs = _layer_errs(g.cpu().numpy().astype(np.float64), gr)
    print(f"  loss {L:.9e} vs {Lr:.9e}; layer grad errs {errs}", flush=True)
    assert abs(L - Lr) <= 1e-6 * Lr
    assert max(errs) <= 1e-3
    sim.close()


def test_initial_weights_are_near_identity():
    n = (8, 6, 5)
    N = n[0] * n[1] * n[2]
    sim = _ctx(n)
    sim.cnn_init(3)
    w = sim.cnn_weights().astype(np.float64)
    rng = np.random.default_rng(2)
    r = rng.standard_normal((3, N))
    z = sim.cnn_apply(torch.from_numpy(r).to(sim.device)).cpu().numpy()
    assert H.relerr(z, C.forward_apply(w, r, n, quant=True)) <= 1e-3
    assert H.relerr(z, r) <= 0.1
    sim.close()


@pytest.mark.parametrize("B,k", [(3, 3), (4, 6)])
def test_loss_and_gradient_match_oracle(B, k):
    """(3, 3): 1029 layer-1 nodes (two 1024-node reduction chunks, ragged);
    (4, 6): several chunks in every layer."""
    print(f"[gpu] cnn loss/grad B={B} crop={k}", flush=True)
    sim = _ctx((8, 8, 8))
    sim.cnn_init(5)
    rng = np.random.default_rng(100 + k)
    w = _rand_w(rng)
    sim.cnn_set_weights(w)
    x = rng.standard_normal((B, (k + 6) ** 3, 3)).astype(np.float32)
    e = (0.3 * rng.standard_normal((B, k ** 3, 3))).astype(np.float32)
    L, g = sim.cnn_loss_grad(torch.from_numpy(x), torch.from_numpy(e))
    g = g.cpu().numpy().astype(np.float64)
    Lr, gr = C.loss_grad(w.astype(np.float64), x.astype(np.float64), e.astype(np.float64), quant=True)
    errs = _layer_errs(g, gr)
    print(f"  loss {L:.6e} vs {Lr:.6e}; layer grad errs {errs}", flush=True)
    assert abs(L - Lr) <= 1e-4 * Lr
    assert max(errs) <= 3e-3
    L0, g0 = C.loss_grad(w.astype(np.float64), x.astype(np.float64), e.astype(np.float64))
    assert abs(L - L0) <= 2e-2 * L0
    assert max(_layer_errs(g, g0)) <= 5e-2
    sim.close()


def test_pair_store_keeps_the_newest_sixteen():
    n = (6, 5, 4)
    N = n[0] * n[1] * n[2]
    sim = _ctx(n)
    sim.cnn_init(0, max_pairs=16)
    rng = np.random.default_rng(0)
    for i in range(20):
        r = torch.from_numpy(rng.standard_normal((3, N)))
        sim.cnn_add_pair(r, 0.5 * r)
        assert sim.cnn_npairs() == min(i + 1, 16)
    sim.close()


def _reconnection_case():
    wl = synth.small("cnn", dim=3, n=(12, 10, 8), ppc=16, base="c4", fp32=True)
    parts = H.species_arrays(wl, True)
    E, B = synth.fields(wl)
    return wl, parts, E, B


def test_training_and_flexible_gmres():
    from paper_2506_11320_amd import GE_HARVEST_KRYLOV, GE_HARVEST_SOLUTION, GE_PC_CNN
    print("[gpu] cnn harvest/train/FGMRES", flush=True)
    wl, parts, E, B = _reconnection_case()
    sim = H.make_sim(wl, parts, E, B)
    sim.cnn_init(3)
    sim.cnn_harvest(GE_HARVEST_SOLUTION)
    for _ in range(6):
        rep = sim.step(tol=1e-10)
        assert rep["converged"]
    assert sim.cnn_npairs() == 6
    # Krylov pairs: (A v_j, v_j) for the Arnoldi vectors 1..k-1 of the last cycle
    sim.cnn_harvest(GE_HARVEST_SOLUTION | GE_HARVEST_KRYLOV)
    rep = sim.step(tol=1e-10)
    assert sim.cnn_npairs() == 6 + 1 + (rep["iterations"] - 1)
    tr = sim.cnn_train(crop=6, batch=8, iters=80, lr=2e-3, seed=5)
    print(f"  train {tr}", flush=True)
    assert tr["steps"] == 80 and tr["pairs"] == sim.cnn_npairs()
    assert np.isfinite(tr["loss_last"]) and tr["loss_last"] < tr["loss_first"]
    w1 = sim.cnn_weights()
    # training is deterministic: re-initialise and train again
    sim.cnn_init(3)
    sim.cnn_train(crop=6, batch=8, iters=80, lr=2e-3, seed=5)
    assert np.array_equal(sim.cnn_weights(), w1)
    sim.cnn_harvest(0)
    sim.deposit()
    tol = 1e-9
    rp = sim.solve(tol=tol)
    Ep = sim.gather("Eth").cpu().numpy()
    rc = sim.solve(tol=tol, precond=GE_PC_CNN)
    Ec = sim.gather("Eth").cpu().numpy()
    print(f"  plain {rp['iterations']} it, cnn {rc['iterations']} it", flush=True)
    assert rp["converged"] and rc["converged"] and not rc["fallback"]
    assert rc["relres"] <= tol
    assert H.relerr(Ec, Ep) <= 1e-6
    # the true residual of the FGMRES answer, recomputed through the operator
    b = sim.gather("rhs")
    res = (b - sim.apply_operator(torch.from_numpy(Ec).to(sim.device))).cpu().numpy()
    assert np.linalg.norm(res) <= 1.01 * tol * np.linalg.norm(b.cpu().numpy())
    sim.close()


def test_nonfinite_network_falls_back_to_plain_gmres():
    from paper_2506_11320_amd import GE_PC_CNN
    wl, parts, E, B = _reconnection_case()
    sim = H.make_sim(wl, parts, E, B)
    sim.cnn_init(1)
    w = sim.cnn_weights()
    w[27 * 3 * 32 + 5] = np.nan
    sim.cnn_set_weights(w)
    sim.deposit()
    rp = sim.solve(tol=1e-9)
    Ep = sim.gather("Eth").cpu().numpy()
    rc = sim.solve(tol=1e-9, precond=GE_PC_CNN)
    assert rc["fallback"] and rc["converged"] and rc["relres"] <= 1e-9
    assert H.relerr(sim.gather("Eth").cpu().numpy(), Ep) <= 1e-6
    sim.close()


def test_zero_network_falls_back_to_plain_gmres():
    """A network that maps everything to zero makes the flexible least-squares
    problem singular; the solve must finish with plain GMRES."""
    from paper_2506_11320_amd import GE_PC_CNN
    wl, parts, E, B = _reconnection_case()
    sim = H.make_sim(wl, parts, E, B)
    sim.cnn_init(1)
    sim.cnn_set_weights(np.zeros(sim.cnn_size(), dtype=np.float32))
    sim.deposit()
    rp = sim.solve(tol=1e-9)
    Ep = sim.gather("Eth").cpu().numpy()
    rc = sim.solve(tol=1e-9, precond=GE_PC_CNN)
    assert rc["fallback"] and rc["converged"] and rc["relres"] <= 1e-9
    assert H.relerr(sim.gather("Eth").cpu().numpy(), Ep) <= 1e-6
    sim.close()


# the reconnection box (periodic) and the shock box (wall at x = 0, inflow at
# the far end), whose held boundary rows the preconditioner keeps as given
@pytest.mark.parametrize("base,bc", [("c5", (0, 0)), ("c4", (1, 2))])
def test_trained_network_saves_iterations(base, bc):
    """What the learned preconditioner gains: after harvesting plain solves and
    training, CNN-preconditioned FGMRES reaches the same true residual as
    plain GMRES in fewer iterations on each of the following systems, and in
    fewer than with the untrained (near-identity) network on the same system."""
    from paper_2506_11320_amd import GE_HARVEST_KRYLOV, GE_HARVEST_SOLUTION, GE_PC_CNN
    print(f"[gpu] cnn gain {base} bc {bc}", flush=True)
    wl = synth.small("cnn_gain", dim=3, n=(16, 12, 12), ppc=16, base=base, fp32=True, bc=bc)
    parts = H.species_arrays(wl, True)
    E, B = synth.fields(wl)
    sim = H.make_sim(wl, parts, E, B)
    sim.cnn_init(1, max_pairs=128)
    w0 = sim.cnn_weights()
    tol = 1e-8
    sim.cnn_harvest(GE_HARVEST_SOLUTION | GE_HARVEST_KRYLOV)
    for _ in range(6):
        sim.step(tol=tol)
    sim.cnn_harvest(0)
    tr = sim.cnn_train(crop=8, batch=16, iters=300, lr=1e-3, seed=7)
    assert tr["loss_last"] < 0.5 * tr["loss_first"]
    w1 = sim.cnn_weights()
    rows = []
    for _ in range(3):
        sim.deposit()
        rp = sim.solve(tol=tol)
        sim.cnn_set_weights(w0)
        r0 = sim.solve(tol=tol, precond=GE_PC_CNN)
        sim.cnn_set_weights(w1)
        rc = sim.solve(tol=tol, precond=GE_PC_CNN)
        for r in (rp, r0, rc):
            assert r["converged"] and r["relres"] <= tol
        assert not rc["fallback"]
        rows.append((rp["iterations"], r0["iterations"], rc["iterations"]))
        sim.push()
        sim.update_fields()
    print(f"  (plain, untrained, trained) iterations per system: {rows}", flush=True)
    for p_it, u_it, c_it in rows:
        assert c_it < p_it and c_it < u_it
    sim.close()
