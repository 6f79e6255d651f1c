"""Checkpoint and restore (ge_checkpoint / ge_restore) and the one-step Picard
option of the E limiter (GE_PICARD1), through the C ABI.

Resume: a run that writes a checkpoint and goes on, and a fresh context that
restores it and goes on the same way, must agree bit for bit (fields,
particles in cell order, the learned preconditioner's weights and its
preconditioned solve).  Picard: E^{n+theta} and the E limiter coefficients
against the oracle's picard1 step (1e-10, FP64)."""
import numpy as np
import pytest

import oracle as O
import synth
from tests import harness as H

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [
    ("3d_fp32", 3, (6, 5, 4), 20, "c5", True),
    ("2d_fp64", 2, (7, 5, 1), 30, "c2", False),
]


def _wl(dim, n, ppc, base, fp32):
    return synth.small("ckpt", dim=dim, n=n, ppc=ppc, base=base, fp32=fp32).replace(
        lf_E=True, lf_B=True, comoving=True, beta_lim=1.5)


def _state(sim):
    out = {"E": sim.gather("E").cpu().numpy(), "B": sim.gather("B").cpu().numpy()}
    for s in range(sim.nsp):
        for k, v in sim.particles(s).items():
            out[f"{k}{s}"] = v.cpu().numpy()
    return out


@pytest.mark.parametrize("name,dim,n,ppc,base,fp32", CASES)
def test_resume_is_bitwise_identical(name, dim, n, ppc, base, fp32, tmp_path):
    print(f"[gpu] checkpoint/restore {name}", flush=True)
    wl = _wl(dim, n, ppc, base, fp32)
    parts = H.species_arrays(wl, fp32)
    E, B = H.perturbed_fields(wl)
    a = H.make_sim(wl, parts, E, B, ns_j=1, dedner=True)
    for _ in range(2):
        a.step(tol=1e-10, maxit=2000, restart=30)
    path = str(tmp_path / "state.ckpt")
    a.checkpoint(path)
    assert a.step_count() == 2
    for _ in range(2):
        a.step(tol=1e-10, maxit=2000, restart=30)
    ref = _state(a)
    psi_a = a.gather("psi").cpu().numpy()
    a.close()
    b = H.make_bare_sim(wl, ns_j=1, dedner=True)
    b.restore(path)
    assert b.step_count() == 2 and b.nsp == wl.nsp
    for _ in range(2):
        b.step(tol=1e-10, maxit=2000, restart=30)
    got = _state(b)
    assert b.step_count() == 4
    for k in ref:
        assert np.array_equal(got[k], ref[k]), k
    assert np.array_equal(b.gather("psi").cpu().numpy(), psi_a)
    b.close()


def test_checkpoint_keeps_the_learned_preconditioner(tmp_path):
    from paper_2506_11320_amd import GE_HARVEST_SOLUTION, GE_PC_CNN
    print("[gpu] checkpoint with the CNN", flush=True)
    wl = _wl(3, (8, 6, 6), 12, "c4", True)
    parts = H.species_arrays(wl, True)
    E, B = synth.fields(wl)
    a = H.make_sim(wl, parts, E, B)
    a.cnn_init(2)
    a.cnn_harvest(GE_HARVEST_SOLUTION)
    for _ in range(3):
        a.step(tol=1e-10)
    a.cnn_harvest(0)
    a.cnn_train(crop=4, batch=4, iters=20, lr=2e-3, seed=3)
    path = str(tmp_path / "cnn.ckpt")
    a.checkpoint(path)
    w = a.cnn_weights()
    ra = a.step(tol=1e-9, precond=GE_PC_CNN)
    Ea = a.gather("E").cpu().numpy()
    a.close()
    b = H.make_bare_sim(wl)
    b.restore(path)
    assert np.array_equal(b.cnn_weights(), w)
    rb = b.step(tol=1e-9, precond=GE_PC_CNN)
    assert rb["iterations"] == ra["iterations"]
    assert np.array_equal(b.gather("E").cpu().numpy(), Ea)
    b.close()


def test_restore_refusals(tmp_path):
    from paper_2506_11320_amd import GlecsimError
    print("[gpu] restore refusals", flush=True)
    wl = _wl(2, (7, 5, 1), 10, "c2", False)
    parts = H.species_arrays(wl, False)
    E, B = H.perturbed_fields(wl)
    a = H.make_sim(wl, parts, E, B)
    a.step(tol=1e-10)
    path = tmp_path / "a.ckpt"
    a.checkpoint(str(path))
    # between a deposit and its update the state is not a step boundary
    a.deposit()
    with pytest.raises(GlecsimError) as ei:
        a.checkpoint(str(tmp_path / "b.ckpt"))
    assert ei.value.code == -6
    # a context that already has species
    with pytest.raises(GlecsimError) as ei:
        a.restore(str(path))
    assert ei.value.code == -6
    a.close()
    # other parameters
    c = H.make_bare_sim(wl, beta_lim=1.0)
    with pytest.raises(GlecsimError) as ei:
        c.restore(str(path))
    assert ei.value.code == -1 and "differ" in str(ei.value)
    c.close()
    # a flipped byte and a truncated file
    raw = bytearray(path.read_bytes())
    raw[len(raw) // 2] ^= 0x40
    (tmp_path / "bad.ckpt").write_bytes(bytes(raw))
    (tmp_path / "short.ckpt").write_bytes(path.read_bytes()[:-100])
    for bad in ["bad.ckpt", "short.ckpt", "missing.ckpt"]:
        d = H.make_bare_sim(wl)
        with pytest.raises(GlecsimError) as ei:
            d.restore(str(tmp_path / bad))
        assert ei.value.code == -1, bad
        d.close()


@pytest.mark.parametrize("dim,n,base", [(2, (7, 5, 1), "c2"), (3, (5, 4, 3), "c5")])
def test_picard_limiter_matches_oracle(dim, n, base):
    from paper_2506_11320_amd import GE_PICARD1
    print(f"[gpu] picard limiter {dim}d", flush=True)
    wl = synth.small("picard", dim=dim, n=n, ppc=20, base=base, fp32=False).replace(
        lf_E=True, lf_B=True, comoving=True, beta_lim=1.5)
    parts = H.species_arrays(wl, False)
    E, B = H.perturbed_fields(wl)
    G, sp = H.oracle_species(wl, parts)
    r = O.step(G, sp, E, B, dt=wl.dt, theta=wl.theta, comoving=True, lf_E=True, lf_B=True, beta_lim=1.5,
               a_mode=wl.a_mode, solve="dense", limiter_lag="picard1")
    lag = O.step(G, sp, E, B, dt=wl.dt, theta=wl.theta, comoving=True, lf_E=True, lf_B=True, beta_lim=1.5,
                 a_mode=wl.a_mode, solve="dense")
    sim = H.make_sim(wl, parts, E, B, limiter_lag=GE_PICARD1)
    sim.deposit()
    rep = sim.solve(tol=1e-13, maxit=4000, restart=40)
    assert rep["converged"]
    Eth = sim.gather("Eth").cpu().numpy()
    assert H.relerr(Eth, r["Eth"]) < 1e-10
    assert H.relerr(Eth, lag["Eth"]) > 1e-9  # the Picard step changes the answer
    assert H.relerr(sim.gather("kappa_E").cpu().numpy(), r["kE"]) < 1e-10
    sim.push()
    sim.update_fields()
    assert H.relerr(sim.gather("E").cpu().numpy(), r["E"]) < 1e-10
    assert H.relerr(sim.gather("B").cpu().numpy(), r["B"]) < 1e-10
    sim.close()
