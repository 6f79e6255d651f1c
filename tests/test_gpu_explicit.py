"""The explicit-PIC current (Sec. 3.1, explicit form) on the GPU path against
the oracle, on seeded synthetic inputs (1e-10 FP64, 1e-5 FP32 relative), and
the state rule that the implicit solve needs a new deposit afterwards."""
import numpy as np
import pytest

import oracle as O
import synth
from tests import harness as H

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [
    ("1d_fp64", 1, (13, 1, 1), 70, "c1", False),
    ("2d_fp32", 2, (7, 5, 1), 70, "c3", True),
    ("3d_fp64", 3, (5, 3, 3), 70, "c5", False),
    ("3d_fp32", 3, (5, 4, 3), 70, "c5", True),
]


def _wl(dim, n, ppc, base, fp32):
    wl = synth.small("expl", dim=dim, n=n, ppc=ppc, base=base, fp32=fp32)
    return wl.replace(dx=(0.5, 1, 1)) if dim == 1 else wl


@pytest.mark.parametrize("ns_j", [0, 2])
@pytest.mark.parametrize("comoving", [True, False])
@pytest.mark.parametrize("name,dim,n,ppc,base,fp32", CASES)
def test_explicit_current_matches_oracle(name, dim, n, ppc, base, fp32, comoving, ns_j):
    print(f"[gpu] explicit current {name} comoving={comoving} ns_j={ns_j}", flush=True)
    wl = _wl(dim, n, ppc, base, fp32)
    parts = H.species_arrays(wl, fp32)
    E, B = H.perturbed_fields(wl)
    G, sp = H.oracle_species(wl, parts)
    ref = O.explicit_current(G, sp, comoving, n_smooth_u=wl.n_smooth_u, n_smooth_j=ns_j)
    sim = H.make_sim(wl, parts, E, B, comoving=comoving, ns_j=ns_j)
    J = sim.explicit_current().cpu().numpy()
    assert H.relerr(J, ref) < (1e-5 if fp32 else 1e-10)
    assert np.array_equal(sim.gather("J_eff").cpu().numpy(), J)
    sim.close()


def test_explicit_current_then_implicit_step_needs_a_new_deposit():
    print("[gpu] explicit current state rule", flush=True)
    from paper_2506_11320_amd import GlecsimError
    wl = _wl(2, (6, 5, 1), 30, "c2", False)
    parts = H.species_arrays(wl, False)
    E, B = H.perturbed_fields(wl)
    sim = H.make_sim(wl, parts, E, B)
    sim.explicit_current()
    with pytest.raises(GlecsimError):
        sim.solve(tol=1e-10)
    # a full step afterwards is the same as on a fresh context
    sim.step(tol=1e-12, maxit=500, restart=30)
    ref = H.make_sim(wl, parts, E, B)
    ref.step(tol=1e-12, maxit=500, restart=30)
    for f in ("E", "B"):
        assert np.array_equal(sim.gather(f).cpu().numpy(), ref.gather(f).cpu().numpy())
    sim.close()
    ref.close()
