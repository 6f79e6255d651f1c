"""The allocation-free diagnostics entry point (ge_diagnostics_noalloc),
through the C ABI, against ge_diagnostics: the same kernels and summation
order, so the results must agree bit for bit; two contexts in a row, the
second smaller (the static scratch keeps the first call's contents)."""
import numpy as np
import pytest

import synth
from tests import harness as H

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _case(dim, n, ppc, base, fp32):
    wl = synth.small("noalloc", dim=dim, n=n, ppc=ppc, base=base, fp32=fp32)
    if dim == 1:
        wl = wl.replace(dx=(0.5, 1, 1))
    parts = H.species_arrays(wl, fp32)
    E, B = H.perturbed_fields(wl)
    return wl, H.make_sim(wl, parts, E, B)


def _same(a, b):
    assert a["W_E"] == b["W_E"] and a["W_B"] == b["W_B"] and a["gauss"] == b["gauss"]
    assert a["K"] == b["K"] and a["P"] == b["P"]


def test_noalloc_diagnostics_equal_the_allocating_ones():
    print("[gpu] noalloc diagnostics: large then small", flush=True)
    from paper_2506_11320_amd import GlecsimError
    wl, sim = _case(3, (9, 7, 6), 40, "c5", True)
    sim.step(tol=1e-10, maxit=2000, restart=30)
    a, b = sim.diagnostics(), sim.diagnostics(noalloc=True)
    _same(a, b)
    assert a["W_E"] > 0 and a["W_B"] > 0 and all(k > 0 for k in a["K"])
    # an unsettled push is refused (settling may allocate)
    sim.deposit()
    sim.solve(tol=1e-8, maxit=2000, restart=30)
    sim.push()
    with pytest.raises(GlecsimError) as ei:
        sim.diagnostics(noalloc=True)
    assert ei.value.code == -6
    sim.sync()
    _same(sim.diagnostics(), sim.diagnostics(noalloc=True))
    sim.close()
    # second, smaller input on the same GPU (the scratch holds the first one's sums)
    wl2, sim2 = _case(2, (5, 4, 1), 9, "c2", False)
    sim2.step(tol=1e-10, maxit=2000, restart=30)
    b2 = sim2.diagnostics(noalloc=True)
    a2 = sim2.diagnostics()
    _same(a2, b2)
    assert np.isfinite(b2["gauss"]) and b2["W_B"] > 0
    sim2.close()
