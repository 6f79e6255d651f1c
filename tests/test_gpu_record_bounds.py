"""FP64 particle records at buffer sizes that are whole multiples of the
allocation granularity.  A record is 56 bytes in FP64; a read that reaches
past the record's last byte reaches past the buffer at its last record, which
faults exactly when the buffer ends on a mapping boundary.  4 194 304
particles per species (64x32x32 cells, 64 per cell) make each buffer exactly
224 MiB.  Every kernel that reads records runs here on such buffers: the
deposit, the push, the explicit-current passes, the read-back and the
moment diagnostics; the FP64 results are checked against the FP32 path on the
same (rounded) particles to the FP32 tolerance."""
import numpy as np
import pytest

import synth
from tests import harness as H

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_fp64_3d_records_ending_on_a_2mib_boundary():
    n, ppc = (64, 32, 32), 64
    print(f"[gpu] FP64 3D records, grid {n}, {ppc} per cell and species", flush=True)
    wl = synth.small("bounds", dim=3, n=n, ppc=ppc, base="c5", fp32=False)
    nper = n[0] * n[1] * n[2] * ppc
    assert nper * 7 * 8 == 224 * 2 ** 20
    E, B = H.perturbed_fields(wl)
    out = {}
    for f32 in (False, True):
        w = wl.replace(fp32=f32)
        parts = H.species_arrays(w, f32)
        assert all(p["cell"].size == nper for p in parts)
        sim = H.make_sim(w, parts, E, B)
        sim.deposit()
        out[f32] = {k: sim.gather(k).cpu().numpy() for k in ("Mt", "M0", "J_lab", "J_eff", "rho", "mm")}
        sim.close()
    for k in out[False]:
        assert _rel(out[True][k], out[False][k]) < 1e-5, k
    # the other record readers on FP64 buffers of the same size
    parts = H.species_arrays(wl, False)
    sim = H.make_sim(wl, parts, E, B)
    d = sim.diagnostics()
    K0 = sum(0.5 * wl.m[s] * np.sum(p["w"] * np.sum(p["v"] ** 2, axis=0)) for s, p in enumerate(parts))
    assert abs(sum(d["K"]) - K0) <= 1e-12 * K0
    got = sim.particles(1)
    assert np.array_equal(got["v"].cpu().numpy(), parts[1]["v"])
    J = sim.explicit_current().cpu().numpy()
    assert np.isfinite(J).all() and np.abs(J).max() > 0
    rep = sim.step(tol=1e-8, maxit=500, restart=30)
    assert rep["converged"]
    assert sum(sim.particles(s)["cell"].numel() for s in range(2)) == 2 * nper
    sim.explicit_step()
    assert np.isfinite(sim.gather("E").cpu().numpy()).all()
    sim.close()
