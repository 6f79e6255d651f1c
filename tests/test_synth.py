"""The seeded input generator: Philox4x32-10 known answers and the loading
recipe's invariants (it holds no arithmetic of the PIC method)."""
import os
import numpy as np
import pytest

import synth


def test_philox_known_answers():
    # Known-answer vectors of Philox4x32-10 (Salmon et al., SC'11).
    assert synth.philox4x32_10([0, 0, 0, 0], [0, 0]) == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    assert synth.philox4x32_10([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2) == [0x408F276D, 0x41C83B0E, 0xA20BC7C6,
                                                                       0x6D5451FD]
    assert synth.philox4x32_10([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0]) == [
        0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c4", "c5"])
def test_loading_is_cell_sorted_and_regenerable(name):
    wl = synth.small("t", dim=synth.workloads()[name].dim, n=(5, 4, 3), ppc=3, base=name)
    full = synth.particles(wl, 1)
    assert np.all(np.diff(full["cell"]) >= 0)
    assert np.all(full["off"][: wl.dim] > 0) and np.all(full["off"][: wl.dim] < 1)
    # any range of cells regenerates bit-identically
    cb, ce = 1, min(4, wl.ncells)
    part = synth.particles(wl, 1, cb, ce)
    sl = slice(cb * wl.ppc, ce * wl.ppc)
    for k in ["cell", "w"]:
        assert np.array_equal(part[k], full[k][sl])
    for k in ["off", "v"]:
        assert np.array_equal(part[k], full[k][:, sl])
    # FP32 offsets are the FP64 ones exactly (24-bit grid), and stay < 1
    p32 = synth.particles(wl, 1, f32=True)
    assert np.array_equal(p32["off"].astype(np.float64), full["off"])
    assert np.all(p32["off"][: wl.dim] < 1)


def test_paired_loading_has_equal_positions():
    wl = synth.workloads()["c1"].replace(n=(8, 1, 1), ppc=4)
    e, i = synth.particles(wl, 0), synth.particles(wl, 1)
    assert np.array_equal(e["off"], i["off"])
    assert not np.array_equal(e["v"], i["v"])


def test_maxwellian_moments():
    wl = synth.workloads()["c2"].replace(n=(32, 32, 1), ppc=64)
    p = synth.particles(wl, 0)
    v = p["v"]
    assert abs(v[0].mean() - 0.2) < 3 * 0.02 / np.sqrt(v.shape[1]) * 3
    assert abs(v[1].std() / 0.02 - 1) < 0.02
    assert np.linalg.norm(v - np.array(wl.u0)[:, None], axis=0).max() <= 4.5 * 0.02 + 1e-12


def test_walled_loading_skips_the_ghost_cells():
    """A walled workload stores a ghost cell column along x: no particles in
    it, the same per-range regeneration, and no tangential E on the wall."""
    wl = synth.workloads()["c4"].replace(n=(6, 4, 3), ppc=3)
    assert wl.nstore == (7, 4, 3) and wl.ncells == 84 and wl.nphys == 72
    full = synth.particles(wl, 0)
    assert full["cell"].size == wl.nphys * wl.ppc
    assert np.all(full["cell"] % 7 != 6)
    assert np.all(np.diff(full["cell"]) >= 0)
    part = synth.particles(wl, 0, 5, 20)  # a range across two ghost cells (6 and 13)
    sel = (full["cell"] >= 5) & (full["cell"] < 20)
    assert part["cell"].size == sel.sum() == (15 - 2) * wl.ppc
    assert np.array_equal(part["cell"], full["cell"][sel]) and np.array_equal(part["v"], full["v"][:, sel])
    E, B = synth.fields(wl)
    i = np.arange(wl.ncells) % 7
    assert np.all(E[1:, i == 0] == 0) and np.any(E[2, i == 3] != 0)
    np.testing.assert_allclose(B[:, i == 6], np.array(wl.B0)[:, None] * np.ones((1, 12)))


def test_inflow_injection_flux():
    """The particles entering through x = L: in the last physical cell
    column, inside the slab |u_x| dt next to the plane, and on average
    ppc |u_x| dt / dx per column and step (the flux n |u_x| dt A)."""
    wl = synth.workloads()["c4"].replace(n=(6, 4, 3), ppc=27)
    r = wl.ppc * abs(wl.u0[0]) * wl.dt / wl.dx[0]
    tot = 0
    K = 40
    for k in range(K):
        p = synth.inflow(wl, 1, k)
        tot += p["cell"].size
        if p["cell"].size:
            assert np.all(p["cell"] % 7 == 5)
            assert np.all(p["off"][0] >= 1 - abs(wl.u0[0]) * wl.dt / wl.dx[0]) and np.all(p["off"][0] < 1)
        assert np.array_equal(synth.inflow(wl, 1, k)["v"], p["v"])  # regenerable per step
    ncol = 4 * 3
    assert tot == ncol * int(np.floor(K * r))
    assert abs(tot / (K * ncol) - r) < 1.0 / K


def test_committed_configs_match_the_workloads():
    """configs/<name>.json (written by synth/write_configs.py) records exactly
    what synth.workloads() defines, for every workload."""
    from synth.write_configs import OUT, render
    names = sorted(synth.workloads())
    assert sorted(f[:-5] for f in os.listdir(OUT) if f.endswith(".json")) == names
    for name, wl in synth.workloads().items():
        with open(os.path.join(OUT, f"{name}.json")) as f:
            assert f.read() == render(wl), name
