"""The seeded input generator: Philox4x32-10 known answers and the loading
recipe's invariants (it holds no arithmetic of the PIC method)."""
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
