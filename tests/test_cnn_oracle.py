"""Pins of the FP64 reference of the learned preconditioner (oracle/cnn.py)
against things other than itself: scipy's periodic correlation, the exact
identity map of the structured weights, adjointness, linearity in the
weights, positive homogeneity, translation equivariance, central finite
differences of the loss and known BF16 roundings."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import cnn as C


def _rand_w(rng, scale=1.0):
    parts = []
    for ci, co in C.LAYERS:
        parts.append(rng.standard_normal(27 * ci * co) * scale * np.sqrt(2.0 / (27 * ci)))
    return np.concatenate(parts)


def test_sizes():
    assert C.NW == 32832
    W = C.split(np.arange(C.NW, dtype=float))
    assert [w.shape for w in W] == [(27, 32, 3), (27, 32, 32), (27, 3, 32)]
    assert W[1][0, 0, 0] == 27 * 3 * 32


def test_bf16_rounding_known_values():
    one = 1.0
    vals = np.array([one, one + 2.0 ** -8, one + 3 * 2.0 ** -8, one + 2.0 ** -7, -3.0 - 2.0 ** -7, 0.0, 2.0 ** -130])
    got = C.bf16(vals)
    # ties go to the even mantissa; 1 + 2^-7 is representable; subnormals keep their top bits
    assert got[0] == 1.0
    assert got[1] == 1.0
    assert got[2] == 1.0 + 2.0 ** -6
    assert got[3] == 1.0 + 2.0 ** -7
    assert got[4] == -3.0  # -3 - 2^-7: tie between -3 and -3 - 2^-6 -> even (-3)
    assert got[5] == 0.0
    assert got[6] == 2.0 ** -130
    # relative error bound of round-to-nearest with 8 significant bits
    x = np.random.default_rng(0).standard_normal(10000)
    assert np.max(np.abs(C.bf16(x) - x) / np.abs(x)) <= 2.0 ** -8 * (1 + 1e-12)


def test_periodic_conv_matches_scipy_wrap_correlation():
    rng = np.random.default_rng(1)
    nz, ny, nx = 4, 5, 6
    x = rng.standard_normal((3, nz, ny, nx))
    W = rng.standard_normal((27, 4, 3))
    got = C.conv_periodic(x, W)
    for co in range(4):
        ref = np.zeros((nz, ny, nx))
        for ci in range(3):
            K = np.zeros((3, 3, 3))
            for t in range(27):
                K[t // 9, (t // 3) % 3, t % 3] = W[t, co, ci]
            ref += ndimage.correlate(x[ci], K, mode="wrap")
        assert np.max(np.abs(got[co] - ref)) < 1e-12


def test_valid_conv_is_the_interior_of_the_periodic_conv():
    rng = np.random.default_rng(2)
    m = 7
    x = rng.standard_normal((2, m, m, m))
    W = rng.standard_normal((27, 3, 2))
    per = C.conv_periodic(x, W)
    val = C.conv_valid(x[None], W)[0]
    assert val.shape == (3, m - 2, m - 2, m - 2)
    assert np.max(np.abs(val - per[:, 1:m - 1, 1:m - 1, 1:m - 1])) < 1e-12


def test_adjoint_and_weight_gradient_identities():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 4, 6, 6, 6))
    d = rng.standard_normal((2, 5, 4, 4, 4))
    W = rng.standard_normal((27, 5, 4))
    lhs = np.sum(C.conv_valid(x, W) * d)
    assert abs(lhs - np.sum(x * C.conv_valid_adjoint(d, W))) < 1e-10 * abs(lhs) + 1e-10
    dW = rng.standard_normal(W.shape)
    assert abs(np.sum(C.conv_valid(x, dW) * d) - np.sum(C.weight_grad(x, d) * dW)) < 1e-10 * abs(lhs) + 1e-9


def test_identity_weights_are_the_identity_map():
    rng = np.random.default_rng(4)
    n = (5, 4, 3)
    r = rng.standard_normal((3, n[0] * n[1] * n[2]))
    w = C.identity_weights()
    assert np.array_equal(C.forward_grid(w, r, n), r)
    # with the BF16 roundings the map returns the rounded input
    assert np.array_equal(C.forward_grid(w, r, n, quant=True), C.bf16(r).astype(np.float32).astype(np.float64))
    assert np.allclose(C.forward_apply(w, r, n), r, rtol=0, atol=1e-14)


def test_positive_homogeneity_and_translation_equivariance():
    rng = np.random.default_rng(5)
    n = (6, 5, 4)
    N = n[0] * n[1] * n[2]
    w = _rand_w(rng)
    r = rng.standard_normal((3, N))
    z = C.forward_grid(w, r, n)
    assert np.max(np.abs(C.forward_grid(w, 2.5 * r, n) - 2.5 * z)) < 1e-12 * np.max(np.abs(z))
    # ReLU makes N non-odd: N(-r) != -N(r) in general
    assert np.max(np.abs(C.forward_grid(w, -r, n) + z)) > 1e-3 * np.max(np.abs(z))
    sh = (1, 2, 3)  # (z, y, x) shift
    rs = np.roll(r.reshape(3, n[2], n[1], n[0]), sh, axis=(1, 2, 3)).reshape(3, N)
    zs = np.roll(z.reshape(3, n[2], n[1], n[0]), sh, axis=(1, 2, 3)).reshape(3, N)
    assert np.max(np.abs(C.forward_grid(w, rs, n) - zs)) < 1e-12
    # normalisation by the RMS does not change the answer (homogeneity)
    assert np.max(np.abs(C.forward_apply(w, r, n) - z)) < 1e-12 * np.max(np.abs(z))


def test_loss_gradient_matches_central_differences():
    rng = np.random.default_rng(6)
    B, n = 2, 2
    w = _rand_w(rng)
    x = rng.standard_normal((B, (n + 6) ** 3, 3))
    e = rng.standard_normal((B, n ** 3, 3))
    L, g = C.loss_grad(w, x, e)
    assert L > 0
    h = 1e-6
    offs = [0, 27 * 3 * 32, 27 * 3 * 32 + 27 * 32 * 32, C.NW]
    worst = 0.0
    for l in range(3):
        idx = rng.choice(np.arange(offs[l], offs[l + 1]), size=25, replace=False)
        for i in idx:
            wp = w.copy(); wp[i] += h
            wm = w.copy(); wm[i] -= h
            fd = (C.loss_grad(wp, x, e)[0] - C.loss_grad(wm, x, e)[0]) / (2 * h)
            worst = max(worst, abs(fd - g[i]) / (np.max(np.abs(g[offs[l]:offs[l + 1]])) + 1e-300))
    assert worst < 1e-6, worst


def test_loss_of_crops_equals_grid_forward():
    """A crop cut from a periodic grid, run in the valid geometry, gives the
    whole-grid output at nodes origin + 3 + o."""
    rng = np.random.default_rng(7)
    n = (9, 8, 10)
    N = n[0] * n[1] * n[2]
    w = _rand_w(rng)
    r = rng.standard_normal((3, N))
    z = C.forward_grid(w, r, n).reshape(3, n[2], n[1], n[0])
    rg = r.reshape(3, n[2], n[1], n[0])
    k = 2
    org = (5, 1, 7)  # x, y, z origin of the input crop
    xs = [(org[0] + i) % n[0] for i in range(k + 6)]
    ys = [(org[1] + i) % n[1] for i in range(k + 6)]
    zs = [(org[2] + i) % n[2] for i in range(k + 6)]
    crop = rg[:, zs][:, :, ys][:, :, :, xs]                    # [3, z, y, x]
    tgt = z[:, zs[3:3 + k]][:, :, ys[3:3 + k]][:, :, :, xs[3:3 + k]]
    in_crops = crop.transpose(1, 2, 3, 0).reshape(1, -1, 3)
    t = tgt.transpose(1, 2, 3, 0).reshape(1, -1, 3)
    L, _ = C.loss_grad(w, in_crops, t)
    assert L < 1e-24
