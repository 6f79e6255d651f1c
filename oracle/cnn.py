"""FP64 reference of the learned preconditioner z = N(r) (test infrastructure).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: plain numpy in double
precision, used by the tests and the benchmark's reporting; the product path
never imports it and it shares no code with the GPU library.

The network is not part of the paper's method: the paper solves the implicit
field system (Sec. 2.1, with the mass-matrix term of Sec. 3.1) by a Krylov
method and says nothing of how.  Here a learned right preconditioner is tried
inside flexible GMRES; the GMRES residual decides convergence, so the network
can only change the iteration count, never the converged field.

Definition (readings stated once here and used everywhere):
  * Three 3x3x3 convolutions, 3 -> 32 -> 32 -> 3 channels, ReLU after the
    first two, no bias terms, so N(s r) = s N(r) for s > 0.
  * Weights of layer l are W_l[t][co][ci] with tap t = tx + 3 ty + 9 tz,
    tx, ty, tz in {0, 1, 2}; flat weight vector = the three layers
    concatenated (27*(3*32 + 32*32 + 32*3) = 32832 numbers).
  * Whole-grid (periodic) layer: out[co](x) = sum_t sum_ci W[t][co][ci] in[ci](x + t - 1),
    indices wrapping on every axis; grid arrays are [c][N] with the linear
    node index i + nx (j + ny k).
  * Training crops (valid geometry): input box (n+6)^3, output box n^3; output
    node o reads input node o + t, so after three layers output node o sits
    on input node o + 3.  Loss = mean over crops, nodes and the 3 channels of
    (N(r) - e)^2.
  * The GPU runs BF16 operands with FP32 accumulation.  ``quant=True`` makes
    this reference round the same tensors to BF16 (round to nearest even,
    through FP32) at the same places: the scaled input, the weights, the
    activations after each ReLU, and in the backward pass dL/dz (formed in
    FP32 as the GPU does) and the two data gradients; all sums stay in FP64.
    Where the GPU's FP32 sum and the FP64 sum fall on different sides of a
    BF16 rounding boundary the two round differently (a rare one-ulp flip);
    with dyadic inputs and weights whose sums are exact in FP32 no flip can
    happen and the forward pass agrees bit for bit.

Parity: pinned in tests by scipy's periodic correlation, the identity
structure of the initial weights, positive homogeneity, translation
equivariance and central finite differences of the loss.
"""
from __future__ import annotations

import numpy as np

LAYERS = [(3, 32), (32, 32), (32, 3)]  # (cin, cout)
NW = sum(27 * ci * co for ci, co in LAYERS)
CENTRE = 13  # tap (1, 1, 1)


def split(w):
    """Flat weights -> [W1, W2, W3], W_l of shape [27, cout, cin]."""
    w = np.asarray(w, dtype=np.float64)
    assert w.shape == (NW,)
    out, o = [], 0
    for ci, co in LAYERS:
        out.append(w[o:o + 27 * ci * co].reshape(27, co, ci))
        o += 27 * ci * co
    return out


def bf16(x):
    """Round to BF16 (round to nearest even) through FP32; returns float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def taps():
    for t in range(27):
        yield t, t % 3, (t // 3) % 3, t // 9


def conv_periodic(x, W):
    """x [cin, nz, ny, nx] -> [cout, nz, ny, nx], periodic, centred taps."""
    out = np.zeros((W.shape[1],) + x.shape[1:])
    for t, tx, ty, tz in taps():
        shifted = np.roll(x, shift=(-(tz - 1), -(ty - 1), -(tx - 1)), axis=(1, 2, 3))
        out += np.einsum("oc,czyx->ozyx", W[t], shifted)
    return out


def conv_valid(x, W):
    """x [B, cin, m, m, m] -> [B, cout, m-2, m-2, m-2]: out(o) = sum_t W[t] x(o + t)."""
    m = x.shape[-1]
    k = m - 2
    out = np.zeros((x.shape[0], W.shape[1], k, k, k))
    for t, tx, ty, tz in taps():
        out += np.einsum("oc,bczyx->bozyx", W[t], x[:, :, tz:tz + k, ty:ty + k, tx:tx + k])
    return out


def conv_valid_adjoint(d, W):
    """Adjoint of conv_valid: d [B, cout, k, k, k] -> [B, cin, k+2, k+2, k+2]."""
    k = d.shape[-1]
    out = np.zeros((d.shape[0], W.shape[2], k + 2, k + 2, k + 2))
    for t, tx, ty, tz in taps():
        out[:, :, tz:tz + k, ty:ty + k, tx:tx + k] += np.einsum("oc,bozyx->bczyx", W[t], d)
    return out


def weight_grad(x, d):
    """dL/dW[t][co][ci] = sum_{b,o} d[b,co](o) x[b,ci](o + t) for conv_valid."""
    k = d.shape[-1]
    g = np.zeros((27, d.shape[1], x.shape[1]))
    for t, tx, ty, tz in taps():
        g[t] = np.einsum("bozyx,bczyx->oc", d, x[:, :, tz:tz + k, ty:ty + k, tx:tx + k])
    return g


def grid_to_chw(v, n):
    """[3][N] (x fastest) -> [3, nz, ny, nx]."""
    nx, ny, nz = n
    return np.asarray(v, dtype=np.float64).reshape(3, nz, ny, nx)


def forward_grid(w, r, n, scale=1.0, quant=False):
    """z = N(r) on the whole periodic grid: r [3][N] -> z [3][N].

    The input is multiplied by ``scale`` before the network and the output
    divided by it (the GPU normalises the input to unit RMS that way)."""
    W = split(w)
    q = bf16 if quant else (lambda a: a)
    W = [q(Wl) for Wl in W]
    x = q(grid_to_chw(r, n) * scale)
    a1 = q(np.maximum(conv_periodic(x, W[0]), 0.0))
    a2 = q(np.maximum(conv_periodic(a1, W[1]), 0.0))
    z = conv_periodic(a2, W[2])
    if quant:
        z = z.astype(np.float32).astype(np.float64)  # the GPU stores the last layer in FP32
    return (z / scale).reshape(3, -1)


def forward_apply(w, r, n, quant=False):
    """What the library's whole-grid application computes: r normalised to unit RMS."""
    r = np.asarray(r, dtype=np.float64)
    rms = np.sqrt(np.mean(r * r))
    return forward_grid(w, r, n, 1.0 / rms if rms > 0 else 1.0, quant)


def loss_grad(w, in_crops, tgt, quant=False):
    """Loss and flat gradient for crops.

    in_crops [B, (n+6)^3, 3], tgt [B, n^3, 3], both crop-local with x fastest.
    Returns (loss, grad[NW]).  With quant=True the BF16 roundings of the GPU
    are applied (see the module header)."""
    in_crops = np.asarray(in_crops, dtype=np.float64)
    tgt = np.asarray(tgt, dtype=np.float64)
    B, v6, _ = in_crops.shape
    m = round(v6 ** (1 / 3))
    n = m - 6
    assert m ** 3 == v6 and tgt.shape == (B, n ** 3, 3)
    q = bf16 if quant else (lambda a: a)
    W = [q(Wl) for Wl in split(w)]
    x = q(in_crops.reshape(B, m, m, m, 3).transpose(0, 4, 1, 2, 3))
    e = tgt.reshape(B, n, n, n, 3).transpose(0, 4, 1, 2, 3)
    p1 = conv_valid(x, W[0])
    a1 = q(np.maximum(p1, 0.0))
    p2 = conv_valid(a1, W[1])
    a2 = q(np.maximum(p2, 0.0))
    z = conv_valid(a2, W[2])
    if quant:
        z = z.astype(np.float32).astype(np.float64)
    cnt = 3.0 * B * n ** 3
    diff = z - e
    loss = float(np.sum(diff * diff) / cnt)
    if quant:
        # the GPU forms dL/dz in FP32 as (2/cnt) * (z - e) before rounding to
        # BF16; the same FP32 operations here make both sides round the same value
        s32 = np.float32(2.0) / np.float32(cnt)
        dz = q((s32 * (z.astype(np.float32) - e.astype(np.float32))).astype(np.float64))
    else:
        dz = 2.0 * diff / cnt
    g3 = weight_grad(a2, dz)
    d2 = q(conv_valid_adjoint(dz, W[2]) * (a2 > 0))
    g2 = weight_grad(a1, d2)
    d1 = q(conv_valid_adjoint(d2, W[1]) * (a1 > 0))
    g1 = weight_grad(x, d1)
    return loss, np.concatenate([g1.ravel(), g2.ravel(), g3.ravel()])


def identity_weights():
    """Weights with N(r) = r exactly: layer 1 splits each component x_i into
    the channel pair (+x_i, -x_i), layer 2 passes the pairs through the ReLU
    unchanged, layer 3 recombines x_i = relu(x_i) - relu(-x_i); centre taps only."""
    W1 = np.zeros((27, 32, 3))
    W2 = np.zeros((27, 32, 32))
    W3 = np.zeros((27, 3, 32))
    for i in range(3):
        W1[CENTRE, 2 * i, i] = 1.0
        W1[CENTRE, 2 * i + 1, i] = -1.0
        for j in (0, 1):
            W2[CENTRE, 2 * i + j, 2 * i + j] = 1.0
        W3[CENTRE, i, 2 * i] = 1.0
        W3[CENTRE, i, 2 * i + 1] = -1.0
    return np.concatenate([W1.ravel(), W2.ravel(), W3.ravel()])
