"""FP64 NumPy reference of the small convolutional preconditioner network
(test infrastructure only, shares no code with the GPU library).

Network: L convolution layers with kernel 3 (3x3 in 2D, 3x3x3 in 3D),
'same' zero padding, bias, ReLU between layers (none after the last).
Activations are channels-last arrays [batch, (z,) y, x, channels].

Parameter layout (flat vector, per layer l): W_l[tap][c_in][c_out] followed
by b_l[c_out]; taps are ordered with the offset along x fastest, then y, then
z, each offset in (-1, 0, +1):
    tap = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)       (3D)
    tap = (dy + 1) * 3 + (dx + 1)                      (2D)
and out[p] = b + sum_tap sum_ci x[p + offset(tap)][ci] W[tap][ci][:].

Loss: mean squared error over all entries (inputs and targets are already
normalised by the residual scale):
    L = (1/N) sum (y - e)^2,  N = batch * points * channels
"""
from __future__ import annotations

import numpy as np


def offsets(dim):
    out = []
    rng = (-1, 0, 1)
    if dim == 2:
        for dy in rng:
            for dx in rng:
                out.append((0, dy, dx))
    else:
        for dz in rng:
            for dy in rng:
                for dx in rng:
                    out.append((dz, dy, dx))
    return out


def unflatten(params, dim, channels):
    """Split the flat parameter vector into [(W, b), ...]."""
    taps = 9 if dim == 2 else 27
    layers, o = [], 0
    for ci, co in zip(channels[:-1], channels[1:]):
        W = np.asarray(params[o:o + taps * ci * co], dtype=np.float64).reshape(taps, ci, co)
        o += taps * ci * co
        b = np.asarray(params[o:o + co], dtype=np.float64)
        o += co
        layers.append((W, b))
    assert o == len(params)
    return layers


def n_params(dim, channels):
    taps = 9 if dim == 2 else 27
    return sum(taps * ci * co + co for ci, co in zip(channels[:-1], channels[1:]))


def _shift(x, off, dim):
    """y[p] = x[p + off] with zeros outside (x: [B, Z, Y, X, C])."""
    y = np.zeros_like(x)
    dz, dy, dx = off
    Z, Y, X = x.shape[1:4]

    def sl(d, n):
        # destination and source slices along one axis
        if d >= 0:
            return slice(0, n - d), slice(d, n)
        return slice(-d, n), slice(0, n + d)

    (zd, zs), (yd, ys), (xd, xs) = sl(dz, Z), sl(dy, Y), sl(dx, X)
    y[:, zd, yd, xd, :] = x[:, zs, ys, xs, :]
    return y


def _as5(x, dim):
    return x[:, None] if dim == 2 else x


def conv(x, W, b, dim):
    """'same' convolution (cross-correlation) of x [B, (Z,) Y, X, Cin]."""
    x5 = _as5(np.asarray(x, dtype=np.float64), dim)
    out = np.zeros(x5.shape[:4] + (W.shape[2],))
    for t, off in enumerate(offsets(dim)):
        out += _shift(x5, off, dim) @ W[t]
    out += b
    return out[:, 0] if dim == 2 else out


def forward(x, params, dim, channels):
    """Returns the list of activations [x, a_1, ..., a_{L-1}, y]."""
    acts = [np.asarray(x, dtype=np.float64)]
    layers = unflatten(params, dim, channels)
    for l, (W, b) in enumerate(layers):
        z = conv(acts[-1], W, b, dim)
        if l < len(layers) - 1:
            z = np.maximum(z, 0.0)
        acts.append(z)
    return acts


def loss(y, e):
    y = np.asarray(y, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    return float(np.mean((y - e) ** 2))


def loss_grad(y, e):
    y = np.asarray(y, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    return 2.0 * (y - e) / y.size


def backward(x, params, dim, channels, dy):
    """Gradient of sum(dy * y) with respect to the flat parameters and x,
    by the adjoint convolutions written out (no automatic differentiation)."""
    layers = unflatten(params, dim, channels)
    acts = forward(x, params, dim, channels)
    offs = offsets(dim)
    grads = []
    dz = np.asarray(dy, dtype=np.float64)
    for l in range(len(layers) - 1, -1, -1):
        W, b = layers[l]
        a5 = _as5(acts[l], dim)
        dz5 = _as5(dz, dim)
        Cin, Cout = W.shape[1], W.shape[2]
        dW = np.zeros_like(W)
        for t, off in enumerate(offs):
            sh = _shift(a5, off, dim).reshape(-1, Cin)
            dW[t] = sh.T @ dz5.reshape(-1, Cout)
        db = dz5.reshape(-1, Cout).sum(0)
        grads.append((dW, db))
        # gradient w.r.t. the layer input: adjoint of the shift is the
        # opposite shift
        da5 = np.zeros(a5.shape)
        for t, off in enumerate(offs):
            neg = (-off[0], -off[1], -off[2])
            da5 += _shift(dz5 @ W[t].T, neg, dim)
        da = da5[:, 0] if dim == 2 else da5
        if l > 0:
            dz = da * (acts[l] > 0.0)
        else:
            dx = da
    flat = []
    for dW, db in reversed(grads):
        flat.append(dW.reshape(-1))
        flat.append(db)
    return np.concatenate(flat), dx
