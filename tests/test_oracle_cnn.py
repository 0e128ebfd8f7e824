"""Pins of the CPU CNN reference: forward against scipy.signal.correlate
(an independent library convolution) and the analytic backward against
central finite differences."""
import numpy as np
import pytest
from scipy import signal

from oracle import cnn_ref


@pytest.mark.parametrize("dim", [2, 3])
def test_conv_matches_scipy_correlate(dim):
    rng = np.random.default_rng(0)
    shape = (5, 7) if dim == 2 else (4, 5, 6)
    Cin, Cout = 3, 2
    x = rng.standard_normal((2,) + shape + (Cin,))
    taps = 9 if dim == 2 else 27
    W = rng.standard_normal((taps, Cin, Cout))
    b = rng.standard_normal(Cout)
    got = cnn_ref.conv(x, W, b, dim)
    # scipy: kernel array indexed by (dz,) dy, dx + 1
    for s in range(2):
        for co in range(Cout):
            ref = np.full(shape, b[co])
            for ci in range(Cin):
                k = W[:, ci, co].reshape((3, 3) if dim == 2 else (3, 3, 3))
                ref = ref + signal.correlate(x[s, ..., ci], k, mode="same")
            assert np.abs(got[s, ..., co] - ref).max() <= 1e-12


@pytest.mark.parametrize("dim,channels", [(2, (3, 4, 4, 2)), (3, (4, 3, 3))])
def test_backward_matches_finite_differences(dim, channels):
    rng = np.random.default_rng(1)
    shape = (6, 5) if dim == 2 else (4, 3, 5)
    x = rng.standard_normal((2,) + shape + (channels[0],))
    P = cnn_ref.n_params(dim, channels)
    params = rng.standard_normal(P) * 0.5
    e = rng.standard_normal((2,) + shape + (channels[-1],))

    def L(pv, xv):
        return cnn_ref.loss(cnn_ref.forward(xv, pv, dim, channels)[-1], e)

    y = cnn_ref.forward(x, params, dim, channels)[-1]
    dy = cnn_ref.loss_grad(y, e)
    g, gx = cnn_ref.backward(x, params, dim, channels, dy)
    h = 1e-6
    idx = rng.choice(P, size=min(P, 40), replace=False)
    for i in idx:
        pp, pm = params.copy(), params.copy()
        pp[i] += h
        pm[i] -= h
        fd = (L(pp, x) - L(pm, x)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)) + 1e-8, (i, fd, g[i])
    flat = x.reshape(-1)
    for i in rng.choice(flat.size, size=20, replace=False):
        xp, xm = flat.copy(), flat.copy()
        xp[i] += h
        xm[i] -= h
        fd = (L(params, xp.reshape(x.shape)) - L(params, xm.reshape(x.shape))) / (2 * h)
        assert abs(fd - gx.reshape(-1)[i]) <= 1e-7 * max(1.0, abs(fd)) + 1e-8


def test_loss_grad_is_derivative_of_loss():
    rng = np.random.default_rng(2)
    y = rng.standard_normal((3, 4, 4, 2))
    e = rng.standard_normal((3, 4, 4, 2))
    g = cnn_ref.loss_grad(y, e)
    h = 1e-6
    for i in rng.choice(y.size, size=10, replace=False):
        yp, ym = y.reshape(-1).copy(), y.reshape(-1).copy()
        yp[i] += h
        ym[i] -= h
        fd = (cnn_ref.loss(yp.reshape(y.shape), e) - cnn_ref.loss(ym.reshape(y.shape), e)) / (2 * h)
        assert abs(fd - g.reshape(-1)[i]) <= 1e-8
