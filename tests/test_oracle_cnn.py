"""Pins of the proposal network's FP64 reference (oracle/cnn.py), on the CPU.

A single-channel stride-1 convolution is scipy.ndimage.correlate with zero padding; stride 2
is stride 1 subsampled; the data gradient is the exact adjoint; weight, bias and whole-network
gradients match central differences (the network is piecewise linear in its weights, so the
differences are exact away from ReLU kinks); the loss gradient matches central differences.
"""
import numpy as np
import pytest
from scipy import ndimage

from oracle import cnn


def _rng(seed):
    return np.random.default_rng(seed)


@pytest.mark.parametrize("shape", [(5, 6, 7), (1, 4, 9)])
def test_single_channel_is_ndimage_correlate(shape):
    rng = _rng(1)
    x = rng.standard_normal(shape)
    w = rng.standard_normal((1, 1, 3, 3, 3))
    y = cnn.conv3d(x[None], w, np.array([0.25]), 1)[0]
    want = ndimage.correlate(x, w[0, 0], mode="constant", cval=0.0) + 0.25
    assert np.max(np.abs(y - want)) <= 1e-12


@pytest.mark.parametrize("shape", [(6, 7, 8), (5, 5, 3)])
def test_stride_two_is_stride_one_subsampled(shape):
    rng = _rng(2)
    x = rng.standard_normal((3,) + shape)
    w = rng.standard_normal((4, 3, 3, 3, 3))
    b = rng.standard_normal(4)
    full = cnn.conv3d(x, w, b, 1)
    half = cnn.conv3d(x, w, b, 2)
    assert half.shape[1:] == cnn.out_shape(shape, 2)
    assert np.max(np.abs(half - full[:, ::2, ::2, ::2])) <= 1e-12


@pytest.mark.parametrize("stride", [1, 2])
def test_backward_is_adjoint_and_matches_differences(stride):
    rng = _rng(3 + stride)
    x = rng.standard_normal((3, 5, 6, 7))
    w = rng.standard_normal((4, 3, 3, 3, 3))
    b = rng.standard_normal(4)
    y = cnn.conv3d(x, w, b, stride)
    g = rng.standard_normal(y.shape)
    dx, dw, db = cnn.conv3d_backward(x, w, g, stride)
    # <conv(x) - b, g> = <x, dx>: the data gradient is the adjoint
    lin = np.sum((y - b[:, None, None, None]) * g)
    assert abs(lin - np.sum(x * dx)) <= 1e-10 * abs(lin)
    # linear in w and b: central differences along random directions are exact
    E = rng.standard_normal(w.shape)
    h = 1e-3
    fd = (np.sum(cnn.conv3d(x, w + h * E, b, stride) * g) -
          np.sum(cnn.conv3d(x, w - h * E, b, stride) * g)) / (2 * h)
    assert abs(fd - np.sum(dw * E)) <= 1e-9 * max(1.0, abs(fd))
    e = rng.standard_normal(4)
    fdb = (np.sum(cnn.conv3d(x, w, b + h * e, stride) * g) -
           np.sum(cnn.conv3d(x, w, b - h * e, stride) * g)) / (2 * h)
    assert abs(fdb - np.sum(db * e)) <= 1e-9 * max(1.0, abs(fdb))


def test_network_gradient_matches_differences():
    rng = _rng(7)
    params = cnn.init_params(rng, channels=4)
    x = rng.standard_normal((1, 8, 10, 9))
    out, cache = cnn.forward(params, x)
    assert out.shape == (3, 4, 5, 5)
    g = rng.standard_normal(out.shape)
    grads = cnn.backward(params, cache, g)
    h = 1e-6
    for layer in range(4):
        E = rng.standard_normal(params[layer][0].shape)
        plus = [(w + (h * E if i == layer else 0), b) for i, (w, b) in enumerate(params)]
        minus = [(w - (h * E if i == layer else 0), b) for i, (w, b) in enumerate(params)]
        fd = (np.sum(cnn.forward(plus, x)[0] * g) - np.sum(cnn.forward(minus, x)[0] * g)) / (2 * h)
        an = np.sum(grads[layer][0] * E)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), layer


def test_loss_targets_and_gradient():
    rng = _rng(8)
    atoms = np.array([[1.0, 6.0, 4.0, 2.0, 1.3, 2.0], [1.5, 12.4, 9.0, 6.6, 1.8, 1.6]])
    oshape = (5, 7, 8)
    T, M, S, D = cnn.targets(oshape, atoms)
    assert T[1, 2, 3] == pytest.approx(1.0) and M[1, 2, 3] == 1 and S[1, 2, 3] == 1.3
    assert T[3, 4, 6] == pytest.approx(np.exp(-(0.2 ** 2 + 0.5 ** 2 + 0.3 ** 2) / 2))
    assert D[3, 4, 6] == 1.6 and M[0, 0, 0] == 0
    out = rng.standard_normal((3,) + oshape)
    L, g = cnn.loss(out, atoms)
    E = rng.standard_normal(out.shape)
    h = 1e-6
    fd = (cnn.loss(out + h * E, atoms)[0] - cnn.loss(out - h * E, atoms)[0]) / (2 * h)
    assert abs(fd - np.sum(g * E)) <= 1e-7 * max(1.0, abs(fd))
