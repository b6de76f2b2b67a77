"""Plain FP64 reference of the proposal network: 3D convolutions, their gradients, the
network and its training loss.

TEST INFRASTRUCTURE ONLY (see the package docstring). NumPy in float64, loops over the 27
taps written out; no blocking or fusion.

The proposal network reads the adjoint of the residual, scaled like the certificate
(x = Phi^T r / lambda, the quantity whose correlation with an atom is eta in section 1.2), and
predicts where the next atom of Algorithms 1 and 2 (step 1) lies and its (sigma, d): four 3x3x3
convolutions with 32 channels, the first of stride 2, ReLU between them; output channels are a
centre heatmap logit, sigma and d on the half-resolution grid. The paper has no such network
(it takes the grid maximum); its layer sizes follow the project's target, and everything about
it here is a reading listed in the design notes.

Conventions:
  * activations are ``[C][Z][Y][X]``; weights ``[C_out][C_in][3][3][3]`` indexed
    ``[co][ci][tz][ty][tx]``; biases ``[C_out]``;
  * a convolution with stride s maps input voxel ``s * o + t - 1`` (t in {0, 1, 2} per axis,
    zero outside the volume) to output voxel o, which runs over ``ceil(n / s)`` per axis:
    y[co][o] = b[co] + sum_{ci, t} w[co][ci][t] x[ci][s o + t - 1]
    (a cross-correlation, as in ``scipy.ndimage.correlate`` with zero padding for s = 1);
  * half-resolution voxel o sits at full-resolution position 2 o.

Pins (tests/test_oracle_cnn.py): single-channel stride 1 equals ``ndimage.correlate``; stride 2
equals stride 1 subsampled; the data gradient is the exact adjoint; weight and bias gradients
and the loss gradient match central differences.
"""
from __future__ import annotations

import numpy as np

HEAT_SIGMA = 1.0  # width of a target blob, half-resolution voxels
NEAR = 1.0  # sigma and d are fitted within this distance of a centre (half-resolution voxels)


def out_shape(shape, stride):
    """Spatial output shape of a stride-s convolution: ceil(n / s) per axis."""
    return tuple((n + stride - 1) // stride for n in shape)


def _window(x, t, stride, oshape):
    """x[:, s o + t - 1] for every output voxel o (zero outside), t = (tz, ty, tx)."""
    C = x.shape[0]
    out = np.zeros((C,) + oshape)
    idx = []
    for a in range(3):
        o = np.arange(oshape[a])
        src = stride * o + t[a] - 1
        ok = (src >= 0) & (src < x.shape[1 + a])
        idx.append((o[ok], src[ok]))
    (oz, sz), (oy, sy), (ox, sx) = idx
    out[np.ix_(np.arange(C), oz, oy, ox)] = x[np.ix_(np.arange(C), sz, sy, sx)]
    return out


def conv3d(x, w, b, stride=1):
    """The convolution of the module docstring."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    oshape = out_shape(x.shape[1:], stride)
    y = np.zeros((w.shape[0],) + oshape) + np.asarray(b, dtype=np.float64)[:, None, None, None]
    for tz in range(3):
        for ty in range(3):
            for tx in range(3):
                xw = _window(x, (tz, ty, tx), stride, oshape)  # [ci][o]
                y += np.einsum("oc,czyx->ozyx", w[:, :, tz, ty, tx], xw)
    return y


def conv3d_backward(x, w, dy, stride=1):
    """Gradients of <dy, conv3d(x, w, b)>: (dx, dw, db)."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    dy = np.asarray(dy, dtype=np.float64)
    oshape = dy.shape[1:]
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    for tz in range(3):
        for ty in range(3):
            for tx in range(3):
                t = (tz, ty, tx)
                xw = _window(x, t, stride, oshape)
                dw[:, :, tz, ty, tx] = np.einsum("ozyx,czyx->oc", dy, xw)
                # scatter w^T dy back to the input voxels s o + t - 1
                g = np.einsum("oc,ozyx->czyx", w[:, :, tz, ty, tx], dy)
                idx = []
                for a in range(3):
                    o = np.arange(oshape[a])
                    src = stride * o + t[a] - 1
                    ok = (src >= 0) & (src < x.shape[1 + a])
                    idx.append((o[ok], src[ok]))
                (oz, sz), (oy, sy), (ox, sx) = idx
                C = x.shape[0]
                dx[np.ix_(np.arange(C), sz, sy, sx)] += g[np.ix_(np.arange(C), oz, oy, ox)]
    db = dy.sum(axis=(1, 2, 3))
    return dx, dw, db


def relu(v):
    return np.maximum(v, 0.0)


def init_params(rng, channels=32, n_in=1, n_out=3):
    """He-initialised weights of the four layers (zero biases)."""
    dims = [(channels, n_in), (channels, channels), (channels, channels), (n_out, channels)]
    params = []
    for co, ci in dims:
        std = np.sqrt(2.0 / (27 * ci))
        params.append((rng.standard_normal((co, ci, 3, 3, 3)) * std, np.zeros(co)))
    return params


STRIDES = (2, 1, 1, 1)


def forward(params, x):
    """Network output [3][Z'][Y'][X'] for input x [1][Z][Y][X], with the cached activations."""
    acts = [np.asarray(x, dtype=np.float64)]
    pre = []
    h = acts[0]
    for i, ((w, b), s) in enumerate(zip(params, STRIDES)):
        z = conv3d(h, w, b, s)
        pre.append(z)
        h = relu(z) if i < len(params) - 1 else z
        acts.append(h)
    return h, (acts, pre)


def backward(params, cache, dout):
    """Parameter gradients [(dw, db)] of <dout, forward(params, x)>."""
    acts, pre = cache
    grads = [None] * len(params)
    g = np.asarray(dout, dtype=np.float64)
    for i in range(len(params) - 1, -1, -1):
        if i < len(params) - 1:
            g = g * (pre[i] > 0)
        dx, dw, db = conv3d_backward(acts[i], params[i][0], g, STRIDES[i])
        grads[i] = (dw, db)
        g = dx
    return grads


def targets(oshape, atoms):
    """Targets on the half-resolution grid for the atoms still to be found ([k][6] rows
    (w, mx, my, mz, sigma, d), full-resolution centres): heatmap T(o) = max_j exp(-|o - m_j/2|^2
    / (2 HEAT_SIGMA^2)); mask M(o) = 1 within NEAR of the nearest centre, where sigma and d of
    that atom are the targets S(o), D(o)."""
    Z, Y, X = oshape
    oz, oy, ox = np.meshgrid(np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    T = np.zeros(oshape)
    best = np.full(oshape, np.inf)
    S = np.zeros(oshape)
    D = np.zeros(oshape)
    for a in np.asarray(atoms, dtype=np.float64):
        d2 = (ox - a[1] / 2) ** 2 + (oy - a[2] / 2) ** 2 + (oz - a[3] / 2) ** 2
        T = np.maximum(T, np.exp(-d2 / (2 * HEAT_SIGMA ** 2)))
        closer = d2 < best
        best = np.where(closer, d2, best)
        S = np.where(closer, a[4], S)
        D = np.where(closer, a[5], D)
    M = (best <= NEAR ** 2).astype(np.float64)
    return T, M, S, D


def loss(out, atoms):
    """L = (1 / V') sum_o [(h - T)^2 + M ((sigma_hat - S)^2 + (d_hat - D)^2)] over the V'
    half-resolution voxels, and dL/dout."""
    out = np.asarray(out, dtype=np.float64)
    T, M, S, D = targets(out.shape[1:], atoms)
    V = out[0].size
    r0, r1, r2 = out[0] - T, out[1] - S, out[2] - D
    L = (np.sum(r0 ** 2) + np.sum(M * (r1 ** 2 + r2 ** 2))) / V
    g = np.stack([2 * r0, 2 * M * r1, 2 * M * r2]) / V
    return L, g
