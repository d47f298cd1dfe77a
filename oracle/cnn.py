"""FP64 reference of the learned preconditioning stage (not in the paper: parity unpinned
by the paper; pinned here by finite differences and brute-force convolution).

Network C(r) on one slab residual r of shape (n_t, Nz, Ny, Nx) on the node lattice:
  s   = sqrt(mean(r^2))                      (s = 0 -> C(r) = 0)
  h_0 = r / s                                channels = temporal DoFs
  h_l = relu(conv_l(h_{l-1})), l < L;  h_L = conv_L(h_{L-1})
  C(r) = s * h_L, set to zero on Dirichlet nodes
conv_l(h)[co, v] = b[co] + sum_{tap, ci} W[tap, co, ci] h[ci, v + off(tap)], 3x3x3 taps,
tap = dx + 3 (dy + 3 dz) with offset (dx - 1, dy - 1, dz - 1), zero outside the lattice.
C is positively homogeneous: C(a r) = a C(r) for a > 0.

Parameters are one flat vector: for each layer, W (27 * C_out * C_in, tap-major, then
output channel, then input channel) followed by b (C_out).

Training loss for a pair (r, e): L = ||C(r) - e||^2 / ||e||^2.
"""
from __future__ import annotations

import numpy as np


def param_count(channels):
    return sum(27 * channels[l + 1] * channels[l] + channels[l + 1] for l in range(len(channels) - 1))


def unpack(theta, channels):
    out = []
    o = 0
    for l in range(len(channels) - 1):
        ci, co = channels[l], channels[l + 1]
        W = theta[o:o + 27 * co * ci].reshape(27, co, ci)
        o += 27 * co * ci
        b = theta[o:o + co]
        o += co
        out.append((W, b))
    return out


def init_params(channels, seed: int) -> np.ndarray:
    """He-style initialisation from a seeded PCG64 stream (weights ~ N(0, 2 / (27 C_in)), b = 0)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for l in range(len(channels) - 1):
        ci, co = channels[l], channels[l + 1]
        parts.append(rng.standard_normal(27 * co * ci) * np.sqrt(2.0 / (27 * ci)))
        parts.append(np.zeros(co))
    return np.concatenate(parts)


def _shift(h, dz, dy, dx):
    """h[..., z + dz, y + dy, x + dx] with zeros outside (dz, dy, dx in {-1, 0, 1})."""
    out = np.zeros_like(h)
    Z, Y, X = h.shape[-3:]
    zs = slice(max(0, -dz), Z - max(0, dz))
    ys = slice(max(0, -dy), Y - max(0, dy))
    xs = slice(max(0, -dx), X - max(0, dx))
    zt = slice(max(0, dz), Z - max(0, -dz))
    yt = slice(max(0, dy), Y - max(0, -dy))
    xt = slice(max(0, dx), X - max(0, -dx))
    out[..., zs, ys, xs] = h[..., zt, yt, xt]
    return out


def taps():
    return [(t % 3 - 1, (t // 3) % 3 - 1, t // 9 - 1) for t in range(27)]   # (dx, dy, dz)


def conv(h, W, b):
    """(C_in, Z, Y, X) -> (C_out, Z, Y, X)."""
    out = np.zeros((W.shape[1],) + h.shape[1:])
    for t, (dx, dy, dz) in enumerate(taps()):
        out += np.tensordot(W[t], _shift(h, dz, dy, dx), axes=(1, 0))
    return out + b[:, None, None, None]


def conv_backward(h, W, g):
    """Given input h and upstream gradient g of conv(h): (dW, db, dh)."""
    dW = np.zeros_like(W)
    dh = np.zeros_like(h)
    for t, (dx, dy, dz) in enumerate(taps()):
        sh = _shift(h, dz, dy, dx)
        dW[t] = np.tensordot(g, sh, axes=([1, 2, 3], [1, 2, 3]))
        dh += _shift(np.tensordot(W[t].T, g, axes=(1, 0)), -dz, -dy, -dx)
    db = g.sum(axis=(1, 2, 3))
    return dW, db, dh


def forward(theta, channels, r, bmask=None, keep=False):
    """C(r) for r of shape (n_t, Z, Y, X); bmask (Z, Y, X) True on Dirichlet nodes."""
    s = float(np.sqrt(np.mean(r ** 2)))
    layers = unpack(theta, channels)
    if s == 0.0:
        return (np.zeros_like(r), None) if keep else np.zeros_like(r)
    hs = [r / s]
    for l, (W, b) in enumerate(layers):
        a = conv(hs[-1], W, b)
        if l < len(layers) - 1:
            a = np.maximum(a, 0.0)
        hs.append(a)
    z = s * hs[-1]
    if bmask is not None:
        z[:, bmask] = 0.0
    return (z, (s, hs)) if keep else z


def loss_and_grad(theta, channels, r, e, bmask=None):
    """L = ||C(r) - e||^2 / ||e||^2 and dL/dtheta."""
    z, (s, hs) = forward(theta, channels, r, bmask, keep=True)
    ee = float(np.sum(e ** 2))
    d = z - e
    L = float(np.sum(d ** 2)) / ee
    g = 2.0 * d / ee
    if bmask is not None:
        g[:, bmask] = 0.0
    g = g * s                          # through z = s h_L
    layers = unpack(theta, channels)
    grads = []
    for l in range(len(layers) - 1, -1, -1):
        W, b = layers[l]
        dW, db, dh = conv_backward(hs[l], W, g)
        grads.append((dW, db))
        if l > 0:
            g = dh * (hs[l] > 0)       # relu of layer l-1
    grads = grads[::-1]
    return L, np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])


def output_gradient(theta, channels, r, dz, bmask=None):
    """Gradient of sum(dz * C(r)) with respect to theta (s held fixed)."""
    z, (s, hs) = forward(theta, channels, r, bmask, keep=True)
    g = dz.copy()
    if bmask is not None:
        g[:, bmask] = 0.0
    g = g * s
    layers = unpack(theta, channels)
    grads = []
    for l in range(len(layers) - 1, -1, -1):
        W, b = layers[l]
        dW, db, dh = conv_backward(hs[l], W, g)
        grads.append((dW, db))
        if l > 0:
            g = dh * (hs[l] > 0)
    grads = grads[::-1]
    return np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])


def adam_step(theta, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad ** 2
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------- rounding scales
# Per-element scales of the rounding error of a low-precision evaluation of the same network
# (weights, activations and upstream gradients rounded to a format of unit roundoff u, products
# and sums in a wider format), for element-by-element comparisons.  Rounding errors of different
# terms are independent to first order, so the error of a sum has the scale u times the square
# root of the summed variances of its terms: a term w h contributes w^2 var(h) (error carried in
# h) plus (w h)^2 (rounding of w); each rounded result adds its own square.  Variances propagate
# through the layers like the values do (squared weights acting on variances).  The functions
# return sigma / u.

def _forward_vars(theta, channels, r, bmask):
    z, (s, hs) = forward(theta, channels, r, bmask, keep=True)
    layers = unpack(theta, channels)
    var = [hs[0] ** 2]                                  # rounding of the normalised input
    for l, (W, b) in enumerate(layers):
        zero = np.zeros_like(b)
        v = conv(var[-1], W ** 2, zero) + conv(hs[l] ** 2, W ** 2, zero)
        if l < len(layers) - 1:
            v = v * (hs[l + 1] > 0) + hs[l + 1] ** 2      # relu, then rounding of the activation
        var.append(v)
    return s, hs, var, layers


def forward_rounding_scale(theta, channels, r, bmask=None):
    """sigma(v) / u for every output element of C(r)."""
    s, hs, var, layers = _forward_vars(theta, channels, r, bmask)
    out = s * np.sqrt(var[-1])
    if bmask is not None:
        out[:, bmask] = 0.0
    return out


def output_gradient_rounding_scale(theta, channels, r, dz, bmask=None):
    """sigma / u for every entry of output_gradient (weight gradients sum g h over the lattice,
    bias gradients sum g)."""
    s, hs, hvar, layers = _forward_vars(theta, channels, r, bmask)
    g = dz.copy()
    if bmask is not None:
        g[:, bmask] = 0.0
    g = g * s
    gvar = g ** 2                                       # rounding of the upstream gradient
    out = []
    for l in range(len(layers) - 1, -1, -1):
        W, b = layers[l]
        dW_a, _, _ = conv_backward(hvar[l], W, g ** 2)   # error carried in h
        dW_b, db_v, _ = conv_backward(hs[l] ** 2, W, gvar)   # error carried in g
        out.append((np.sqrt(dW_a + dW_b), np.sqrt(db_v)))
        if l > 0:
            _, _, dh = conv_backward(hs[l], W, g)
            _, _, dv1 = conv_backward(hs[l], W ** 2, gvar)
            _, _, dv2 = conv_backward(hs[l], W ** 2, g ** 2)
            mask = hs[l] > 0
            g = dh * mask
            gvar = (dv1 + dv2) * mask + g ** 2
    out = out[::-1]
    return np.concatenate([np.concatenate([a.ravel(), c]) for a, c in out])


def output_gradient_flip_bound(theta, channels, r, dz, bmask=None, u=2.0 ** -9, k=8.0):
    """Bound on the change of every entry of output_gradient when the relu decisions differ at
    the pre-activations that lie within k rounding scales (k u sigma) of zero: a low-precision
    evaluation may take either branch there.  A flipped decision at node v changes the upstream
    gradient there by at most |dh(v)|; that change reaches the weight and bias gradients of the
    layer below and, through |W|, the layers further down (absolute sums: flips are few and
    need not be independent)."""
    z, (s, hs) = forward(theta, channels, r, bmask, keep=True)
    _, _, hvar, layers = _forward_vars(theta, channels, r, bmask)
    # pre-activations of the hidden layers and their rounding scales
    pre = []
    for l, (W, b) in enumerate(layers[:-1]):
        a = conv(hs[l], W, b)
        sig = np.sqrt(conv(hvar[l], W ** 2, np.zeros_like(b)) + conv(hs[l] ** 2, W ** 2, np.zeros_like(b)))
        pre.append(np.abs(a) <= k * u * sig)
    g = dz.copy()
    if bmask is not None:
        g[:, bmask] = 0.0
    g = g * s
    E = np.zeros_like(g)                      # bound on the change of g at this layer
    out = []
    for l in range(len(layers) - 1, -1, -1):
        W, b = layers[l]
        dWe, dbe, _ = conv_backward(np.abs(hs[l]), W, E)
        out.append((dWe, dbe))
        if l > 0:
            _, _, dh = conv_backward(hs[l], W, g)
            _, _, dhE = conv_backward(hs[l], np.abs(W), E)
            amb = pre[l - 1]
            mask = hs[l] > 0
            g = dh * mask
            E = dhE * (mask | amb) + np.abs(dh) * amb
    out = out[::-1]
    return np.concatenate([np.concatenate([a.ravel(), c]) for a, c in out])
