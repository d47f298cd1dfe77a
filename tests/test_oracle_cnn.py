"""Pins of the FP64 reference network of the learned stage (finite differences, brute force)."""
import numpy as np

from oracle import cnn


def _brute_conv(h, W, b):
    C, Z, Y, X = h.shape
    out = np.zeros((W.shape[1], Z, Y, X))
    for co in range(W.shape[1]):
        for z in range(Z):
            for y in range(Y):
                for x in range(X):
                    s = b[co]
                    for t in range(27):
                        dx, dy, dz = t % 3 - 1, (t // 3) % 3 - 1, t // 9 - 1
                        zz, yy, xx = z + dz, y + dy, x + dx
                        if 0 <= zz < Z and 0 <= yy < Y and 0 <= xx < X:
                            s += W[t, co, :] @ h[:, zz, yy, xx]
                    out[co, z, y, x] = s
    return out


def test_conv_matches_loops():
    rng = np.random.default_rng(0)
    h = rng.standard_normal((3, 4, 5, 3))
    W = rng.standard_normal((27, 2, 3))
    b = rng.standard_normal(2)
    assert np.allclose(cnn.conv(h, W, b), _brute_conv(h, W, b), atol=1e-12)


def test_gradients_by_finite_differences():
    rng = np.random.default_rng(1)
    ch = [2, 3, 3, 2]
    theta = cnn.init_params(ch, 5) + 0.05 * rng.standard_normal(cnn.param_count(ch))
    r = rng.standard_normal((2, 4, 3, 5))
    e = rng.standard_normal((2, 4, 3, 5))
    bm = np.zeros((4, 3, 5), dtype=bool)
    bm[0] = True
    L, g = cnn.loss_and_grad(theta, ch, r, e, bm)
    idx = rng.choice(len(theta), 25, replace=False)
    for i in idx:
        d = np.zeros_like(theta)
        d[i] = 1e-6
        fd = (cnn.loss_and_grad(theta + d, ch, r, e, bm)[0] - cnn.loss_and_grad(theta - d, ch, r, e, bm)[0]) / 2e-6
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])
    dz = rng.standard_normal(r.shape)
    go = cnn.output_gradient(theta, ch, r, dz, bm)
    for i in idx[:10]:
        d = np.zeros_like(theta)
        d[i] = 1e-6
        fd = (np.sum(dz * cnn.forward(theta + d, ch, r, bm)) - np.sum(dz * cnn.forward(theta - d, ch, r, bm))) / 2e-6
        assert abs(fd - go[i]) <= 1e-6 * max(1.0, abs(go[i]))


def test_homogeneity_and_mask():
    rng = np.random.default_rng(2)
    ch = [3, 4, 3]
    theta = cnn.init_params(ch, 7)
    r = rng.standard_normal((3, 3, 4, 4))
    bm = np.zeros((3, 4, 4), dtype=bool)
    bm[:, 0, :] = True
    z = cnn.forward(theta, ch, r, bm)
    assert np.allclose(cnn.forward(theta, ch, 3.5 * r, bm), 3.5 * z, atol=1e-12)
    assert np.all(z[:, bm] == 0)
    assert np.all(cnn.forward(theta, ch, 0 * r, bm) == 0)


def test_adam_matches_closed_form_first_step():
    # first Adam step moves every parameter by lr * sign(g) (bias-corrected moments)
    g = np.array([0.3, -2.0, 1e-3])
    th, m, v = cnn.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    assert np.allclose(th, -0.01 * np.sign(g))


def _bf16(a):
    """Round to bfloat16 (round to nearest even on the float32 bit pattern), returned as float32."""
    x = np.ascontiguousarray(a, dtype=np.float32)
    bits = x.view(np.uint32).astype(np.uint64)
    bits = (bits + 0x7FFF + ((bits >> 16) & 1)) & 0xFFFF0000
    return bits.astype(np.uint32).view(np.float32)


def _forward_bf16(theta, ch, r, bm):
    # a low-precision evaluation of the same network on the CPU: BF16 weights and activations,
    # float32 sums and output
    s = float(np.sqrt(np.mean(r ** 2)))
    h = _bf16(r / s)
    layers = cnn.unpack(theta, ch)
    for l, (W, b) in enumerate(layers):
        Wb = _bf16(W)
        out = np.zeros((W.shape[1],) + h.shape[1:], dtype=np.float32)
        for t, (dx, dy, dz) in enumerate(cnn.taps()):
            out += np.tensordot(Wb[t], cnn._shift(h, dz, dy, dx), axes=(1, 0)).astype(np.float32)
        out += b[:, None, None, None].astype(np.float32)
        h = _bf16(np.maximum(out, 0.0)) if l < len(layers) - 1 else out
    z = s * h.astype(np.float64)
    z[:, bm] = 0.0
    return z


def test_rounding_scale_bounds_a_bf16_evaluation():
    # the per-element scale used by the GPU parity tests: a BF16/float32 evaluation on the CPU
    # stays within 8 scales of the FP64 network at every element, and the scale is not vacuous
    # (typical errors are a sizeable fraction of it)
    rng = np.random.default_rng(4)
    ch = [4, 16, 16, 4]
    theta = cnn.init_params(ch, 9)
    r = rng.standard_normal((4, 7, 6, 8))
    bm = np.zeros((7, 6, 8), dtype=bool)
    bm[0] = bm[-1] = True
    bm[:, 0] = bm[:, :, -1] = True
    zr = cnn.forward(theta, ch, r, bm)
    sig = cnn.forward_rounding_scale(theta, ch, r, bm)
    u = 2.0 ** -9
    zl = _forward_bf16(theta, ch, r, bm)
    inner = ~np.broadcast_to(bm, zr.shape)
    ratio = np.abs(zl - zr)[inner] / (u * sig[inner])
    assert ratio.max() <= 8.0
    assert 0.05 <= np.sqrt(np.mean(ratio ** 2)) <= 3.0
    # an error planted at one voxel next to the boundary exceeds the bound there
    zbad = zl.copy()
    zbad[1, 1, 1, 1] += 0.1 * np.abs(zr).max()
    assert (np.abs(zbad - zr) > 8.0 * u * sig + 1e-7 * np.abs(zr).max()).sum() == 1


def _output_gradient_bf16(theta, ch, r, dz, bm):
    # BF16 activations, weights and upstream gradients, float32 sums
    s = float(np.sqrt(np.mean(r ** 2)))
    layers = cnn.unpack(theta, ch)
    hs = [_bf16(r / s)]
    for l, (W, b) in enumerate(layers[:-1]):
        Wb = _bf16(W)
        out = np.zeros((W.shape[1],) + r.shape[1:], dtype=np.float32)
        for t, (dx, dy, dz_) in enumerate(cnn.taps()):
            out += np.tensordot(Wb[t], cnn._shift(hs[-1], dz_, dy, dx), axes=(1, 0)).astype(np.float32)
        hs.append(_bf16(np.maximum(out + b[:, None, None, None].astype(np.float32), 0.0)))
    g = dz.copy()
    g[:, bm] = 0.0
    g = _bf16(g * s)
    grads = []
    for l in range(len(layers) - 1, -1, -1):
        W, b = layers[l]
        dW = np.zeros(W.shape, dtype=np.float32)
        for t, (dx, dy, dz_) in enumerate(cnn.taps()):
            dW[t] = np.tensordot(g, cnn._shift(hs[l], dz_, dy, dx), axes=([1, 2, 3], [1, 2, 3]))
        db = g.astype(np.float32).sum(axis=(1, 2, 3))
        grads.append((dW.astype(np.float64), db.astype(np.float64)))
        if l > 0:
            Wb = _bf16(W)
            dh = np.zeros(hs[l].shape, dtype=np.float32)
            for t, (dx, dy, dz_) in enumerate(cnn.taps()):
                dh += cnn._shift(np.tensordot(Wb[t].T, g, axes=(1, 0)), -dz_, -dy, -dx).astype(np.float32)
            g = _bf16(dh * (hs[l] > 0))
    grads = grads[::-1]
    return np.concatenate([np.concatenate([a.ravel(), c]) for a, c in grads])


def test_gradient_rounding_scale_bounds_a_bf16_evaluation():
    # weight and bias gradients of a BF16/float32 evaluation stay within 8 rounding scales plus
    # twice the bound for relu decisions taken differently near zero, at every entry; the bound
    # stays small at most entries
    for seed in (5, 6):
        rng = np.random.default_rng(seed)
        ch = [4, 16, 16, 4]
        theta = cnn.init_params(ch, 10 + seed)
        r = rng.standard_normal((4, 6, 7, 5))
        dz = rng.standard_normal(r.shape)
        bm = np.zeros((6, 7, 5), dtype=bool)
        bm[0] = bm[-1] = True
        gr = cnn.output_gradient(theta, ch, r, dz, bm)
        u = 2.0 ** -9
        bound = (8.0 * u * cnn.output_gradient_rounding_scale(theta, ch, r, dz, bm)
                 + 2.0 * cnn.output_gradient_flip_bound(theta, ch, r, dz, bm, u=u) + 1e-6 * np.abs(gr).max())
        gl = _output_gradient_bf16(theta, ch, r, dz, bm)
        assert np.all(np.abs(gl - gr) <= bound)
        assert np.median(bound) <= 0.05 * np.abs(gr).max()
        # the same bound fails for a gradient with one layer's entries swapped in pairs
        o = 27 * ch[1] * ch[0] + ch[1]
        bad = gl.copy()
        bad[o:o + 200] = bad[o:o + 200].reshape(100, 2)[:, ::-1].ravel()
        assert (np.abs(bad - gr) > bound).sum() >= 20
