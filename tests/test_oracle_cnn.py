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
