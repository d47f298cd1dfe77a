"""Learned preconditioning stage on the GPU against the FP64 reference network.

Activations, weights and upstream gradients are BF16 (unit roundoff u = 2^-9) with FP32
accumulation.  Outputs and parameter gradients are compared element by element: every entry
must lie within 8 rounding scales u sigma of the reference (sigma from propagating the squared
terms of every sum through the layers, oracle.cnn.*_rounding_scale), and a gradient entry may
in addition move by twice the bound on relu decisions taken the other way at pre-activations
within a few rounding scales of zero (oracle.cnn.output_gradient_flip_bound).  A CPU test
checks these bounds against a BF16 evaluation on the CPU.  The relative 2-norms (3e-2 output,
6e-2 gradients, per layer) are checked as well.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import stmg_inputs as si
from oracle import cnn as ref
from oracle import spacetime

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

CFG = si.Config(dim=3, problem=0, time_method=0, p=2, k=1, n_time_cells=4, n_cells=(4, 5, 3), tau=0.05,
                perturb=0.1, coef="lognormal", coef_sigma=1.0, seed=31)


def _setup(channels=None, seed=3):
    from paper_2408_04372_amd import Handle
    cfg = CFG
    verts, coef = si.draw_problem(cfg)
    h = Handle(cfg, verts, coef, vcycle_dtypes=3, precision=2, omega=-1.0, rtol=1e-8, max_iter=200)
    ch = channels or [cfg.n_t, 16, 16, cfg.n_t]
    h.cnn_create(ch)
    theta = ref.init_params(ch, seed).astype(np.float32)
    h.cnn_set_params(theta)
    op = spacetime.from_config(cfg, verts, coef)
    bm = op.bmask.reshape(tuple(cfg.nodes[::-1]))
    return cfg, h, ch, theta, op, bm


def _vec(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV).reshape(-1).contiguous()


def test_forward_matches_reference():
    cfg, h, ch, theta, op, bm = _setup()
    r = si.random_slab_vector(cfg, 5)
    z = torch.zeros(r.size, dtype=torch.float64, device=DEV)
    h.cnn_forward(_vec(r), z)
    zr = ref.forward(theta.astype(np.float64), ch, r.reshape((cfg.n_t,) + tuple(cfg.nodes[::-1])), bm)
    zg = z.cpu().numpy().reshape(zr.shape)
    err = np.linalg.norm(zg - zr) / np.linalg.norm(zr)
    sig = ref.forward_rounding_scale(theta.astype(np.float64), ch, r.reshape(zr.shape), bm)
    u = 2.0 ** -9
    ratio = np.abs(zg - zr) / (8.0 * u * sig + 1e-7 * np.abs(zr).max())
    print("forward rel err", err, "max element error / bound", ratio.max(), "at", np.unravel_index(ratio.argmax(),
                                                                                              ratio.shape))
    assert err < 3e-2
    assert ratio.max() <= 1.0
    assert np.all(zg[:, bm] == 0)
    # positive homogeneity survives the BF16 path exactly up to rounding of the scale
    h.cnn_forward(_vec(4.0 * r), z)
    assert np.linalg.norm(z.cpu().numpy().reshape(zr.shape) - 4.0 * zg) < 1e-6 * np.linalg.norm(zg)
    h.close()


def test_param_gradient_matches_reference():
    cfg, h, ch, theta, op, bm = _setup()
    rng = np.random.default_rng(8)
    r = si.random_slab_vector(cfg, 6)
    dz = rng.standard_normal(r.shape)
    gg = h.cnn_param_grad(_vec(r), _vec(dz))
    shape = (cfg.n_t,) + tuple(cfg.nodes[::-1])
    gr = ref.output_gradient(theta.astype(np.float64), ch, r.reshape(shape), dz.reshape(shape), bm)
    err = np.linalg.norm(gg - gr) / np.linalg.norm(gr)
    th64 = theta.astype(np.float64)
    u = 2.0 ** -9
    bound = (8.0 * u * ref.output_gradient_rounding_scale(th64, ch, r.reshape(shape), dz.reshape(shape), bm)
             + 2.0 * ref.output_gradient_flip_bound(th64, ch, r.reshape(shape), dz.reshape(shape), bm, u=u)
             + 1e-6 * np.abs(gr).max())
    ratio = np.abs(gg - gr) / bound
    print("gradient rel err", err, "max element error / bound", ratio.max(), "at", int(ratio.argmax()),
          "median bound / max", np.median(bound) / np.abs(gr).max())
    assert err < 6e-2
    assert ratio.max() <= 1.0
    # per layer as well (catches a transposed or flipped layer)
    o = 0
    for l in range(len(ch) - 1):
        n = 27 * ch[l + 1] * ch[l] + ch[l + 1]
        e = np.linalg.norm(gg[o:o + n] - gr[o:o + n]) / np.linalg.norm(gr[o:o + n])
        assert e < 6e-2, (l, e)
        o += n
    h.close()


def test_training_reduces_loss():
    cfg, h, ch, theta, op, bm = _setup()
    r = si.random_slab_vector(cfg, 7)
    e = op.solve(r)
    rt, et = _vec(r), _vec(e)
    losses = [h.cnn_train_step(rt, et, 3e-3) for _ in range(60)]
    print("loss", losses[0], "->", losses[-1])
    assert losses[-1] < 0.7 * losses[0]
    th = h.cnn_get_params()
    assert np.all(np.isfinite(th)) and np.abs(th - theta).max() > 0
    h.close()


def test_learned_solve_and_fallback():
    cfg, h, ch, theta, op, bm = _setup()
    b = si.random_slab_vector(cfg, 9)
    x = torch.zeros(b.size, dtype=torch.float64, device=DEV)
    info = h.solve(_vec(b), x)
    res = np.linalg.norm(b.ravel() - op.matrix() @ x.cpu().numpy()) / np.linalg.norm(b)
    print("learned (untrained)", info, "oracle residual", res)
    assert res <= 1e-8
    assert info["cnn_used"] + info["cnn_fallbacks"] == info["iterations"]
    # corrupted weights: the stage must be rejected every time and the solve still converges
    h.cnn_set_params(theta * 1e6)
    x.zero_()
    info2 = h.solve(_vec(b), x)
    res2 = np.linalg.norm(b.ravel() - op.matrix() @ x.cpu().numpy()) / np.linalg.norm(b)
    print("learned (corrupted)", info2)
    assert res2 <= 1e-8
    assert info2["cnn_used"] == 0 and info2["cnn_fallbacks"] == info2["iterations"]
    h.close()
