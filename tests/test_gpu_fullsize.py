"""Parity at the full benchmark size (heat 3D, 32^3 Q4 cells with perturbed vertices, dG(2),
8 time cells: 51.5 M space-time DoFs), in the launch configuration the benchmark times.

The assembled oracle does not fit at this size, so the operator and one smoother step are
compared on sampled entries computed one by one by the oracle (cell-local assembly of the
same definitions), and the V-cycle and the solve are checked through properties that hold
at any size: linearity and contraction of the V-cycle, and the true residual of the solve
(the GPU's own and the oracle's on sampled rows).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import stmg_inputs as si
from oracle import sampled

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
CFG = si.paper_config(2)


@pytest.fixture(scope="module")
def setup():
    from paper_2408_04372_amd import Handle
    verts, coef = si.draw_problem(CFG)
    print("creating full-size handle", CFG.name, flush=True)
    h = Handle(CFG, verts, coef, vcycle_dtypes=3, precision=0, rtol=1e-8, restart=30, max_iter=300,
               omega=-1.0)
    smp = sampled.Sampler(CFG, verts, coef)
    pts = sampled.sample_points(CFG, 24, 4, seed=2024)
    yield h, smp, pts
    h.close()


def _dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype=dtype).reshape(-1).contiguous()


def _entries(t, pts, n_x):
    torch.cuda.synchronize()
    idx = torch.tensor([i * n_x + g for i, g in pts], device=DEV)
    return t[idx].double().cpu().numpy()


def test_operator_sampled_entries(setup):
    h, smp, pts = setup
    n_x = smp.space.n_x
    x = np.random.default_rng(1).standard_normal((CFG.n_t, n_x))
    ref = smp.operator_entries(x, pts)
    scale = np.abs(ref).max()
    for dt, tol in ((torch.float64, 1e-12), (torch.float32, 3e-5)):
        xt = _dev(x, dt)
        yt = torch.empty_like(xt)
        h.vmult(xt, yt)
        got = _entries(yt, pts, n_x)
        err = np.abs(got - ref).max() / scale
        print(dt, "operator sampled max rel err", err, flush=True)
        assert err < tol


def test_smoother_sampled_entries(setup):
    h, smp, pts = setup
    n_x = smp.space.n_x
    r = np.random.default_rng(2).standard_normal((CFG.n_t, n_x))
    omega = h.info["omega"][0]
    ref = smp.asm_entries(r, omega, pts)
    rt = _dev(r)
    u = torch.zeros_like(rt)
    h.smooth(rt, u, steps=1)
    got = _entries(u, pts, n_x)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print("smoother sampled max rel err", err, "omega", omega, flush=True)
    assert err < 1e-10


def test_vcycle_linear_and_contracting(setup):
    h, smp, pts = setup
    n = h.size(0)
    g = torch.Generator(device="cpu").manual_seed(3)
    r1 = torch.randn(n, generator=g, dtype=torch.float64).to(DEV)
    r2 = torch.randn(n, generator=g, dtype=torch.float64).to(DEV)
    z1, z2, z3 = (torch.empty_like(r1) for _ in range(3))
    h.vcycle(r1, z1)
    h.vcycle(r2, z2)
    h.vcycle(r1 + 2.0 * r2, z3)
    lin = (torch.linalg.norm(z3 - z1 - 2.0 * z2) / torch.linalg.norm(z3)).item()
    Sz = torch.empty_like(r1)
    h.vmult(z1, Sz)
    contraction = (torch.linalg.norm(r1 - Sz) / torch.linalg.norm(r1)).item()
    print("vcycle linearity", lin, "contraction", contraction, flush=True)
    assert lin < 1e-12
    assert contraction < 0.9


@pytest.mark.parametrize("precision", [0, 1])
def test_solve_true_residual(setup, precision):
    h, smp, pts = setup
    n_x = smp.space.n_x
    b = si.random_slab_vector(CFG, 1001)
    bt = _dev(b)
    x = torch.zeros_like(bt)
    h.set_precision(precision)
    info = h.solve(bt, x)
    h.set_precision(0)
    print("solve", precision, info, flush=True)
    assert info["rel_residual"] <= 1e-8
    xs = x.cpu().numpy().reshape(CFG.n_t, n_x)
    res = b.reshape(CFG.n_t, n_x)
    rows = np.array([res[i, g] for i, g in pts]) - smp.operator_entries(xs, pts)
    assert np.abs(rows).max() <= 1e-8 * np.linalg.norm(b)
