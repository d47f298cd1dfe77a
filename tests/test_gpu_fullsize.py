"""Parity at the full sizes of the five workloads, in their launch configurations:
  heat 3D 32^3 Q4 perturbed dG(2) c=8 (51.5 M DoFs, the benchmark: FP64 V-cycle, exact cell blocks),
  wave 3D 64^3 Q3 cGP(2) c=4 (57.5 M DoFs, FP32 V-cycle, exact cell blocks),
  heat 3D 128^3 Q4 dG(1) c=2 (540 M DoFs, FP32 V-cycle, separable cell blocks, restart 10),
  heat 3D 64^3 Q2 dG(1) c=4 (17.2 M DoFs, FP32 V-cycle, exact cell blocks).

The assembled oracle does not fit at these sizes, so the operator and one smoother step are
compared on sampled entries computed one by one by the oracle (cell-local assembly of the
same definitions), and so are the grid transfers of the first p- and h-level pairs; the
V-cycle and the solve are checked through properties that hold at any size: linearity and
contraction of the V-cycle, and the true residual of the solve (the GPU's own and the
oracle's on sampled rows).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import stmg_inputs as si
from oracle import sampled

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

# config index -> (handle settings, V-cycle dtype)
LAUNCH = {
    2: (dict(vcycle_dtypes=3, precision=0, restart=30, asm_variant=0), torch.float64),
    3: (dict(vcycle_dtypes=2, precision=1, restart=30, asm_variant=0), torch.float32),
    4: (dict(vcycle_dtypes=2, precision=1, restart=10, asm_variant=1), torch.float32),
    5: (dict(vcycle_dtypes=2, precision=1, restart=30, asm_variant=0), torch.float32),
}


@pytest.fixture(scope="module", params=[2, 3, 4, 5], ids=lambda i: f"config{i}")
def setup(request):
    from paper_2408_04372_amd import Handle
    idx = request.param
    cfg = si.paper_config(idx)
    kw, vdt = LAUNCH[idx]
    verts, coef = si.draw_problem(cfg)
    print(f"creating full-size handle {cfg.name} ({cfg.n_st} DoFs)", flush=True)
    h = Handle(cfg, verts, coef, rtol=1e-8, max_iter=300, omega=-1.0, **kw)
    print("setup s", h.info["setup_seconds"], "device GB", h.info["device_bytes"] / 1e9, flush=True)
    smp = sampled.Sampler(cfg, verts, coef)
    pts = sampled.sample_points(cfg, 24, 4, seed=2024 + idx)
    yield cfg, h, smp, pts, vdt, kw
    h.close()
    torch.cuda.empty_cache()


def _dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype=dtype).reshape(-1).contiguous()


def _entries(t, pts, n_x):
    torch.cuda.synchronize()
    idx = torch.tensor([i * n_x + g for i, g in pts], device=DEV)
    return t[idx].double().cpu().numpy()


def test_operator_sampled_entries(setup):
    cfg, h, smp, pts, vdt, kw = setup
    n_x = smp.space.n_x
    x = np.random.default_rng(1).standard_normal((cfg.n_t, n_x))
    ref = smp.operator_entries(x, pts)
    scale = np.abs(ref).max()
    for dt, tol in ((torch.float64, 1e-12), (torch.float32, 3e-5)):
        xt = _dev(x, dt)
        yt = torch.empty_like(xt)
        h.vmult(xt, yt)
        got = _entries(yt, pts, n_x)
        del xt, yt
        err = np.abs(got - ref).max() / scale
        print(cfg.name, dt, "operator sampled max rel err", err, flush=True)
        assert err < tol


def test_smoother_sampled_entries(setup):
    cfg, h, smp, pts, vdt, kw = setup
    n_x = smp.space.n_x
    r = np.random.default_rng(2).standard_normal((cfg.n_t, n_x))
    omega = h.info["omega"][0]
    ref = smp.asm_entries(r, omega, pts, separable=kw["asm_variant"] == 1)
    rt = _dev(r, vdt)
    u = torch.zeros_like(rt)
    h.smooth(rt, u, steps=1)
    got = _entries(u, pts, n_x)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(cfg.name, "smoother sampled max rel err", err, "omega", omega, flush=True)
    assert err < (1e-10 if vdt == torch.float64 else 2e-5)


def test_transfer_sampled_entries(setup):
    """Prolongation and restriction across the first p-level and the first h-level pair, on
    sampled entries of the oracle's tensor-product transfers (FP64 workloads also in FP32)."""
    cfg, h, smp, pts, vdt, kw = setup
    spaces = smp.level_spaces()
    assert h.info["n_levels"] == len(spaces)
    pairs = [0] + [l for l in range(len(spaces) - 1) if spaces[l].cells != spaces[l + 1].cells][:1]
    rng = np.random.default_rng(6)
    for l in pairs:
        fine, coarse = spaces[l], spaces[l + 1]
        assert h.info["n_x"][l] == fine.n_x and h.info["n_x"][l + 1] == coarse.n_x
        n_t = h.info["n_t_level"][l]
        ptf = sampled.lattice_points(fine.p, fine.cells, n_t, 24, 4, seed=50 + l)
        ptc = sampled.lattice_points(coarse.p, coarse.cells, n_t, 24, 4, seed=80 + l)
        ec = rng.standard_normal((n_t, coarse.n_x))
        ref_p = smp.prolong_entries(ec, l, ptf)
        for dt, tol in ((torch.float64, 1e-13), (torch.float32, 1e-6)):
            if dt == torch.float64 and vdt != torch.float64:
                continue
            f = torch.empty(h.size(l), dtype=dt, device=DEV)
            h.prolongate(_dev(ec, dt), f, level=l)
            err = np.abs(_entries(f, ptf, fine.n_x) - ref_p).max() / np.abs(ref_p).max()
            del f
            print(cfg.name, f"level {l} prolongation {dt} sampled max rel err", err, flush=True)
            assert err < tol
        del ec
        rf = rng.standard_normal((n_t, fine.n_x))
        ref_r = smp.restrict_entries(rf, l, ptc)
        for dt, tol in ((torch.float64, 1e-13), (torch.float32, 1e-6)):
            if dt == torch.float64 and vdt != torch.float64:
                continue
            c = torch.empty(h.size(l + 1), dtype=dt, device=DEV)
            h.restrict(_dev(rf, dt), c, level=l)
            err = np.abs(_entries(c, ptc, coarse.n_x) - ref_r).max() / np.abs(ref_r).max()
            del c
            print(cfg.name, f"level {l} restriction {dt} sampled max rel err", err, flush=True)
            assert err < tol
        del rf


def test_vcycle_linear_and_contracting(setup):
    cfg, h, smp, pts, vdt, kw = setup
    n = h.size(0)
    g = torch.Generator(device="cpu").manual_seed(3)
    r1 = torch.randn(n, generator=g, dtype=vdt).to(DEV)
    r2 = torch.randn(n, generator=g, dtype=vdt).to(DEV)
    z1, z2, z3 = (torch.empty_like(r1) for _ in range(3))
    h.vcycle(r1, z1)
    h.vcycle(r2, z2)
    h.vcycle(r1 + 2.0 * r2, z3)
    lin = (torch.linalg.norm(z3 - z1 - 2.0 * z2) / torch.linalg.norm(z3)).item()
    Sz = torch.empty_like(r1)
    h.vmult(z1, Sz)
    contraction = (torch.linalg.norm(r1 - Sz) / torch.linalg.norm(r1)).item()
    del r1, r2, z1, z2, z3, Sz
    print(cfg.name, "vcycle linearity", lin, "contraction", contraction, flush=True)
    assert lin < (1e-12 if vdt == torch.float64 else 1e-5)
    assert contraction < 1.0


def test_solve_true_residual(setup):
    cfg, h, smp, pts, vdt, kw = setup
    n_x = smp.space.n_x
    b = si.random_slab_vector(cfg, 1001)
    bt = _dev(b)
    x = torch.zeros_like(bt)
    info = h.solve(bt, x)
    print(cfg.name, "solve", info, flush=True)
    assert info["rel_residual"] <= 1e-8
    xs = x.cpu().numpy().reshape(cfg.n_t, n_x)
    del bt, x
    res = b.reshape(cfg.n_t, n_x)
    rows = np.array([res[i, g] for i, g in pts]) - smp.operator_entries(xs, pts)
    assert np.abs(rows).max() <= 1e-8 * np.linalg.norm(b)
