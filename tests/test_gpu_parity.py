"""GPU parity: the C-ABI library against the FP64 CPU oracle on the same seeded inputs.

Tolerances: the FP64 kernels sum in a fixed order that differs from the oracle's
(sum factorisation instead of assembled sparse rows, cell contributions summed node by
node in a fixed cell order, or per brick and then in brick-colour order), so results agree
to a few ulps of the largest entry: 1e-12 relative to the max norm.  FP32 kernels: 2e-5 (a few FP32 ulps times the sum-factorisation depth).
Solutions: 1e-10 relative (FP64 path), true residual 1e-8 (FP32-preconditioned path).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import stmg_inputs as si
from oracle import krylov, mg, spacetime
from tests.gpu_common import BRICK_CASES, CASES, PATCH_CASES, oracle_op, problem, rel_err

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _handle(cfg, verts, coef, **kw):
    from paper_2408_04372_amd import Handle
    kw.setdefault("vcycle_dtypes", 3)
    return Handle(cfg, verts, coef, **kw)


def _t(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype=dtype).contiguous()


def _np(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


@pytest.mark.parametrize("name", list(CASES))
def test_vmult_fp64_fp32(name):
    cfg, verts, coef = problem(name)
    print(f"case {name}", flush=True)
    op = oracle_op(cfg, verts, coef)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((cfg.n_t, cfg.n_x))
    ref = op.apply(x)
    with _handle(cfg, verts, coef, omega=0.5) as h:
        y = torch.empty(cfg.n_t * cfg.n_x, dtype=torch.float64, device=DEV)
        h.vmult(_t(x).view(-1), y)
        assert rel_err(_np(y), ref) < 1e-12
        y32 = torch.empty(cfg.n_t * cfg.n_x, dtype=torch.float32, device=DEV)
        h.vmult(_t(x, torch.float32).view(-1), y32)
        assert rel_err(_np(y32), ref) < 2e-5


@pytest.mark.parametrize("name", ["heat2d_q2_dg1", "heat3d_q2_dg1_pert", "wave3d_q3_cgp2",
                                  "heat2d_q4_cgp2_pert", "wave3d_q2_cgp1_ragged"])
def test_transfers_and_coarse_operators(name):
    cfg, verts, coef = problem(name)
    op = oracle_op(cfg, verts, coef)
    H = mg.Hierarchy(op, omegas=[1.0] * 16)
    L = len(H.levels)
    rng = np.random.default_rng(4)
    with _handle(cfg, verts, coef, omega=0.5) as h:
        assert h.info["n_levels"] == L
        for l in range(L):
            lev = H.levels[L - 1 - l]
            assert h.info["n_x"][l] == lev.op.n_x and h.info["p"][l] == lev.op.space.p
            x = rng.standard_normal(lev.S.shape[0])
            y = torch.empty(x.size, dtype=torch.float64, device=DEV)
            h.vmult(_t(x), y, level=l)
            assert rel_err(_np(y), lev.S @ x) < 1e-12
        for l in range(L - 1):
            io = L - 1 - l          # oracle index of the fine level
            nc = H.levels[io - 1].S.shape[0]
            nf = H.levels[io].S.shape[0]
            xc = rng.standard_normal(nc)
            xf = rng.standard_normal(nf)
            for dt, tol in ((torch.float64, 1e-13), (torch.float32, 1e-6)):
                f = torch.empty(nf, dtype=dt, device=DEV)
                h.prolongate(_t(xc, dt), f, level=l)
                assert rel_err(_np(f), H.prolong(io, xc)) < tol
                c = torch.empty(nc, dtype=dt, device=DEV)
                h.restrict(_t(xf, dt), c, level=l)
                assert rel_err(_np(c), H.restrict(io, xf)) < tol


@pytest.mark.parametrize("name", list(CASES))
def test_smoother(name):
    cfg, verts, coef = problem(name)
    print(f"case {name}", flush=True)
    op = oracle_op(cfg, verts, coef)
    lev = mg.Level(op=op, S=op.matrix())
    lev.blocks = mg.asm_blocks(op, lev.S)
    rng = np.random.default_rng(5)
    b = rng.standard_normal(lev.S.shape[0])
    x0 = rng.standard_normal(lev.S.shape[0])
    omega = 0.37
    ref = mg.smooth(lev, b, x0, 2, omega=omega)
    with _handle(cfg, verts, coef, omega=omega) as h:
        for dt, tol in ((torch.float64, 1e-11), (torch.float32, 2e-4)):
            x = _t(x0, dt)
            h.smooth(_t(b, dt), x, steps=2, level=0)
            assert rel_err(_np(x), ref) < tol, dt


@pytest.mark.parametrize("name", ["heat2d_q2_dg1", "heat3d_q2_dg1_pert", "wave3d_q3_cgp2",
                                  "wave2d_q3_dg2", "heat3d_q1_dg0"])
def test_vcycle(name):
    cfg, verts, coef = problem(name)
    op = oracle_op(cfg, verts, coef)
    H = mg.Hierarchy(op, n_smooth=cfg.n_smooth)
    rng = np.random.default_rng(6)
    r = rng.standard_normal(op.matrix().shape[0])
    ref = H.vcycle(r)
    with _handle(cfg, verts, coef, omega=0.5) as h:
        L = h.info["n_levels"]
        for l in range(L - 1):
            h.set_omega(l, H.levels[L - 1 - l].omega)
        for dt, tol in ((torch.float64, 1e-10), (torch.float32, 1e-4)):
            z = torch.empty(r.size, dtype=dt, device=DEV)
            h.vcycle(_t(r, dt), z)
            assert rel_err(_np(z), ref) < tol, dt


@pytest.mark.parametrize("name", ["heat2d_q2_dg1", "heat3d_q2_dg1_pert", "wave3d_q3_cgp2"])
def test_mg_step(name):
    """Two stationary multigrid iterations x <- x + V(b - S x) (Alg. stmg on the residual) against
    the oracle's residual and V-cycle, with the residual and correction of each step."""
    cfg, verts, coef = problem(name)
    op = oracle_op(cfg, verts, coef)
    S = op.matrix()
    H = mg.Hierarchy(op, n_smooth=cfg.n_smooth)
    b = si.random_slab_vector(cfg, 21).ravel()
    with _handle(cfg, verts, coef, omega=0.5) as h:
        L = h.info["n_levels"]
        for l in range(L - 1):
            h.set_omega(l, H.levels[L - 1 - l].omega)
        for dt, tol in ((torch.float64, 1e-10), (torch.float32, 1e-4)):
            x_ref = np.zeros(b.size)
            bt = _t(b, dt)
            x = torch.zeros_like(bt)
            r = torch.empty_like(bt)
            z = torch.empty_like(bt)
            for _ in range(2):
                r_ref = b - S @ x_ref
                z_ref = H.vcycle(r_ref)
                x_ref = x_ref + z_ref
                h.mg_step(bt, x, r, z)
                assert rel_err(_np(r), r_ref) < tol, dt
                assert rel_err(_np(z), z_ref) < tol, dt
                assert rel_err(_np(x), x_ref) < tol, dt


@pytest.mark.parametrize("rule", [0.0, -1.0])
@pytest.mark.parametrize("name", ["heat2d_q2_dg1", "heat3d_q2_dg1_pert", "wave3d_q3_cgp2"])
def test_omega_estimate(name, rule):
    cfg, verts, coef = problem(name)
    op = oracle_op(cfg, verts, coef)
    H = mg.Hierarchy(op, omega_rule=rule)
    with _handle(cfg, verts, coef, omega=rule) as h:
        L = h.info["n_levels"]
        got = h.info["omega"][: L - 1]
        ref = [H.levels[L - 1 - l].omega for l in range(L - 1)]
    # 15-step Arnoldi Ritz values are sensitive to rounding (both sides orthogonalise twice, in
    # different summation orders: classical Gram-Schmidt on the GPU, modified in the oracle)
    assert np.allclose(got, ref, rtol=1e-4)


@pytest.mark.parametrize("name,gs", [("heat2d_q2_dg1", 0), ("heat3d_q2_dg1_pert", 0), ("wave3d_q3_cgp2", 0),
                                     ("heat2d_q4_cgp2_pert", 0), ("wave3d_q2_cgp1_ragged", 0),
                                     ("heat3d_q2_dg1_pert", 1), ("wave3d_q3_cgp2", 1)])
def test_solve_fp64_matches_direct(name, gs):
    cfg, verts, coef = problem(name)
    op = oracle_op(cfg, verts, coef)
    b = si.random_slab_vector(cfg, 11)
    xd = op.solve(b)
    with _handle(cfg, verts, coef, rtol=1e-12, precision=0, max_iter=300, gram_schmidt=gs) as h:
        x = torch.zeros(b.size, dtype=torch.float64, device=DEV)
        info = h.solve(_t(b).view(-1), x)
        err = np.linalg.norm(_np(x) - xd.ravel()) / np.linalg.norm(xd)
    print(name, info)
    assert info["rel_residual"] <= 1e-12
    assert err < 1e-10


@pytest.mark.parametrize("name", ["heat2d_q2_dg1", "heat3d_q2_dg1_pert", "wave3d_q3_cgp2"])
def test_solve_fp32_preconditioner(name):
    cfg, verts, coef = problem(name)
    op = oracle_op(cfg, verts, coef)
    b = si.random_slab_vector(cfg, 12)
    xd = op.solve(b)
    with _handle(cfg, verts, coef, rtol=1e-8, precision=1, max_iter=300) as h:
        x = torch.zeros(b.size, dtype=torch.float64, device=DEV)
        info = h.solve(_t(b).view(-1), x)
        xs = _np(x)
    res = np.linalg.norm(b.ravel() - op.matrix() @ xs) / np.linalg.norm(b)
    err = np.linalg.norm(xs - xd.ravel()) / np.linalg.norm(xd)
    print(name, info, "oracle residual", res, "error", err)
    assert res <= 1e-8
    assert info["rel_residual"] <= 1e-8


@pytest.mark.parametrize("name", ["wave2d_q3_dg2", "wave3d_q3_cgp2", "wave3d_q2_cgp1_ragged"])
def test_wave_velocity_matches_oracle(name):
    from oracle import rhs
    cfg, verts, coef = problem(name)
    op = oracle_op(cfg, verts, coef)
    rng = np.random.default_rng(31)
    U = rng.standard_normal((cfg.n_t, op.n_x))
    u0 = rng.standard_normal(op.n_x)
    v0 = rng.standard_normal(op.n_x)
    ref = rhs.velocity(op, U, u0, v0)
    ref0 = rhs.velocity(op, U)
    with _handle(cfg, verts, coef) as h:
        V = torch.empty(U.size, dtype=torch.float64, device=DEV)
        h.wave_velocity(_t(U).view(-1), V, _t(u0), _t(v0))
        got = _np(V).reshape(ref.shape)
        h.wave_velocity(_t(U).view(-1), V)
        got0 = _np(V).reshape(ref.shape)
    assert rel_err(got, ref) < 1e-12
    assert rel_err(got0, ref0) < 1e-12


def test_wave_velocity_rejects_heat():
    from paper_2408_04372_amd import StmgError
    cfg, verts, coef = problem("heat2d_q2_dg1")
    with _handle(cfg, verts, coef) as h:
        U = torch.zeros(h.size(0), dtype=torch.float64, device=DEV)
        with pytest.raises(StmgError):
            h.wave_velocity(U, torch.empty_like(U))


FDM_CASES = ["heat2d_q2_dg1", "wave2d_q3_dg2", "heat3d_q1_dg0", "wave3d_q3_cgp2_c4"]


@pytest.mark.parametrize("name", FDM_CASES)
def test_smoother_separable(name):
    cfg, verts, coef = problem(name)
    print(f"case {name}", flush=True)
    op = oracle_op(cfg, verts, coef)
    lev = mg.Level(op=op, S=op.matrix())
    lev.blocks = mg.fdm_blocks(op)
    rng = np.random.default_rng(15)
    b = rng.standard_normal(lev.S.shape[0])
    x0 = rng.standard_normal(lev.S.shape[0])
    omega = 0.37
    ref = mg.smooth(lev, b, x0, 2, omega=omega)
    with _handle(cfg, verts, coef, omega=omega, asm_variant=1) as h:
        for dt, tol in ((torch.float64, 1e-11), (torch.float32, 2e-4)):
            x = _t(x0, dt)
            h.smooth(_t(b, dt), x, steps=2, level=0)
            err = rel_err(_np(x), ref)
            print(dt, "separable smoother rel err", err)
            assert err < tol, dt


@pytest.mark.parametrize("name", FDM_CASES)
def test_vcycle_and_solve_separable(name):
    cfg, verts, coef = problem(name)
    op = oracle_op(cfg, verts, coef)
    H = mg.Hierarchy(op, n_smooth=cfg.n_smooth, asm_variant=1, omega_rule=-1.0)
    rng = np.random.default_rng(16)
    r = rng.standard_normal(op.matrix().shape[0])
    ref = H.vcycle(r)
    b = si.random_slab_vector(cfg, 17)
    xd = op.solve(b)
    with _handle(cfg, verts, coef, omega=-1.0, asm_variant=1, rtol=1e-12, precision=0, max_iter=300) as h:
        L = h.info["n_levels"]
        got_omega = h.info["omega"][: L - 1]
        assert np.allclose(got_omega, [H.levels[L - 1 - l].omega for l in range(L - 1)], rtol=1e-4)
        for l in range(L - 1):
            h.set_omega(l, H.levels[L - 1 - l].omega)
        for dt, tol in ((torch.float64, 1e-10), (torch.float32, 1e-4)):
            z = torch.empty(r.size, dtype=dt, device=DEV)
            h.vcycle(_t(r, dt), z)
            assert rel_err(_np(z), ref) < tol, dt
        x = torch.zeros(b.size, dtype=torch.float64, device=DEV)
        info = h.solve(_t(b).view(-1), x)
        err = np.linalg.norm(_np(x) - xd.ravel()) / np.linalg.norm(xd)
    print(name, info, "error", err)
    assert info["rel_residual"] <= 1e-12
    assert err < 1e-10


@pytest.mark.parametrize("name", PATCH_CASES)
def test_smoother_vertex_patch(name):
    """Two steps of the separable vertex-patch smoother against the oracle's patch blocks."""
    cfg, verts, coef = problem(name)
    print(f"case {name}", flush=True)
    op = oracle_op(cfg, verts, coef)
    lev = mg.Level(op=op, S=op.matrix())
    lev.blocks = mg.fdm_patch_blocks(op)
    rng = np.random.default_rng(18)
    b = rng.standard_normal(lev.S.shape[0])
    x0 = rng.standard_normal(lev.S.shape[0])
    omega = 0.29
    ref = mg.smooth(lev, b, x0, 2, omega=omega)
    with _handle(cfg, verts, coef, omega=omega, asm_variant=2) as h:
        for dt, tol in ((torch.float64, 1e-11), (torch.float32, 2e-4)):
            x = _t(x0, dt)
            h.smooth(_t(b, dt), x, steps=2, level=0)
            err = rel_err(_np(x), ref)
            print(dt, "vertex-patch smoother rel err", err)
            assert err < tol, dt


@pytest.mark.parametrize("name", ["heat2d_q2_dg1", "heat3d_q1_dg0", "heat3d_q4_dg1_brick"])
def test_vcycle_and_solve_vertex_patch(name):
    cfg, verts, coef = problem(name)
    op = oracle_op(cfg, verts, coef)
    H = mg.Hierarchy(op, n_smooth=cfg.n_smooth, asm_variant=2, omega_rule=-1.0)
    rng = np.random.default_rng(19)
    r = rng.standard_normal(op.matrix().shape[0])
    ref = H.vcycle(r)
    b = si.random_slab_vector(cfg, 20)
    xd = op.solve(b)
    with _handle(cfg, verts, coef, omega=-1.0, asm_variant=2, rtol=1e-12, precision=0, max_iter=300) as h:
        L = h.info["n_levels"]
        got_omega = h.info["omega"][: L - 1]
        assert np.allclose(got_omega, [H.levels[L - 1 - l].omega for l in range(L - 1)], rtol=1e-4)
        for l in range(L - 1):
            h.set_omega(l, H.levels[L - 1 - l].omega)
        for dt, tol in ((torch.float64, 1e-10), (torch.float32, 1e-4)):
            z = torch.empty(r.size, dtype=dt, device=DEV)
            h.vcycle(_t(r, dt), z)
            assert rel_err(_np(z), ref) < tol, dt
        x = torch.zeros(b.size, dtype=torch.float64, device=DEV)
        info = h.solve(_t(b).view(-1), x)
        err = np.linalg.norm(_np(x) - xd.ravel()) / np.linalg.norm(xd)
    print(name, info, "error", err)
    assert info["rel_residual"] <= 1e-12
    assert err < 1e-10


def test_vertex_patch_rejects_unsupported_meshes():
    from paper_2408_04372_amd import StmgError
    cfg, verts, coef = problem("heat3d_q2_dg1_pert")
    with pytest.raises(StmgError):
        _handle(cfg, verts, coef, asm_variant=2)
    cfg = si.Config(dim=3, problem=0, time_method=0, p=2, k=1, n_time_cells=1, n_cells=(3, 1, 2), tau=0.1, seed=3)
    verts, coef = si.draw_problem(cfg)
    with pytest.raises(StmgError):                 # one cell along y: no interior vertex
        _handle(cfg, verts, coef, asm_variant=2)


def test_separable_rejects_perturbed_mesh():
    from paper_2408_04372_amd import StmgError
    cfg, verts, coef = problem("heat3d_q2_dg1_pert")
    with pytest.raises(StmgError):
        _handle(cfg, verts, coef, asm_variant=1)


@pytest.mark.parametrize("name", ["heat2d_q2_dg1", "heat2d_q4_cgp2_pert", "wave2d_q3_dg2", "wave3d_q3_cgp2",
                                  "wave3d_q2_cgp1_ragged"])
def test_slab_rhs_matches_oracle(name):
    from oracle import rhs
    cfg, verts, coef = problem(name)
    op = oracle_op(cfg, verts, coef)
    rng = np.random.default_rng(41)
    F = rng.standard_normal((cfg.n_t, op.n_x))
    F0, u0, v0 = (rng.standard_normal(op.n_x) for _ in range(3))
    cgp = cfg.time_method == 1
    ref = rhs.rhs(op, F, F0 if cgp else None, u0, v0)
    ref_f = rhs.rhs(op, F, F0 if cgp else None)
    with _handle(cfg, verts, coef) as h:
        b = torch.empty(F.size, dtype=torch.float64, device=DEV)
        h.slab_rhs(b, _t(F).view(-1), _t(F0) if cgp else None, _t(u0), _t(v0))
        got = _np(b).reshape(ref.shape)
        h.slab_rhs(b, _t(F).view(-1), _t(F0) if cgp else None)
        got_f = _np(b).reshape(ref.shape)
    assert rel_err(got, ref) < 1e-12
    assert rel_err(got_f, ref_f) < 1e-12


@pytest.mark.parametrize("path", [0, 1, 2])
@pytest.mark.parametrize("name", ["heat3d_q4_dg1_brick", "wave3d_q3_cgp2_brick", "heat3d_q2_dg1_c4_brick",
                                  "heat3d_q2_dg1_long", "heat3d_q2_dg1_pert", "heat2d_q2_dg1"])
def test_kernel_paths(name, path):
    """Operator, smoother (exact and separable blocks where the mesh allows) and V-cycle through each
    way of summing cell contributions: bricks (0, Cartesian 3D levels), per-cell buffers (1) and
    2^d colour launches (2), against the oracle."""
    cfg, verts, coef = problem(name)
    print(f"case {name} path {path}", flush=True)
    op = oracle_op(cfg, verts, coef)
    rng = np.random.default_rng(51)
    x = rng.standard_normal((cfg.n_t, cfg.n_x))
    ref = op.apply(x)
    variants = [0] if verts is not None else [0, 1]
    for av in variants:
        H = mg.Hierarchy(op, n_smooth=cfg.n_smooth, asm_variant=av, omega_rule=-1.0)
        lev = H.levels[-1]
        b = rng.standard_normal(lev.S.shape[0])
        x0 = rng.standard_normal(lev.S.shape[0])
        omega = 0.37
        sref = mg.smooth(lev, b, x0, 2, omega=omega)
        r = rng.standard_normal(lev.S.shape[0])
        vref = H.vcycle(r)
        with _handle(cfg, verts, coef, omega=-1.0, asm_variant=av, kernel_path=path) as h:
            L = h.info["n_levels"]
            for dt, tol in ((torch.float64, 1e-12), (torch.float32, 2e-5)):
                y = torch.empty(x.size, dtype=dt, device=DEV)
                h.vmult(_t(x, dt).view(-1), y)
                assert rel_err(_np(y), ref) < tol, (dt, "vmult")
            h.set_omega(0, omega)
            for dt, tol in ((torch.float64, 1e-11), (torch.float32, 2e-4)):
                xs = _t(x0, dt)
                h.smooth(_t(b, dt), xs, steps=2, level=0)
                assert rel_err(_np(xs), sref) < tol, (dt, "smooth", av)
            for l in range(L - 1):
                h.set_omega(l, H.levels[L - 1 - l].omega)
            for dt, tol in ((torch.float64, 1e-10), (torch.float32, 1e-4)):
                z = torch.empty(r.size, dtype=dt, device=DEV)
                h.vcycle(_t(r, dt), z)
                assert rel_err(_np(z), vref) < tol, (dt, "vcycle", av)


@pytest.mark.parametrize("name", BRICK_CASES)
def test_brick_operator_levels(name):
    """Every level's operator of a Cartesian hierarchy (bricks on the finest and p-levels, the
    general kernel on h-levels, where the coefficient varies inside a cell) against the oracle, and
    the brick path bitwise equal between two handles."""
    cfg, verts, coef = problem(name)
    op = oracle_op(cfg, verts, coef)
    H = mg.Hierarchy(op, omegas=[1.0] * 16)
    L = len(H.levels)
    rng = np.random.default_rng(52)
    with _handle(cfg, verts, coef, omega=0.5) as h, _handle(cfg, verts, coef, omega=0.5) as h2:
        for l in range(L):
            S = H.levels[L - 1 - l].S
            xv = rng.standard_normal(S.shape[0])
            y = torch.empty(xv.size, dtype=torch.float64, device=DEV)
            h.vmult(_t(xv), y, level=l)
            assert rel_err(_np(y), S @ xv) < 1e-12, l
            y2 = torch.empty_like(y)
            h2.vmult(_t(xv), y2, level=l)
            assert torch.equal(y, y2), l
