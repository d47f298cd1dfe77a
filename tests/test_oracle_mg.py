"""Pins of the oracle's multigrid parts (Section 3: transfers, ASM smoother, V-cycle)."""
import numpy as np
import pytest

from oracle import krylov, mg, spacetime, spatial, temporal
from stmg_inputs import Config, draw_problem, random_slab_vector, small_configs


def _op(cfg):
    verts, coef = draw_problem(cfg)
    return spacetime.from_config(cfg, verts, coef)


@pytest.mark.parametrize("dim,pc,pf,hc,hf", [(2, 1, 2, 3, 3), (3, 2, 4, 2, 2), (2, 2, 2, 2, 4),
                                             (3, 1, 1, 2, 4), (3, 1, 3, 2, 2)])
def test_prolongation_reproduces_coarse_polynomials(dim, pc, pf, hc, hf):
    # nested spaces: interpolating a Q_pc polynomial on the coarse lattice and prolongating
    # gives the fine-lattice interpolant of the same polynomial
    cells_c, cells_f = (hc,) * dim, (hf,) * dim
    one = np.ones(int(np.prod(cells_f)))
    fine = spatial.Space(dim, cells_f, pf, None, (0,) * dim, (1,) * dim, one, cells_f, 1)
    coarse = spatial.Space(dim, cells_c, pc, None, (0,) * dim, (1,) * dim, one, cells_f, hf // hc)
    P = mg.prolongation(coarse, fine)
    rng = np.random.default_rng(1)
    coeff = rng.standard_normal((pc + 1,) * dim)

    def poly(X):
        val = np.zeros(len(X))
        for idx in np.ndindex(*coeff.shape):
            term = coeff[idx] * np.ones(len(X))
            for d in range(dim):
                term = term * X[:, d] ** idx[d]
            val += term
        return val

    uc = poly(spatial.node_coordinates(coarse))
    uf = poly(spatial.node_coordinates(fine))
    assert np.allclose(P @ uc, uf, atol=1e-12)
    # partition of unity
    assert np.allclose(P @ np.ones(coarse.n_x), 1.0, atol=1e-13)


def test_restriction_is_adjoint():
    cfg = small_configs()[1]
    op = _op(cfg)
    H = mg.Hierarchy(op, omegas=[1.0] * 3)
    rng = np.random.default_rng(2)
    for i in range(1, len(H.levels)):
        nf = H.levels[i].S.shape[0]
        nc = H.levels[i - 1].S.shape[0]
        x = rng.standard_normal(nc)
        y = rng.standard_normal(nf)
        assert abs(H.prolong(i, x) @ y - x @ H.restrict(i, y)) < 1e-11 * np.sqrt(nf)


@pytest.mark.parametrize("method,problem", [(0, 0), (1, 1)])
def test_asm_single_cell_is_exact(method, problem):
    # one spatial cell and one time cell: the ASM block is the whole interior system
    cfg = Config(dim=3, problem=problem, time_method=method, p=3, k=2, n_time_cells=1,
                 n_cells=(1, 1, 1), tau=0.2, perturb=0.0)
    op = _op(cfg)
    lev = mg.Level(op=op, S=op.matrix())
    lev.blocks = mg.asm_blocks(op, lev.S)
    b = random_slab_vector(cfg, 3)
    u = mg.smooth(lev, b, np.zeros_like(b), 1, omega=1.0)
    assert np.allclose(u, op.solve(b).ravel(), atol=1e-12)


def test_asm_block_sizes():
    # block size (k+1)(p+1)^d for dG(k) and k(p+1)^d for cGP(k) on interior cells (Section 3.3)
    for method, k, per in [(0, 2, 3), (1, 2, 2)]:
        cfg = Config(dim=3, time_method=method, k=k, p=2, n_time_cells=2, n_cells=(3, 3, 3), tau=0.1)
        op = _op(cfg)
        blocks = mg.asm_blocks(op, op.matrix())
        assert max(len(idx) for idx, _ in blocks) == per * 27
        assert len(blocks) == 27 * 2


def test_asm_blocks_are_principal_submatrices():
    cfg = Config(dim=2, time_method=1, problem=1, k=2, p=2, n_time_cells=3, n_cells=(3, 3, 1),
                 tau=0.1, perturb=0.1, coef="lognormal", coef_sigma=1.0, seed=2)
    op = _op(cfg)
    S = op.matrix().toarray()
    blocks = mg.asm_blocks(op, op.matrix())
    for idx, inv in blocks[::5]:
        assert np.allclose(inv @ S[np.ix_(idx, idx)], np.eye(len(idx)), atol=1e-10)
        # the same spatial cell gives the same block in every time cell (M_tau, N~ repeat)
    Nx = op.n_x
    b0 = [b for b in blocks if b[0][0] // Nx < 2]
    b2 = [b for b in blocks if b[0][0] // Nx >= 4]
    assert np.allclose(b0[0][1], b2[0][1], atol=1e-12)


@pytest.mark.parametrize("ci", [0, 1, 2])
def test_vcycle_fgmres_reaches_direct_solution(ci):
    cfg = small_configs()[ci]
    op = _op(cfg)
    H = mg.Hierarchy(op, n_smooth=1)
    assert all(0 < w <= 1 for w in H.omegas)
    b = random_slab_vector(cfg, 5)
    x, it, rr = krylov.fgmres(op.apply, b, H.vcycle, rtol=1e-11, restart=40, max_iter=200)
    xd = op.solve(b)
    assert rr <= 1e-11
    assert np.linalg.norm(x - xd.ravel()) <= 1e-9 * np.linalg.norm(xd)
    assert it < 60


def test_vcycle_is_linear_and_reduces_error():
    cfg = small_configs()[1]
    op = _op(cfg)
    H = mg.Hierarchy(op, n_smooth=2)
    b1 = random_slab_vector(cfg, 1)
    b2 = random_slab_vector(cfg, 2)
    z = H.vcycle(2.0 * b1 - 3.0 * b2)
    assert np.allclose(z, 2.0 * H.vcycle(b1) - 3.0 * H.vcycle(b2), atol=1e-10)
    # as a stationary iteration x <- x + V(b - S x) the error contracts
    xd = op.solve(b1).ravel()
    x = np.zeros_like(xd)
    e0 = np.linalg.norm(xd)
    for _ in range(6):
        x = x + H.vcycle(b1.ravel() - op.apply(x))
    assert np.linalg.norm(x - xd) < 0.5 * e0


def test_separable_blocks_exact_for_constant_coefficient():
    # Cartesian mesh, constant coefficient: the assembled operator is a Kronecker product, so the
    # separable surrogate is the exact principal block (Section 3.3 blocks, fast diagonalisation)
    for cfg in [Config(dim=3, problem=0, time_method=0, p=2, k=1, n_time_cells=2, n_cells=(3, 2, 3),
                          tau=0.05, coef="one", seed=3),
                Config(dim=2, problem=1, time_method=1, p=3, k=2, n_time_cells=2, n_cells=(3, 4, 1),
                          tau=0.05, coef="one", seed=4)]:
        verts, coef = draw_problem(cfg)
        op = spacetime.from_config(cfg, verts, coef * 2.5)
        exact = mg.asm_blocks(op, op.matrix())
        fdm = mg.fdm_blocks(op)
        assert len(exact) == len(fdm)
        for (i1, b1), (i2, b2) in zip(exact, fdm):
            assert np.array_equal(i1, i2)
            assert np.allclose(b1, b2, rtol=1e-10, atol=1e-10 * np.abs(b1).max())


def test_separable_blocks_use_cell_mean_coefficient():
    # a variable coefficient changes the surrogate only through rho_K: scaling one cell's
    # coefficient scales the spatial stiffness part of its block (checked on a 1-cell mesh)
    cfg = Config(dim=3, problem=0, time_method=0, p=2, k=0, n_time_cells=1, n_cells=(1, 1, 1), tau=1.0,
                    coef="one", seed=5)
    verts, coef = draw_problem(cfg)
    op1 = spacetime.from_config(cfg, verts, coef)
    op3 = spacetime.from_config(cfg, verts, 3.0 * coef)
    (i1, b1), = mg.fdm_blocks(op1)
    (i3, b3), = mg.fdm_blocks(op3)
    # dG(0): block = tau-mass term + (A_tau = 1) * M: B = M_tau A~ + N~ M~ with M_tau = tau = 1
    B1, B3 = np.linalg.inv(b1), np.linalg.inv(b3)
    Mt = op1.Mi.toarray()[np.ix_(i1, i1)]
    assert np.allclose(B3 - Mt, 3.0 * (B1 - Mt), rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("method", [0, 1])
def test_time_multigrid_hierarchy_solves(method):
    # spatial levels, then k- and tau-levels on the coarsest mesh (Section 3.2): the V-cycle
    # as FGMRES preconditioner reaches the direct solve
    cfg = Config(dim=2, problem=1, time_method=method, p=2, k=2, n_time_cells=4, n_cells=(4, 4, 1),
                 tau=0.05, coef="lognormal", coef_sigma=0.5, seed=61)
    verts, coef = draw_problem(cfg)
    op = spacetime.from_config(cfg, verts, coef)
    H = mg.Hierarchy(op, omega_rule=-1.0, time_mg=True)
    kinds = [lev.Pt is not None for lev in H.levels[1:]]
    assert any(kinds) and not all(kinds)
    assert H.levels[0].op.slab.n_t < op.slab.n_t
    b = random_slab_vector(cfg, 3).ravel()
    S = op.matrix()
    x, it, rel = krylov.fgmres(lambda v: S @ v, b, H.vcycle, rtol=1e-12, restart=40, max_iter=200)
    assert rel <= 1e-12
    assert np.linalg.norm(x - op.solve(b).ravel()) <= 1e-9 * np.linalg.norm(x)


@pytest.mark.parametrize("problem,method,k,c,perturb", [(0, 0, 2, 1, 0.0), (1, 1, 2, 1, 0.15), (0, 0, 1, 1, 0.15)])
def test_omega_estimate_is_exact_on_tiny_levels(problem, method, k, c, perturb):
    # With no more interior DoFs than Arnoldi steps, the Krylov space of ASM * S (started on the
    # interior) is the whole interior space, so the Ritz values are the eigenvalues of ASM * S
    # there (eq. relaxation); they are compared with a dense eigen-solve of the same product
    cfg = Config(dim=2, problem=problem, time_method=method, p=1, k=k, n_time_cells=c, n_cells=(3, 3, 1),
                 tau=0.1, perturb=perturb, coef="lognormal", coef_sigma=0.4, seed=29)
    op = _op(cfg)
    lev = mg.Level(op=op, S=op.matrix())
    lev.blocks = mg.asm_blocks(op, lev.S)
    inner = np.flatnonzero(~np.tile(op.bmask, op.n_t))
    assert 0 < inner.size <= 15
    n = op.n_t * op.n_x
    cols = []
    for g in inner:
        e = np.zeros(n)
        e[g] = 1.0
        cols.append(mg.asm_apply(lev, lev.S @ e)[inner])
    # S is not symmetric (time stepping), so the eigenvalues come in complex pairs; the rule
    # takes their real parts
    ev = np.linalg.eigvals(np.array(cols).T)
    lmax, lmin = ev.real.max(), ev.real.min()
    assert 0.0 < lmin <= lmax
    w_bal = 2.0 / (lmax + lmin)
    w_top = 1.5 / lmax
    assert mg.estimate_omega(lev, rule=0.0) == pytest.approx(min(max(w_bal, 1e-3), 1.0), rel=1e-10)
    assert mg.estimate_omega(lev, rule=-1.5) == pytest.approx(min(max(w_top, 1e-3), 1.0), rel=1e-10)
    assert w_top < 1.0          # the pin is not decided by the clamp


# --------------------------------------------------------------------------- vertex patches

@pytest.mark.parametrize("dim,p", [(2, 3), (3, 2)])
@pytest.mark.parametrize("method,problem", [(0, 0), (1, 1)])
def test_single_vertex_patch_is_exact(dim, p, method, problem):
    # 2^d cells and one time cell: the only interior vertex's patch holds every interior DoF, so
    # one additive Schwarz step with omega = 1 is the direct solve
    cells = (2, 2, 2) if dim == 3 else (2, 2, 1)
    cfg = Config(dim=dim, problem=problem, time_method=method, p=p, k=2, n_time_cells=1, n_cells=cells,
                 tau=0.2, perturb=0.1, coef="lognormal", coef_sigma=1.0, seed=8)
    op = _op(cfg)
    S = op.matrix()
    assert len(mg.vertex_patches(op.space)) == 1
    lev = mg.Level(op=op, S=S, blocks=mg.patch_blocks(op, S))
    b = random_slab_vector(cfg, 4)
    u = mg.smooth(lev, b, np.zeros_like(b), 1, omega=1.0)
    assert np.allclose(u, op.solve(b).ravel(), atol=1e-11)


def test_vertex_patches_cover_interior_nodes():
    # a node lies strictly inside the patch of vertex v along axis a for v_a = g_a / p when it sits
    # on a cell face (g_a % p == 0), else for v_a in {c_a, c_a + 1} (c_a its cell); the patch count
    # of a node is the product over the axes, restricted to interior vertices
    cfg = Config(dim=3, p=2, k=0, n_time_cells=1, n_cells=(3, 4, 2), tau=0.1)
    space = _op(cfg).space
    count = np.zeros(space.n_x, dtype=int)
    for v, nodes in mg.vertex_patches(space):
        assert len(nodes) == (2 * space.p - 1) ** 3
        count[nodes] += 1
    N = space.nodes
    for g in range(space.n_x):
        c = [g % N[0], (g // N[0]) % N[1], g // (N[0] * N[1])]
        if any(x == 0 or x == m - 1 for x, m in zip(c, N)):
            assert count[g] == 0
            continue
        want = 1
        for a in range(3):
            if c[a] % space.p == 0:
                want *= 1
            else:
                ca = c[a] // space.p
                want *= sum(1 for v in (ca, ca + 1) if 1 <= v <= space.cells[a] - 1)
        assert count[g] == want


def test_separable_patches_exact_for_constant_coefficient():
    # Cartesian mesh and constant coefficient: the patch operator is a Kronecker product of the
    # assembled 1D patch matrices, so the separable patch block is the exact one
    for cfg in [Config(dim=3, problem=0, time_method=0, p=2, k=1, n_time_cells=2, n_cells=(3, 2, 4),
                       tau=0.05, coef="one", seed=3),
                Config(dim=2, problem=1, time_method=1, p=3, k=2, n_time_cells=2, n_cells=(3, 4, 1),
                       tau=0.05, coef="one", seed=4)]:
        verts, coef = draw_problem(cfg)
        op = spacetime.from_config(cfg, verts, coef * 1.7)
        exact = mg.patch_blocks(op, op.matrix())
        fdm = mg.fdm_patch_blocks(op)
        assert len(exact) == len(fdm) > 0
        for (i1, b1), (i2, b2) in zip(exact, fdm):
            assert np.array_equal(i1, i2)
            assert np.allclose(b1, b2, rtol=1e-10, atol=1e-10 * np.abs(b1).max())


def test_separable_patches_use_patch_mean_coefficient():
    # scaling the coefficient of one cell of a 2^3 patch by s changes the patch's mean by (s - 1)/8
    cfg = Config(dim=3, problem=0, time_method=0, p=2, k=0, n_time_cells=1, n_cells=(2, 2, 2), tau=1.0,
                 coef="one", seed=5)
    verts, coef = draw_problem(cfg)
    c2 = coef.copy()
    c2[5] = 9.0                     # rho_mean = (7 + 9) / 8 = 2
    op1 = spacetime.from_config(cfg, verts, coef)
    op2 = spacetime.from_config(cfg, verts, c2)
    (i1, b1), = mg.fdm_patch_blocks(op1)
    (i2, b2), = mg.fdm_patch_blocks(op2)
    Mt = op1.Mi.toarray()[np.ix_(i1, i1)]
    B1, B2 = np.linalg.inv(b1), np.linalg.inv(b2)
    assert np.allclose(B2 - Mt, 2.0 * (B1 - Mt), rtol=1e-10, atol=1e-12)


def test_vertex_patch_hierarchy_solves():
    # V-cycle with exact and separable vertex patches as an FGMRES preconditioner reaches the
    # direct solution (Alg. stmg with the patch smoother on every level)
    cfg = Config(dim=3, problem=1, time_method=1, p=2, k=2, n_time_cells=2, n_cells=(4, 4, 4), tau=0.05,
                 coef="lognormal", coef_sigma=0.5, seed=9)
    op = _op(cfg)
    b = random_slab_vector(cfg, 6)
    xd = op.solve(b).ravel()
    for av in (2, 3):
        H = mg.Hierarchy(op, asm_variant=av, omega_rule=-1.5)
        x, it, rr = krylov.fgmres(op.apply, b, H.vcycle, rtol=1e-11, restart=40, max_iter=200)
        assert rr <= 1e-11 and it < 80
        assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)
