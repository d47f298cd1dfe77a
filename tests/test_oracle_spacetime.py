"""Pins of the oracle's slab operator and right-hand sides (Sections 2.1-2.2, 5.1)."""
import json
import os

import numpy as np
import pytest

from oracle import basis, norms, rhs, spacetime, spatial, temporal
from stmg_inputs import Config, draw_problem, paper_config, random_slab_vector

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_paper_dof_counts():
    # lattice and temporal DoF conventions reproduce the counts printed in Table tab:iter-wave-hc
    data = json.load(open(os.path.join(GOLDEN, "paper_dof_counts.json")))
    for row in data["rows"]:
        method = 0 if row["method"] == "dG" else 1
        cfg = Config(dim=3, p=row["k"] + 1, k=row["k"], time_method=method,
                     n_cells=(row["cells"],) * 3, n_time_cells=row["time_cells"])
        assert cfg.n_x == row["dofs_space"]
        assert cfg.n_t == row["dofs_time_per_cell"] * row["time_cells"]
        assert cfg.n_st == row["dofs_global"]


def _brute_heat_dg(space, k, c, tau):
    """Dense slab matrix from the variational form of eq. var-heat-dg, integrated directly.

    Unknown (m, i, a) <-> coefficient of phi_a(x) xi_i(t) on time cell m; test (m, j, b).
    Space integrals by a (p+3)-point rule, time integrals by a (k+3)-point rule,
    jump terms from the one-sided limits.  Dirichlet rows/cols replaced by identity.
    """
    M, A = spatial.assemble(space)          # recomputed below with a higher-order rule
    xi, W, Phi, G = spatial.reference_tables(space.p, space.dim, nq=space.p + 3)
    J = spatial.jacobians(space, xi)
    det = np.linalg.det(J)
    Jinv = np.linalg.inv(J)
    rho = space.coef_at(xi)
    dofs = space.cell_dofs()
    N = space.n_x
    Mx = np.zeros((N, N))
    Ax = np.zeros((N, N))
    for K in range(space.n_cells):
        gphys = np.einsum("qji,jqa->qia", Jinv[K], np.array(G))     # J^{-T} grad_ref
        mk = np.einsum("qa,q,qb->ab", Phi, W * det[K], Phi)
        ak = np.einsum("qia,q,qib->ab", gphys, W * det[K] * rho[K], gphys)
        idx = dofs[K]
        Mx[np.ix_(idx, idx)] += mk
        Ax[np.ix_(idx, idx)] += ak
    nodes = basis.gauss_radau_right(k + 1)
    tq, tw = basis.gauss(k + 3)
    V, D = basis.lagrange(nodes, tq)
    V0, _ = basis.lagrange(nodes, np.array([0.0]))
    V1, _ = basis.lagrange(nodes, np.array([1.0]))
    nt = k + 1
    S = np.zeros((c * nt * N, c * nt * N))
    for m in range(c):
        for j in range(nt):           # test temporal
            for i in range(nt):       # trial temporal
                dt_term = np.sum(tw * D[:, i] * V[:, j])            # int xi_i' xi_j dt-hat
                mass_t = tau * np.sum(tw * V[:, i] * V[:, j])      # int xi_i xi_j dt
                jump = V0[0, i] * V0[0, j]                          # u^+ w^+ at t_{m-1}
                blk = dt_term * Mx + mass_t * Ax + jump * Mx
                r = (m * nt + j) * N
                cidx = (m * nt + i) * N
                S[r:r + N, cidx:cidx + N] += blk
                if m > 0:
                    prev = -V1[0, i] * V0[0, j]                     # -u^-_{m-1} w^+
                    cp = ((m - 1) * nt + i) * N
                    S[r:r + N, cp:cp + N] += prev * Mx
    bm = np.tile(space.boundary_mask(), c * nt)
    S[bm, :] = 0.0
    S[:, bm] = 0.0
    S[bm, bm] = 1.0
    return S


@pytest.mark.parametrize("dim,perturb", [(2, 0.1), (3, 0.0)])
def test_slab_matrix_matches_variational_form(dim, perturb):
    cfg = Config(dim=dim, p=2, k=1, n_time_cells=2, n_cells=(2, 2, 2 if dim == 3 else 1),
                 tau=0.3, perturb=perturb, coef="lognormal", coef_sigma=0.7, seed=9)
    verts, coef = draw_problem(cfg)
    op = spacetime.from_config(cfg, verts, coef)
    S = op.matrix().toarray()
    Sb = _brute_heat_dg(op.space, cfg.k, cfg.n_time_cells, cfg.tau)
    if perturb:
        # (p+1)-point Gauss is not exact on perturbed cells: agreement to quadrature error only
        assert np.abs(S - Sb).max() < 2e-3 * np.abs(Sb).max()
    else:
        assert np.allclose(S, Sb, atol=1e-12)


def test_apply_matches_matrix():
    cfg = Config(dim=3, problem=1, time_method=1, p=3, k=2, n_time_cells=3, n_cells=(2, 3, 2),
                 tau=0.1, perturb=0.1, coef="lognormal", coef_sigma=1.0, seed=4)
    verts, coef = draw_problem(cfg)
    op = spacetime.from_config(cfg, verts, coef)
    x = np.random.default_rng(0).standard_normal((cfg.n_t, cfg.n_x))
    assert np.allclose(op.apply(x).ravel(), op.matrix() @ x.ravel(), atol=1e-12)


def test_heat_eoc_config1_family():
    # u = sin(pi x) sin(pi y) sin(pi t): L2(L2) error decreases at rate min(p+1, k+1) = 2
    pi = np.pi
    f = lambda x, t: (pi * np.cos(pi * t) + 2 * pi ** 2 * np.sin(pi * t)) * np.sin(pi * x[..., 0]) * np.sin(pi * x[..., 1])
    ue = lambda x, t: np.sin(pi * t) * np.sin(pi * x[..., 0]) * np.sin(pi * x[..., 1])
    errs = []
    for n in (4, 8, 16):
        cfg = paper_config(1).replace(n_cells=(n, n, 1), tau=1.0 / n, n_time_cells=n)
        op = spacetime.from_config(cfg, None, np.ones(n * n))
        b = rhs.rhs(op, rhs.loads(op.space, f, op.slab.times))
        U = op.solve(b)
        errs.append(norms.l2l2_error(op, U, ue, cfg.k))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert errs[-1] < 1e-3
    assert np.all(rates > 1.9) and np.all(rates < 2.2)


def test_heat_cgp_eoc():
    # cGP(2) with Q3: rate min(p+1, k+1) = 3 when h and tau are refined together
    pi = np.pi
    f = lambda x, t: (pi * np.cos(pi * t) + 2 * pi ** 2 * np.sin(pi * t)) * np.sin(pi * x[..., 0]) * np.sin(pi * x[..., 1])
    ue = lambda x, t: np.sin(pi * t) * np.sin(pi * x[..., 0]) * np.sin(pi * x[..., 1])
    errs = []
    for n in (4, 8):
        cfg = Config(dim=2, problem=0, time_method=1, p=3, k=2, n_cells=(n, n, 1), tau=1.0 / n,
                     n_time_cells=n)
        op = spacetime.from_config(cfg, None, np.ones(n * n))
        F = rhs.loads(op.space, f, op.slab.times)
        F0 = rhs.loads(op.space, f, np.array([0.0]))[0]
        U = op.solve(rhs.rhs(op, F, F0=F0))
        errs.append(norms.l2l2_error(op, U, ue, cfg.k))
    rate = np.log2(errs[0] / errs[1])
    assert 2.7 < rate < 3.4


def test_wave_cgp_conserves_energy():
    # f = 0: cGP(k) conserves E = (v^T M v + u^T A u)/2 at every time-cell end (Lobatto IIIA)
    cfg = Config(dim=2, problem=1, time_method=1, p=2, k=2, n_cells=(4, 4, 1), tau=0.05,
                 n_time_cells=6, coef="lognormal", coef_sigma=1.0, perturb=0.1, seed=5)
    verts, coef = draw_problem(cfg)
    op = spacetime.from_config(cfg, verts, coef)
    X = spatial.node_coordinates(op.space)
    u0 = np.sin(np.pi * X[:, 0]) * np.sin(2 * np.pi * X[:, 1])
    u0[op.bmask] = 0.0
    v0 = np.zeros(op.n_x)
    b = rhs.rhs(op, np.zeros((cfg.n_t, op.n_x)), F0=np.zeros(op.n_x), u0=u0, v0=v0)
    U = op.solve(b)
    V = rhs.velocity(op, U, u0=u0, v0=v0)
    E0 = norms.wave_energy(op, u0, v0)
    nc = op.slab.nt_cell
    for m in range(cfg.n_time_cells):
        e = norms.wave_energy(op, U[(m + 1) * nc - 1], V[(m + 1) * nc - 1])
        assert abs(e - E0) < 1e-11 * E0


def test_wave_dg_energy_decays():
    cfg = Config(dim=2, problem=1, time_method=0, p=2, k=1, n_cells=(4, 4, 1), tau=0.05,
                 n_time_cells=4)
    op = spacetime.from_config(cfg, None, np.ones(16))
    X = spatial.node_coordinates(op.space)
    u0 = np.sin(np.pi * X[:, 0]) * np.sin(np.pi * X[:, 1])
    b = rhs.rhs(op, np.zeros((cfg.n_t, op.n_x)), u0=u0)
    U = op.solve(b)
    V = rhs.velocity(op, U, u0=u0)
    E = [norms.wave_energy(op, u0, np.zeros(op.n_x))]
    for m in range(cfg.n_time_cells):
        E.append(norms.wave_energy(op, U[2 * m + 1], V[2 * m + 1]))
    assert all(E[i + 1] <= E[i] * (1 + 1e-12) for i in range(len(E) - 1))
    assert E[-1] < E[0]


@pytest.mark.parametrize("problem,method", [(0, 0), (1, 1), (0, 1), (1, 0)])
def test_slab_equals_stepping(problem, method):
    # one slab of c cells equals c chained one-cell slabs (initial data passed along)
    cfg = Config(dim=2, problem=problem, time_method=method, p=2, k=2, n_cells=(3, 3, 1),
                 tau=0.07, n_time_cells=3, coef="lognormal", coef_sigma=0.5, seed=8)
    verts, coef = draw_problem(cfg)
    op = spacetime.from_config(cfg, verts, coef)
    X = spatial.node_coordinates(op.space)
    u0 = np.sin(np.pi * X[:, 0]) * np.sin(np.pi * X[:, 1]) * (~op.bmask)
    v0 = np.cos(np.pi * X[:, 0]) * np.sin(np.pi * X[:, 1]) * (~op.bmask) if problem == 1 else None
    f = lambda x, t: np.exp(t) * x[..., 0] * (1 - x[..., 0])
    F = rhs.loads(op.space, f, op.slab.times)
    F0 = rhs.loads(op.space, f, np.array([0.0]))[0]
    U = op.solve(rhs.rhs(op, F, F0=F0, u0=u0, v0=v0))
    one = cfg.replace(n_time_cells=1)
    nc = op.slab.nt_cell
    uc, vc, fprev = u0, v0, F0
    for m in range(3):
        o1 = spacetime.from_config(one.replace(t0=m * cfg.tau), verts, coef)
        F1 = rhs.loads(o1.space, f, o1.slab.times)
        U1 = o1.solve(rhs.rhs(o1, F1, F0=fprev, u0=uc, v0=vc))
        assert np.allclose(U1, U[m * nc:(m + 1) * nc], atol=1e-11)
        if problem == 1:
            vc = rhs.velocity(o1, U1, u0=uc, v0=vc)[-1]
        uc = U1[-1]
        fprev = F1[-1]


def test_solve_residual():
    cfg = Config(dim=3, p=2, k=1, n_cells=(3, 3, 3), n_time_cells=2, tau=0.1, perturb=0.1,
                 coef="lognormal", coef_sigma=1.0, seed=6)
    verts, coef = draw_problem(cfg)
    op = spacetime.from_config(cfg, verts, coef)
    b = random_slab_vector(cfg, 1)
    U = op.solve(b)
    assert np.linalg.norm(op.apply(U) - b) < 1e-12 * np.linalg.norm(b)
    assert np.all(U[:, op.bmask] == 0.0)
