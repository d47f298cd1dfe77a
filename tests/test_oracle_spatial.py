"""Pins of the oracle's spatial Q_p matrices (Section 2, eq. space-matrices)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import spatial
from stmg_inputs import Config, draw_problem
from oracle.spacetime import fine_space


def _space(dim, n, p, perturb=0.0, coef="one", sigma=0.0, seed=3):
    cfg = Config(dim=dim, p=p, n_cells=(n, n, n if dim == 3 else 1), perturb=perturb, coef=coef,
                 coef_sigma=sigma, seed=seed)
    verts, rho = draw_problem(cfg)
    return fine_space(cfg, verts, rho)


def _global_1d(n, p, elem_M, elem_A):
    N = p * n + 1
    M = np.zeros((N, N))
    A = np.zeros((N, N))
    for c in range(n):
        s = slice(c * p, c * p + p + 1)
        M[s, s] += elem_M
        A[s, s] += elem_A
    return M, A


def test_q1_q2_match_textbook_kronecker():
    # Cartesian, rho = 1: A_h = sum_d A1 (x) M1 (x) ..., M_h = M1 (x) M1 (x) M1 with textbook 1D matrices
    n = 3
    h = 1.0 / n
    tb = {1: (h / 6 * np.array([[2, 1], [1, 2]]), 1 / h * np.array([[1, -1], [-1, 1]])),
          2: (h / 30 * np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]]),
              1 / (3 * h) * np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]))}
    for p in (1, 2):
        M1, A1 = _global_1d(n, p, *tb[p])
        for dim in (2, 3):
            sp_ = _space(dim, n, p)
            M, A = spatial.assemble(sp_)
            if dim == 2:
                Mref = np.kron(M1, M1)
                Aref = np.kron(M1, A1) + np.kron(A1, M1)
            else:
                Mref = np.kron(M1, np.kron(M1, M1))
                Aref = (np.kron(M1, np.kron(M1, A1)) + np.kron(M1, np.kron(A1, M1))
                        + np.kron(A1, np.kron(M1, M1)))
            assert np.allclose(M.toarray(), Mref, atol=1e-14)
            assert np.allclose(A.toarray(), Aref, atol=1e-12)


@pytest.mark.parametrize("dim,p", [(2, 2), (2, 4), (3, 2), (3, 3)])
def test_symmetry_definiteness_volume(dim, p):
    sp_ = _space(dim, 3, p, perturb=0.1, coef="lognormal", sigma=1.0)
    M, A = spatial.assemble(sp_)
    Md, Ad = M.toarray(), A.toarray()
    assert np.allclose(Md, Md.T, atol=1e-15) and np.allclose(Ad, Ad.T, atol=1e-13)
    assert np.linalg.eigvalsh(Md).min() > 0
    assert np.linalg.eigvalsh(Ad).min() > -1e-12
    one = np.ones(sp_.n_x)
    assert abs(one @ Md @ one - 1.0) < 1e-13          # |Omega| = 1 (boundary vertices fixed)
    assert np.abs(Ad @ one).max() < 1e-12              # constants lie in the kernel


@pytest.mark.parametrize("dim,p", [(2, 1), (2, 3), (3, 2), (3, 4)])
def test_patch_test_perturbed(dim, p):
    # the interpolant of a global linear function is exact on multilinear cells:
    # interior rows of A_h x vanish and x^T A_h x = |grad u|^2 |Omega| (rho = 1)
    sp_ = _space(dim, 3, p, perturb=0.1)
    M, A = spatial.assemble(sp_)
    X = spatial.node_coordinates(sp_)
    c = np.array([0.3, -1.1, 0.7])[:dim]
    u = X @ c + 0.25
    r = A @ u
    interior = ~sp_.boundary_mask()
    assert np.abs(r[interior]).max() < 1e-12
    assert abs(u @ r - c @ c) < 1e-12


def test_polynomial_moments_cartesian():
    # M_h integrates products of Q_p functions exactly on Cartesian cells
    sp_ = _space(3, 2, 2)
    M, _ = spatial.assemble(sp_)
    X = spatial.node_coordinates(sp_)
    u = X[:, 0] ** 2 * X[:, 1]
    one = np.ones(sp_.n_x)
    assert abs(u @ M @ one - (1 / 3) * (1 / 2)) < 1e-14
    assert abs(u @ M @ u - (1 / 5) * (1 / 3)) < 1e-14


def test_coarse_coefficient_lookup():
    # at ratio 2 the quadrature points of a coarse cell fall into its four/eight children
    sp_ = _space(2, 4, 1, coef="lognormal", sigma=1.0)
    coarse = spatial.Space(dim=2, cells=(2, 2), p=1, verts=None, lo=sp_.lo, hi=sp_.hi,
                           coef_fine=sp_.coef_fine, fine_cells=(4, 4), ratio=2)
    xi = np.array([[0.2, 0.2], [0.8, 0.2], [0.2, 0.8], [0.8, 0.8]])
    got = coarse.coef_at(xi)
    f = sp_.coef_fine.reshape(4, 4)
    assert np.allclose(got[0], [f[0, 0], f[0, 1], f[1, 0], f[1, 1]])
    assert np.allclose(got[3], [f[2, 2], f[2, 3], f[3, 2], f[3, 3]])


def test_point_values_reproduce_polynomials():
    # the Q_p interpolant of a polynomial of degree <= p in each variable is exact everywhere
    from oracle import norms
    from stmg_inputs import Config, draw_problem
    cfg = Config(dim=3, p=2, n_cells=(3, 2, 4), lo=(-1.0, 0.0, 0.5), hi=(1.0, 1.0, 1.5))
    verts, coef = draw_problem(cfg)
    space = fine_space(cfg, verts, coef)
    X = spatial.node_coordinates(space)
    f = lambda P: (1 + P[:, 0] - 2 * P[:, 0] ** 2) * (0.5 + P[:, 1] ** 2) * (2 - P[:, 2] + P[:, 2] ** 2)
    rng = np.random.default_rng(3)
    pts = np.stack([rng.uniform(lo, hi, 20) for lo, hi in zip(cfg.lo, cfg.hi)], axis=1)
    assert np.allclose(norms.point_values(space, f(X), pts), f(pts), rtol=1e-12, atol=1e-12)
