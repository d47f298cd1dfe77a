"""Pins of the oracle's norms and loads: the L2(L2) error of eq. norms (zero for the interpolant
of a space-time polynomial of the discrete degrees, the closed-form norm for the zero solution),
the discrete wave energy of an exactly represented field, and the spatial load vectors of the
slab right-hand sides (partition of unity; mass matrix times nodal values for f in Q_p)."""
import numpy as np
import pytest

from oracle import norms, spacetime, spatial, temporal
from stmg_inputs import Config, draw_problem


def _op(method, p, k, c, cells=(3, 2, 1)):
    cfg = Config(dim=2, problem=0, time_method=method, p=p, k=k, n_time_cells=c, n_cells=cells, tau=0.25,
                 t0=0.5, perturb=0.0, seed=3)
    verts, coef = draw_problem(cfg)
    return cfg, spacetime.from_config(cfg, verts, coef)


@pytest.mark.parametrize("method,p,k", [(0, 2, 2), (0, 3, 1), (1, 2, 2), (1, 1, 3)])
def test_interpolant_of_discrete_polynomial_has_zero_error(method, p, k):
    cfg, op = _op(method, p, k, 3)
    # degree p in each space direction, degree k (dG) or k (cGP trial degree) in time
    tk = k
    u = lambda x, t: (1.0 + x[..., 0] - 0.7 * x[..., 0] ** p) * (0.5 + x[..., 1] ** p) * (1.0 + 0.3 * t ** tk - t)
    X = spatial.node_coordinates(op.space)
    U = np.stack([u(X, t) for t in op.slab.times])
    u0 = u(X, cfg.t0) if method == 1 else None
    scale = norms.l2l2_error(op, np.zeros_like(U), u, k, u0=None if method == 0 else np.zeros(op.n_x))
    err = norms.l2l2_error(op, U, u, k, u0=u0)
    assert scale > 0.1
    assert err < 1e-12 * scale


@pytest.mark.parametrize("method,k", [(0, 1), (1, 2)])
def test_zero_solution_error_is_the_exact_norm(method, k):
    cfg, op = _op(method, 2, k, 4)
    lo, hi = np.array(cfg.lo[:2], float), np.array(cfg.hi[:2], float)
    t0, t1 = cfg.t0, cfg.t0 + cfg.n_time_cells * cfg.tau
    u = lambda x, t: x[..., 0] * t
    exact = np.sqrt((hi[0] ** 3 - lo[0] ** 3) / 3.0 * (hi[1] - lo[1]) * (t1 ** 3 - t0 ** 3) / 3.0)
    U = np.zeros((op.n_t, op.n_x))
    got = norms.l2l2_error(op, U, u, k, u0=np.zeros(op.n_x) if method == 1 else None)
    assert got == pytest.approx(exact, rel=1e-13)


@pytest.mark.parametrize("cells", [(2, 2, 1), (3, 5, 1)])
def test_wave_energy_closed_form(cells):
    # u = v = x(1-x) y(1-y) lies in Q2 and vanishes on the boundary of the unit square, so the
    # discrete energy (v^T M v + u^T A u) / 2 is the exact (int v^2 + int |grad u|^2) / 2
    # = (1/900 + 1/45) / 2 = 21/1800 (coefficient 1)
    cfg = Config(dim=2, problem=1, time_method=1, p=2, k=2, n_time_cells=1, n_cells=cells, tau=0.1)
    verts, coef = draw_problem(cfg)
    op = spacetime.from_config(cfg, verts, coef)
    X = spatial.node_coordinates(op.space)
    u = X[:, 0] * (1 - X[:, 0]) * X[:, 1] * (1 - X[:, 1])
    assert norms.wave_energy(op, u, u) == pytest.approx(21.0 / 1800.0, rel=1e-12)
    assert norms.wave_energy(op, u, np.zeros_like(u)) == pytest.approx(1.0 / 90.0, rel=1e-12)


@pytest.mark.parametrize("dim,p,perturb", [(2, 1, 0.15), (2, 3, 0.1), (3, 2, 0.1)])
def test_loads_partition_of_unity(dim, p, perturb):
    # the nodal basis sums to one and the boundary of the box is not perturbed, so the loads of
    # f = 1 + x0 x1 sum to its integral over the unit box, 1 + 1/4, at every time (the Gauss rule
    # is exact for this integrand on bilinear or trilinear cells)
    from oracle import rhs
    cells = (3, 2, 2) if dim == 3 else (3, 4, 1)
    cfg = Config(dim=dim, problem=0, time_method=0, p=p, k=0, n_time_cells=1, n_cells=cells, tau=0.1,
                 perturb=perturb, seed=8)
    verts, coef = draw_problem(cfg)
    op = spacetime.from_config(cfg, verts, coef)
    f = lambda x, t: (1.0 + x[..., 0] * x[..., 1]) * (1.0 + t)
    F = rhs.loads(op.space, f, np.array([0.0, 2.0]))
    assert F.sum(axis=1) == pytest.approx([1.25, 3.75], rel=1e-12)


@pytest.mark.parametrize("p", [1, 2, 4])
def test_loads_of_a_discrete_field_are_mass_times_nodal_values(p):
    # for f in Q_p the load vector is the assembled mass matrix applied to f's nodal values
    from oracle import rhs
    cfg = Config(dim=2, problem=0, time_method=0, p=p, k=0, n_time_cells=1, n_cells=(3, 2, 1), tau=0.1)
    verts, coef = draw_problem(cfg)
    op = spacetime.from_config(cfg, verts, coef)
    f = lambda x, t: (2.0 - x[..., 0] ** p) * (1.0 + 3.0 * x[..., 1] ** p)
    X = spatial.node_coordinates(op.space)
    M, _ = spatial.assemble(op.space)
    F = rhs.loads(op.space, f, np.array([0.0]))[0]
    ref = M @ f(X, 0.0)
    assert np.allclose(F, ref, rtol=0, atol=1e-14 * np.abs(ref).max())
