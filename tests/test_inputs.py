"""The seeded input recipe shared by the oracle and the GPU tests: determinism, and the stated
structure (interior-only vertex displacement within perturb * h, positive coefficients, layered
SHM medium, boundary-zero slab vectors)."""
import numpy as np
import pytest

import stmg_inputs as si


@pytest.mark.parametrize("idx", [1, 2, 3, 5])
def test_draws_are_deterministic(idx):
    cfg = si.paper_config(idx)
    small = cfg.replace(n_cells=tuple(min(c, 6) for c in cfg.n_cells))
    v1, c1 = si.draw_problem(small)
    v2, c2 = si.draw_problem(small)
    assert (v1 is None) == (v2 is None)
    if v1 is not None:
        assert np.array_equal(v1, v2)
    assert np.array_equal(c1, c2)
    assert np.array_equal(si.random_slab_vector(small, 4), si.random_slab_vector(small, 4))
    assert not np.array_equal(si.random_slab_vector(small, 4), si.random_slab_vector(small, 5))


@pytest.mark.parametrize("dim", [2, 3])
def test_perturbation_is_interior_and_bounded(dim):
    cells = (5, 4, 3) if dim == 3 else (5, 4, 1)
    cfg = si.Config(dim=dim, problem=0, time_method=0, p=1, k=0, n_time_cells=1, n_cells=cells, tau=0.1,
                    perturb=0.2, seed=11)
    verts, _ = si.draw_problem(cfg)
    axes = [np.linspace(cfg.lo[i], cfg.hi[i], cells[i] + 1) for i in range(dim)]
    grid = np.stack(np.meshgrid(*axes[::-1], indexing="ij")[::-1], axis=-1)
    disp = verts - grid
    h = np.array(cfg.h)
    assert np.all(np.abs(disp) <= 0.2 * h + 1e-15)
    for ax in range(dim):
        for end in (0, -1):
            sl = [slice(None)] * dim
            sl[dim - 1 - ax] = end                        # array axes are slowest first
            assert not np.any(disp[tuple(sl)])
    assert np.any(disp)


def test_coefficients_positive_and_layered():
    cfg = si.paper_config(1).replace(coef="lognormal", coef_sigma=0.8, n_cells=(6, 6, 1))
    _, c = si.draw_problem(cfg)
    assert c.shape == (36,) and np.all(c > 0) and np.std(np.log(c)) > 0.3
    shm = si.shm_config(r=0)
    _, rho = si.draw_problem(shm)
    assert set(np.unique(rho)) <= {1.0, 9.0, 16.0} and len(np.unique(rho)) == 3


def test_slab_vector_is_zero_on_the_boundary():
    cfg = si.paper_config(5).replace(n_cells=(4, 3, 2))
    v = si.random_slab_vector(cfg, 7)
    nodes = cfg.nodes
    assert v.shape == (cfg.n_t, int(np.prod(nodes)))
    w = v.reshape((cfg.n_t,) + tuple(nodes[::-1]))
    for ax in range(1, 4):
        for end in (0, -1):
            sl = [slice(None)] * 4
            sl[ax] = end
            assert not np.any(w[tuple(sl)])
    inner = w[:, 1:-1, 1:-1, 1:-1]
    assert abs(inner.mean()) < 0.2 and 0.8 < inner.std() < 1.2
