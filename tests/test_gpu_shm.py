"""Structural-health-monitoring wave example (Section 4.2) at a small size: slab-by-slab
marching through the library against the oracle's marching with direct solves, compared at
the three goal points (point values of the displacement at every temporal DoF), plus
conservation of the discrete energy by cGP(k)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import stmg_inputs as si
from oracle import norms, rhs, spacetime, spatial

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("rough", [False, True])
def test_shm_marching_matches_oracle(rough):
    from paper_2408_04372_amd import shm
    cfg = si.shm_config(r=1, p=2, k=2, n_time_cells=2, rough=rough)
    slabs = 3
    T = slabs * cfg.n_time_cells * cfg.tau
    times, vals, infos, summary, (gu, gv) = shm.run(cfg, T, precision=0, rtol=1e-12, max_iter=400)
    print(summary)
    verts, coef = si.draw_problem(cfg)
    op = spacetime.from_config(cfg, verts, coef)
    u0 = si.shm_initial_values(spatial.node_coordinates(op.space))
    v0 = np.zeros_like(u0)
    ref = []
    E = []
    for _ in range(slabs):
        b = rhs.rhs(op, np.zeros((cfg.n_t, op.n_x)), np.zeros(op.n_x), u0, v0)
        U = op.solve(b)
        V = rhs.velocity(op, U, u0, v0)
        ref.append(norms.point_values(op.space, U, si.SHM_POINTS))
        u0, v0 = U[-1].copy(), V[-1].copy()
        E.append(0.5 * (v0 @ (op.Mi @ v0) + u0 @ (op.Ai @ u0)))
    ref = np.concatenate(ref, axis=0)
    assert vals.shape == ref.shape
    scale = np.abs(ref).max()
    assert scale > 0
    assert np.abs(vals - ref).max() <= 1e-8 * scale
    assert np.abs(gu - u0).max() <= 1e-8 * np.abs(u0).max()
    Eg = 0.5 * (gv @ (op.Mi @ gv) + gu @ (op.Ai @ gu))
    assert np.allclose(E, E[0], rtol=1e-10)          # cGP with f = 0 conserves the energy
    assert abs(Eg - E[-1]) <= 1e-9 * E[-1]
    assert np.all(np.diff(times) > 0)
