"""Slab-by-slab time stepping through the C ABI (right-hand side with the coupling to the
previous slab, solve, velocity, last temporal DoF as the next initial value) against the
oracle's stepping with direct solves; the cGP(k) wave scheme with f = 0 must also conserve
the discrete energy E = (v^T M_h v + u^T A_h u) / 2 from slab to slab."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import stmg_inputs as si
from oracle import rhs, spacetime

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV).reshape(-1).contiguous()


@pytest.mark.parametrize("problem,method", [(1, 1), (1, 0), (0, 0), (0, 1)])
def test_stepping_matches_oracle(problem, method):
    from paper_2408_04372_amd import Handle
    cfg = si.Config(dim=3, problem=problem, time_method=method, p=2, k=2, n_time_cells=2, n_cells=(3, 3, 3),
                    tau=0.05, coef="lognormal", coef_sigma=0.5, seed=51)
    verts, coef = si.draw_problem(cfg)
    op = spacetime.from_config(cfg, verts, coef)
    X = np.stack([c.ravel() for c in np.meshgrid(*[np.linspace(0, 1, m) for m in cfg.nodes[::-1]],
                                                 indexing="ij")[::-1]], axis=1)
    u0 = np.sin(np.pi * X[:, 0]) * np.sin(np.pi * X[:, 1]) * np.sin(np.pi * X[:, 2])
    u0[op.bmask] = 0.0
    v0 = np.zeros_like(u0)
    slabs = 3
    # oracle: direct solves
    ou, ov = u0.copy(), v0.copy()
    energies = []
    for _ in range(slabs):
        b = rhs.rhs(op, np.zeros((cfg.n_t, op.n_x)), np.zeros(op.n_x) if method == 1 else None, ou, ov)
        U = op.solve(b)
        if problem == 1:
            V = rhs.velocity(op, U, ou, ov)
            ov = V[-1].copy()
        ou = U[-1].copy()
    # GPU: the same steps through the library
    with Handle(cfg, verts, coef, precision=0, rtol=1e-13, max_iter=400, omega=-1.0) as h:
        n = h.size(0)
        gu, gv = _t(u0), _t(v0)
        b = torch.empty(n, dtype=torch.float64, device=DEV)
        U = torch.zeros(n, dtype=torch.float64, device=DEV)
        V = torch.empty_like(U)
        M, A = op.Mi, op.Ai
        for _ in range(slabs):
            h.slab_rhs(b, None, torch.zeros_like(gu) if method == 1 else None, gu, gv if problem == 1 else None)
            U.zero_()
            h.solve(b, U)
            if problem == 1:
                h.wave_velocity(U, V, gu, gv)
                gv = V.view(cfg.n_t, -1)[-1].clone()
            gu = U.view(cfg.n_t, -1)[-1].clone()
            uu, vv = gu.cpu().numpy(), gv.cpu().numpy()
            energies.append(0.5 * (vv @ (M @ vv) + uu @ (A @ uu)))
    err_u = np.abs(gu.cpu().numpy() - ou).max() / np.abs(ou).max()
    print(problem, method, "u error", err_u, "energies", energies)
    assert err_u < 1e-9
    if problem == 1:
        err_v = np.abs(gv.cpu().numpy() - ov).max() / np.abs(ov).max()
        assert err_v < 1e-9
        if method == 1:      # cGP: discrete energy conserved with f = 0
            e0 = 0.5 * (v0 @ (M @ v0) + u0 @ (A @ u0))
            assert np.allclose(energies, e0, rtol=1e-9)
        else:                # dG: dissipative
            assert all(e2 <= e1 * (1 + 1e-12) for e1, e2 in zip(energies, energies[1:]))
