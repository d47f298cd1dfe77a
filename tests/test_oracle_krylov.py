"""Pins of the oracle's flexible GMRES (the outer solver of Section 4).

With a fixed linear preconditioner M, flexible GMRES is right-preconditioned GMRES: after k steps
from x0 = 0 its iterate minimises ||b - S x|| over x in M K_k(S M, b).  The minimiser is computed
here independently: an orthonormal basis of the Krylov space from repeated QR factorisations of
[Q, S M q] (library routine), then a dense least-squares solve.  A wrong rotation, a dropped
Hessenberg entry or a misplaced preconditioner application changes the iterate."""
import numpy as np
import pytest

from oracle import krylov, spacetime
from stmg_inputs import draw_problem, random_slab_vector, small_configs


def _krylov_minimiser(S, M, b, k):
    SM = S @ M
    Q = (b / np.linalg.norm(b))[:, None]
    for _ in range(k - 1):
        Q, _ = np.linalg.qr(np.column_stack([Q, SM @ Q[:, -1]]))
    y, *_ = np.linalg.lstsq(SM @ Q, b, rcond=None)
    return M @ (Q @ y)


@pytest.mark.parametrize("ci", [0, 2])
@pytest.mark.parametrize("precond", ["identity", "diagonal"])
@pytest.mark.parametrize("k", [1, 4, 9])
def test_fgmres_iterate_is_the_krylov_minimiser(ci, precond, k):
    cfg = small_configs()[ci]
    verts, coef = draw_problem(cfg)
    op = spacetime.from_config(cfg, verts, coef)
    S = op.matrix().toarray()
    n = S.shape[0]
    if precond == "identity":
        M = np.eye(n)
    else:
        M = np.diag(1.0 / np.abs(np.diag(S)))
    b = random_slab_vector(cfg, 17).ravel()
    x, it, rr = krylov.fgmres(lambda v: S @ v, b, lambda v: M @ v, rtol=1e-30, restart=40, max_iter=k)
    assert it == k
    xs = _krylov_minimiser(S, M, b, k)
    r_gm = np.linalg.norm(b - S @ x)
    r_ref = np.linalg.norm(b - S @ xs)
    assert rr == pytest.approx(r_gm / np.linalg.norm(b), rel=1e-12)
    assert r_gm == pytest.approx(r_ref, rel=1e-9)
    assert np.linalg.norm(x - xs) <= 1e-7 * np.linalg.norm(xs)


def test_fgmres_restart_keeps_the_true_residual():
    # a restarted run returns the true residual of its iterate, and restarting never increases it
    cfg = small_configs()[0]
    verts, coef = draw_problem(cfg)
    op = spacetime.from_config(cfg, verts, coef)
    S = op.matrix().toarray()
    b = random_slab_vector(cfg, 18).ravel()
    last = np.inf
    for k in (5, 10, 15, 20):
        x, it, rr = krylov.fgmres(lambda v: S @ v, b, lambda v: v, rtol=1e-30, restart=5, max_iter=k)
        assert it == k
        assert rr == pytest.approx(np.linalg.norm(b - S @ x) / np.linalg.norm(b), rel=1e-12)
        assert rr <= last * (1 + 1e-12)
        last = rr
