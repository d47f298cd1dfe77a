"""Error norms of eq. norms and the discrete wave energy.

L2(L2): space-time Gauss quadrature ((p+2) points per space direction, k+2 in
time) of (u_h - u)^2 over the slab.  The discrete solution on time cell m is
sum_i U_{m,i}(x) xi_i(t); for cGP the first trial DoF is the previous end value.
"""
from __future__ import annotations

import numpy as np

from . import basis, spatial, temporal
from .spacetime import SlabOperator


def l2l2_error(op: SlabOperator, U: np.ndarray, u_exact, k: int, u0=None) -> float:
    space, s = op.space, op.slab
    xi, W, Phi, _ = spatial.reference_tables(space.p, space.dim, nq=space.p + 2)
    J = spatial.jacobians(space, xi)
    det = np.linalg.det(J)
    X = space.cell_vertices()
    d = space.dim
    Nv = np.ones((xi.shape[0], 2 ** d))
    for v in range(2 ** d):
        for e in range(d):
            Nv[:, v] *= xi[:, e] if (v >> e) & 1 else 1.0 - xi[:, e]
    xq = np.einsum("qv,cvi->cqi", Nv, X)
    dofs = space.cell_dofs()
    tq, tw = basis.gauss(k + 2)
    if s.method == temporal.DG:
        tn = basis.gauss_radau_right(k + 1)
    else:
        tn = basis.gauss_lobatto(k + 1)
    Vt, _ = basis.lagrange(tn, tq)
    nc = s.nt_cell
    c = s.n_t // nc
    tau, t0 = s.tau, s.t0
    N = op.n_x
    prev = np.zeros(N) if u0 is None else u0
    err2 = 0.0
    for m in range(c):
        blk = U[m * nc:(m + 1) * nc]
        if s.method == temporal.DG:
            coeffs = blk
        else:
            coeffs = np.vstack([prev[None, :], blk])
        for qi in range(len(tq)):
            t = t0 + (m + tq[qi]) * tau
            uh_nodes = Vt[qi] @ coeffs                           # spatial nodal vector at time t
            uh = np.einsum("qa,ca->cq", Phi, uh_nodes[dofs])
            ue = u_exact(xq, t)
            err2 += tw[qi] * tau * np.sum((uh - ue) ** 2 * det * W[None, :])
        prev = blk[-1]
    return float(np.sqrt(err2))


def wave_energy(op: SlabOperator, u: np.ndarray, v: np.ndarray) -> float:
    """E = (v^T M_h v + u^T A_h u) / 2 on interior couplings."""
    return 0.5 * float(v @ (op.Mi @ v) + u @ (op.Ai @ u))
