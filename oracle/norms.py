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


def point_values(space, u: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """Values of the Q_p field with nodal values u (N_x,) or (n_planes, N_x) at points (npts, dim)
    of a Cartesian mesh (goal quantities of Section 4.2)."""
    from . import basis
    if space.verts is not None:
        raise ValueError("Cartesian meshes only")
    u2 = np.atleast_2d(u)
    d, p = space.dim, space.p
    nodes = basis.gauss_lobatto(p + 1)
    dofs = space.cell_dofs()
    out = np.zeros((u2.shape[0], len(pts)))
    for q, x in enumerate(np.asarray(pts, dtype=float)):
        cc, phis = [], []
        for a in range(d):
            hx = (space.hi[a] - space.lo[a]) / space.cells[a]
            c = min(int(np.floor((x[a] - space.lo[a]) / hx)), space.cells[a] - 1)
            xi = (x[a] - space.lo[a]) / hx - c
            cc.append(c)
            phis.append(basis.lagrange(nodes, np.array([xi]))[0][0])
        w = phis[0]
        for a in range(1, d):
            w = np.kron(phis[a], w)                      # x fastest, like the cell's local nodes
        K = 0
        stride = 1
        for a in range(d):
            K += cc[a] * stride
            stride *= space.cells[a]
        out[:, q] = u2[:, dofs[K]] @ w
    return out if u.ndim == 2 else out[0]
