"""Slab right-hand sides and velocity recovery (Sections 2.1-2.2).

Loads F^i = (f(., t_i), phi) at the temporal DoF times are integrated in space
with (p+2)-point Gauss rules.  The printed load term "M_tau (x) M_h f" counts
the spatial mass twice when f already holds (f, phi) values; the reading used
is (M_T (x) I) F, i.e. the time integral by the node rule of the temporal basis.
The coupling signs of the cGP systems follow from the alpha and beta defined in
eq. cg-time-weights (the printed cGP right-hand sides carry the opposite sign).

With slab vectors a = e_1 (x) alpha and b_beta = e_1 (x) beta (temporal.Slab):
  heat dG : b = (M_T (x) I)F + (a (x) M_h) u0
  heat cGP: b = (M_T (x) I)F + (b_beta (x) I)F0 - (a (x) M_h + b_beta (x) A_h) u0
  wave dG : b = (M_T (x) I)F + (a (x) M_h) v0 + (A_T M_T^{-1} a (x) M_h) u0
  wave cGP: b = (M_T (x) I)F + (b_beta (x) I)F0 - (a (x) M_h) v0 - (b_beta (x) A_h) u0
                - (A_T M_T^{-1} a (x) M_h) u0 + (A_T M_T^{-1} b_beta (x) M_h) v0
Velocity (wave): V = M_T^{-1}(A_T U + a u0 - b_beta v0) for cGP and
V = M_T^{-1}(A_T U - a u0) for dG (eqs. wave-cg-dg-ade, wave-cg-cg-ade).
"""
from __future__ import annotations

import numpy as np

from . import basis, spatial, temporal
from .spacetime import SlabOperator


def loads(space: spatial.Space, f, times: np.ndarray) -> np.ndarray:
    """F[i, g] = (f(., times[i]), phi_g) with (p+2)-point Gauss per direction."""
    xi, W, Phi, _ = spatial.reference_tables(space.p, space.dim, nq=space.p + 2)
    J = spatial.jacobians(space, xi)
    det = np.linalg.det(J)
    X = space.cell_vertices()
    d = space.dim
    Nv = np.ones((xi.shape[0], 2 ** d))
    for v in range(2 ** d):
        for e in range(d):
            Nv[:, v] *= xi[:, e] if (v >> e) & 1 else 1.0 - xi[:, e]
    xq = np.einsum("qv,cvi->cqi", Nv, X)                     # physical quadrature points
    dofs = space.cell_dofs()
    out = np.zeros((len(times), space.n_x))
    for i, t in enumerate(times):
        fq = f(xq, t)                                         # (n_cells, n_q)
        loc = np.einsum("cq,q,qa->ca", fq * det, W, Phi)
        np.add.at(out[i], dofs.ravel(), loc.ravel())
    return out


def rhs(op: SlabOperator, F: np.ndarray, F0=None, u0=None, v0=None) -> np.ndarray:
    """Slab right-hand side b (n_t, N_x) from loads F at the temporal DoF times."""
    s = op.slab
    N = op.n_x
    u0 = np.zeros(N) if u0 is None else u0
    v0 = np.zeros(N) if v0 is None else v0
    b = s.M_T @ F
    Mu0 = op.Mi @ u0
    Au0 = op.Ai @ u0
    Mv0 = op.Mi @ v0
    if s.problem == temporal.HEAT:
        if s.method == temporal.DG:
            b = b + np.outer(s.a, Mu0)
        else:
            b = b + np.outer(s.b_beta, F0) - np.outer(s.a, Mu0) - np.outer(s.b_beta, Au0)
    else:
        g_a = s.A_T @ np.linalg.solve(s.M_T, s.a)
        if s.method == temporal.DG:
            b = b + np.outer(s.a, Mv0) + np.outer(g_a, Mu0)
        else:
            g_b = s.A_T @ np.linalg.solve(s.M_T, s.b_beta)
            b = (b + np.outer(s.b_beta, F0) - np.outer(s.a, Mv0) - np.outer(s.b_beta, Au0)
                 - np.outer(g_a, Mu0) + np.outer(g_b, Mv0))
    b[:, op.bmask] = 0.0
    return b


def velocity(op: SlabOperator, U: np.ndarray, u0=None, v0=None) -> np.ndarray:
    s = op.slab
    N = op.n_x
    u0 = np.zeros(N) if u0 is None else u0
    v0 = np.zeros(N) if v0 is None else v0
    R = s.A_T @ U
    if s.method == temporal.DG:
        R = R - np.outer(s.a, u0)
    else:
        R = R + np.outer(s.a, u0) - np.outer(s.b_beta, v0)
    return np.linalg.solve(s.M_T, R)


def nodal_interpolant(space: spatial.Space, g) -> np.ndarray:
    """Values of g at the lattice nodes (initial data by interpolation)."""
    return g(spatial.node_coordinates(space))
