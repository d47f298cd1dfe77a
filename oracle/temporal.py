"""Temporal matrices of dG(k) and cGP(k) and their slab-level Kronecker factors.

dG(k), Section 2.1 (eq. dg-time-weights).  Trial = test = P_k on each time cell
with the Lagrange basis at the k+1 right Gauss-Radau points.  The printed
derivative matrix and alpha are garbled; the reading used here comes from the
upwind jump term of eq. var-heat-dg:
    (M_tau)_ij = tau * int_0^1 xi_j xi_i,
    (A_tau)_ij = int_0^1 xi_j' xi_i + xi_j(0) xi_i(0),
    alpha_i    = xi_i(0)   (couples the previous cell's value at its end, the last DoF).

cGP(k), Section 2.2 (eq. cg-time-weights).  Trial P_k at the k+1 Gauss-Lobatto
points, test P_{k-1} at the last k of them.  The first trial DoF is fixed by
continuity; its weights are beta (mass) and alpha (derivative).

Slab level (Sections 2.1-2.2, the all-at-once systems): c time cells give
block lower-bidiagonal temporal factors M_T, A_T.  In every case the slab
operator is S = M_T (x) A_h + N_T (x) M_h with N_T = A_T (heat) or
N_T = A_T M_T^{-1} A_T (wave, after eliminating the velocity).  For the wave
systems this slab form replaces the printed E_ij / C_ij block recurrences,
whose factors are garbled; the diagonal and first sub-diagonal blocks agree
with the printed S and -B.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import basis

HEAT, WAVE = 0, 1
DG, CGP = 0, 1


def dg_local(k: int, tau: float):
    """(M_tau, A_tau, alpha, nodes) of dG(k) on one time cell of length tau."""
    nodes = basis.gauss_radau_right(k + 1)
    xq, wq = basis.gauss(k + 3)
    V, D = basis.lagrange(nodes, xq)
    V0, _ = basis.lagrange(nodes, np.array([0.0]))
    M = tau * (V * wq[:, None]).T @ V                      # M[i,j] = tau sum_q w xi_i xi_j
    A = (V * wq[:, None]).T @ D + np.outer(V0[0], V0[0])   # A[i,j] = int xi_j' xi_i + xi_j(0) xi_i(0)
    alpha = V0[0].copy()
    return M, A, alpha, nodes


def cgp_local(k: int, tau: float):
    """(M_tau, A_tau, alpha, beta, trial_nodes) of cGP(k) on one time cell of length tau."""
    if k < 1:
        raise ValueError("cGP needs k >= 1")
    trial = basis.gauss_lobatto(k + 1)
    test = trial[1:]
    xq, wq = basis.gauss(k + 3)
    Vt, Dt = basis.lagrange(trial, xq)        # trial values / derivatives, columns j = 0..k
    Vs, _ = basis.lagrange(test, xq)          # test values, columns i = 0..k-1
    Mfull = tau * (Vs * wq[:, None]).T @ Vt   # [i, j] = tau int xi_j psi_i
    Afull = (Vs * wq[:, None]).T @ Dt         # [i, j] = int xi_j' psi_i
    M = Mfull[:, 1:]
    A = Afull[:, 1:]
    beta = Mfull[:, 0].copy()
    alpha = Afull[:, 0].copy()
    return M, A, alpha, beta, trial


@dataclass
class Slab:
    """Slab-level temporal data for c time cells."""
    n_t: int            # temporal DoFs in the slab
    nt_cell: int        # temporal DoFs per time cell (k+1 dG, k cGP)
    M_T: np.ndarray
    A_T: np.ndarray
    N_T: np.ndarray
    a: np.ndarray       # couples u0 (dG: +alpha, cGP: alpha) into the first cell
    b_beta: np.ndarray  # cGP only (zeros for dG)
    M_tau: np.ndarray   # diagonal block of M_T
    N_tilde: np.ndarray  # diagonal block of N_T (ASM local temporal factor)
    times: np.ndarray   # absolute time of each temporal DoF
    method: int
    problem: int
    tau: float = 0.0
    t0: float = 0.0


def slab(problem: int, method: int, k: int, c: int, tau: float, t0: float = 0.0) -> Slab:
    if method == DG:
        M, A, alpha, nodes = dg_local(k, tau)
        beta = np.zeros_like(alpha)
        sub_A = -np.outer(alpha, np.eye(len(alpha))[-1])
        sub_M = np.zeros_like(M)
        local_nodes = nodes
    else:
        M, A, alpha, beta, trial = cgp_local(k, tau)
        sub_A = np.outer(alpha, np.eye(len(alpha))[-1])
        sub_M = np.outer(beta, np.eye(len(beta))[-1])
        local_nodes = trial[1:]
    nc = M.shape[0]
    n_t = nc * c
    M_T = np.zeros((n_t, n_t))
    A_T = np.zeros((n_t, n_t))
    for m in range(c):
        s = slice(m * nc, (m + 1) * nc)
        M_T[s, s] = M
        A_T[s, s] = A
        if m > 0:
            sp = slice((m - 1) * nc, m * nc)
            M_T[s, sp] = sub_M
            A_T[s, sp] = sub_A
    if problem == HEAT:
        N_T = A_T.copy()
    else:
        N_T = A_T @ np.linalg.solve(M_T, A_T)
    a = np.zeros(n_t)
    a[:nc] = alpha
    bb = np.zeros(n_t)
    bb[:nc] = beta
    times = np.concatenate([t0 + (m + local_nodes) * tau for m in range(c)])
    return Slab(n_t=n_t, nt_cell=nc, M_T=M_T, A_T=A_T, N_T=N_T, a=a, b_beta=bb,
                M_tau=M_T[:nc, :nc].copy(), N_tilde=N_T[:nc, :nc].copy(), times=times,
                method=method, problem=problem, tau=tau, t0=t0)


def amplification(problem: int, method: int, k: int, z: complex) -> complex:
    """One-step amplification of the scalar heat test equation y' = -(z/tau) y.

    dG: (z M + A) U = alpha y0, y1 = U[-1];  cGP: (z M + A) U = -(alpha + z beta) y0.
    Used only to pin the temporal matrices against Pade approximants of exp(-z).
    """
    if method == DG:
        M, A, alpha, _ = dg_local(k, 1.0)
        U = np.linalg.solve(z * M + A, alpha.astype(complex))
    else:
        M, A, alpha, beta, _ = cgp_local(k, 1.0)
        U = np.linalg.solve(z * M + A, -(alpha + z * beta).astype(complex))
    return U[-1]
