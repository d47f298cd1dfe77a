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


def degree(s: Slab) -> int:
    """Temporal degree k of a slab (dG: k + 1 DoFs per cell, cGP: k)."""
    return s.nt_cell - 1 if s.method == DG else s.nt_cell


def coarsen(s: Slab, kind: str) -> Slab:
    """The next coarser temporal space: 'k' lowers the degree by one, 'tau' merges pairs of
    time cells (Section 3.2, k- and tau-multigrid)."""
    k, c = degree(s), s.n_t // s.nt_cell
    if kind == "k":
        return slab(s.problem, s.method, k - 1, c, s.tau, s.t0)
    return slab(s.problem, s.method, k, c // 2, 2.0 * s.tau, s.t0)


def time_levels(s: Slab) -> list:
    """Temporal coarsening after the spatial levels: k down to its minimum (dG 0, cGP 1), then
    halve the number of time cells while it is even.  Returns the coarser slabs in order."""
    out = []
    cur = s
    kmin = 0 if s.method == DG else 1
    while degree(cur) > kmin:
        cur = coarsen(cur, "k")
        out.append(cur)
    while (cur.n_t // cur.nt_cell) % 2 == 0:
        cur = coarsen(cur, "tau")
        out.append(cur)
    return out


def prolongation(fine: Slab, coarse: Slab) -> np.ndarray:
    """Temporal prolongation P (fine.n_t x coarse.n_t): at every fine temporal DoF time, the
    value of the coarse trial function of each coarse DoF (the coarse space lies in the fine
    one, so this is the embedding; the restriction is P^T).  cGP: the first trial node of
    coarse cell M is the last DoF of cell M - 1; in cell 0 it is the slab's initial value, a
    constrained DoF that carries no correction, so that column is absent."""
    kc = degree(coarse)
    ncc = coarse.nt_cell
    cc = coarse.n_t // ncc
    nodes = basis.gauss_radau_right(kc + 1) if coarse.method == DG else basis.gauss_lobatto(kc + 1)
    P = np.zeros((fine.n_t, coarse.n_t))
    for i, t in enumerate(fine.times):
        s = (t - coarse.t0) / coarse.tau
        M = min(max(int(np.ceil(s - 1e-12)) - 1, 0), cc - 1)
        vals = basis.lagrange(nodes, np.array([s - M]))[0][0]
        if coarse.method == DG:
            P[i, M * ncc:(M + 1) * ncc] = vals
        else:
            P[i, M * ncc:(M + 1) * ncc] = vals[1:]
            if M > 0:
                P[i, M * ncc - 1] += vals[0]
    return P
