"""Flexible GMRES(m) with right preconditioning (Section 4: GMRES, one V-cycle per iteration).

Plain textbook FGMRES: modified Gram-Schmidt Arnoldi, Givens rotations, the
update x = x0 + Z y at restart, and a true-residual check at each restart.
The stopping rule is the true relative residual ||b - S x|| / ||b|| <= rtol.
"""
from __future__ import annotations

import numpy as np


def fgmres(apply_S, b: np.ndarray, prec, x0=None, rtol: float = 1e-8, restart: int = 30,
           max_iter: int = 500):
    b = b.ravel()
    x = np.zeros_like(b) if x0 is None else x0.ravel().copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, 0, 0.0
    it = 0
    while True:
        r = b - apply_S(x)
        beta = np.linalg.norm(r)
        if beta / bnorm <= rtol or it >= max_iter:
            return x, it, beta / bnorm
        m = restart
        V = np.zeros((m + 1, len(b)))
        Z = np.zeros((m, len(b)))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        j_used = 0
        for j in range(m):
            Z[j] = prec(V[j])
            w = apply_S(Z[j])
            for i in range(j + 1):
                H[i, j] = V[i] @ w
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j_used = j + 1
            if abs(g[j + 1]) / bnorm <= rtol or it >= max_iter:
                break
        y = np.linalg.solve(np.triu(H[:j_used, :j_used]), g[:j_used])
        x = x + Z[:j_used].T @ y
