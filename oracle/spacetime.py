"""The all-at-once slab operator S = M_T (x) A_h + N_T (x) M_h (eq. lin-sys).

Sections 2.1-2.2 give the four slab systems (eqs. heat-cg-dg-at-once,
wave-cg-dg-at-once, heat-cg-cg-at-once, wave-cg-cg-at-once); temporal.slab
writes each as one Kronecker sum.  Vectors are full-lattice space-time vectors
of shape (n_t, N_x): row i is the spatial vector of temporal DoF i (the block
layout of eq. heat-cg-dg).  Dirichlet nodes are kept in the vector and the
operator acts as the identity on them; interior rows only see interior columns.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import spatial, temporal


@dataclass
class SlabOperator:
    space: spatial.Space
    slab: temporal.Slab
    M: sp.csr_matrix            # assembled mass (all nodes)
    A: sp.csr_matrix            # assembled stiffness (all nodes)
    Mi: sp.csr_matrix           # Dirichlet-restricted (boundary rows/cols zero)
    Ai: sp.csr_matrix
    bmask: np.ndarray

    @property
    def n_t(self) -> int:
        return self.slab.n_t

    @property
    def n_x(self) -> int:
        return self.space.n_x

    def apply(self, X: np.ndarray) -> np.ndarray:
        """Y = S X for X of shape (n_t, N_x) (Kronecker form, A and M symmetric)."""
        shape = X.shape
        X = X.reshape(self.n_t, self.n_x)
        AX = (self.Ai @ X.T).T
        MX = (self.Mi @ X.T).T
        Y = self.slab.M_T @ AX + self.slab.N_T @ MX + X * self.bmask[None, :]
        return Y.reshape(shape)

    def matrix(self) -> sp.csr_matrix:
        """The assembled full-lattice slab matrix (n_t N_x square)."""
        B = sp.diags(self.bmask.astype(np.float64))
        S = (sp.kron(sp.csr_matrix(self.slab.M_T), self.Ai)
             + sp.kron(sp.csr_matrix(self.slab.N_T), self.Mi)
             + sp.kron(sp.identity(self.n_t), B))
        return S.tocsr()

    def solve(self, b: np.ndarray) -> np.ndarray:
        """Direct sparse solve of S u = b (SuperLU)."""
        S = self.matrix().tocsc()
        return spla.spsolve(S, b.ravel()).reshape(self.n_t, self.n_x)


def build(space: spatial.Space, slab: temporal.Slab) -> SlabOperator:
    M, A = spatial.assemble(space)
    bmask = space.boundary_mask()
    return SlabOperator(space=space, slab=slab, M=M, A=A,
                        Mi=spatial.dirichlet_restrict(M, bmask),
                        Ai=spatial.dirichlet_restrict(A, bmask), bmask=bmask)


def fine_space(cfg, verts: Optional[np.ndarray], coef: np.ndarray) -> spatial.Space:
    """Finest-level space of a configuration object (see stmg_inputs.Config)."""
    d = cfg.dim
    return spatial.Space(dim=d, cells=tuple(cfg.n_cells[:d]), p=cfg.p, verts=verts,
                         lo=tuple(cfg.lo[:d]), hi=tuple(cfg.hi[:d]),
                         coef_fine=np.asarray(coef, dtype=np.float64),
                         fine_cells=tuple(cfg.n_cells[:d]), ratio=1)


def from_config(cfg, verts: Optional[np.ndarray], coef: np.ndarray) -> SlabOperator:
    sl = temporal.slab(cfg.problem, cfg.time_method, cfg.k, cfg.n_time_cells, cfg.tau, cfg.t0)
    return build(fine_space(cfg, verts, coef), sl)
