"""Spatial Q_p finite elements on structured hexahedral (or quadrilateral) meshes.

Sections 1.1 and 2 (eqs. fespace, space-matrices): continuous Q_p on cells given by a
reference mapping, nodal Lagrange basis, M_h = (phi_i, phi_j) and
A_h = (rho grad phi_i, grad phi_j).  Readings used where the paper is silent:
GLL nodes per direction, (p+1)-point Gauss quadrature per direction, bilinear /
trilinear cells built from the vertex lattice, homogeneous Dirichlet data on
the whole boundary (Section 4.1).

Lattice conventions: cell index c = cx + nx*(cy + ny*cz); node index
g = gx + Nx*(gy + Ny*gz) with N = p*n + 1 per direction; cell-local node
a = lx + (p+1)*(ly + (p+1)*lz).

Coefficients on coarse multigrid levels (geometric MG re-discretisation,
Section 3): at a quadrature point with reference coordinate xi in a cell that
covers r^d finest cells, the coefficient is that of the finest descendant cell
whose reference sub-box contains xi (for Cartesian meshes this is the finest
cell that contains the physical point).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Tuple

import numpy as np
import scipy.sparse as sp

from . import basis


@dataclass
class Space:
    dim: int
    cells: Tuple[int, ...]          # cells per direction on this level
    p: int
    verts: Optional[np.ndarray]     # vertex lattice of this level (None: Cartesian box)
    lo: Tuple[float, ...]
    hi: Tuple[float, ...]
    coef_fine: np.ndarray           # coefficient of every finest cell (x fastest)
    fine_cells: Tuple[int, ...]
    ratio: int = 1                  # finest cells per cell of this level, per direction

    @property
    def n(self) -> int:
        return self.p + 1

    @property
    def nodes(self) -> Tuple[int, ...]:
        return tuple(self.p * c + 1 for c in self.cells)

    @property
    def n_x(self) -> int:
        return int(np.prod(self.nodes))

    @property
    def n_cells(self) -> int:
        return int(np.prod(self.cells))

    def cell_coords(self) -> np.ndarray:
        """Integer cell coordinates, shape (n_cells, dim), x fastest."""
        grids = np.meshgrid(*[np.arange(c) for c in self.cells[::-1]], indexing="ij")
        return np.stack([g.ravel() for g in grids[::-1]], axis=1)

    def cell_dofs(self) -> np.ndarray:
        """Global node index of each cell-local node, shape (n_cells, (p+1)^dim)."""
        n = self.n
        loc = np.meshgrid(*[np.arange(n)] * self.dim, indexing="ij")
        loc = np.stack([g.ravel() for g in loc[::-1]], axis=1)     # local (lx, ly, lz), lx fastest
        cc = self.cell_coords()
        gcoord = cc[:, None, :] * self.p + loc[None, :, :]
        N = self.nodes
        idx = np.zeros(gcoord.shape[:2], dtype=np.int64)
        stride = 1
        for d in range(self.dim):
            idx += gcoord[:, :, d] * stride
            stride *= N[d]
        return idx

    def boundary_mask(self) -> np.ndarray:
        """True on lattice nodes that lie on the domain boundary (Dirichlet nodes)."""
        N = self.nodes
        grids = np.meshgrid(*[np.arange(m) for m in N[::-1]], indexing="ij")
        gc = [g.ravel() for g in grids[::-1]]
        mask = np.zeros(self.n_x, dtype=bool)
        for d in range(self.dim):
            mask |= (gc[d] == 0) | (gc[d] == N[d] - 1)
        return mask

    def cell_vertices(self) -> np.ndarray:
        """Corner positions of every cell, shape (n_cells, 2^dim, dim), corner v = vx + 2 vy + 4 vz."""
        cc = self.cell_coords()
        corners = np.array([[(v >> d) & 1 for d in range(self.dim)] for v in range(2 ** self.dim)])
        vc = cc[:, None, :] + corners[None, :, :]
        if self.verts is None:
            h = np.array([(self.hi[d] - self.lo[d]) / self.cells[d] for d in range(self.dim)])
            return np.array(self.lo[: self.dim])[None, None, :] + vc * h[None, None, :]
        idx = tuple(vc[:, :, d] for d in reversed(range(self.dim)))
        return self.verts[idx]

    def coef_at(self, xi: np.ndarray, cells: Optional[np.ndarray] = None) -> np.ndarray:
        """Coefficient at reference points xi (n_q, dim) of every cell (or of the listed
        cells): (n_cells, n_q)."""
        r = self.ratio
        cc = self.cell_coords()
        if cells is not None:
            cc = cc[cells]
        sub = np.minimum(np.floor(xi * r).astype(np.int64), r - 1)      # (n_q, dim)
        fc = cc[:, None, :] * r + sub[None, :, :]
        idx = np.zeros(fc.shape[:2], dtype=np.int64)
        stride = 1
        for d in range(self.dim):
            idx += fc[:, :, d] * stride
            stride *= self.fine_cells[d]
        return self.coef_fine[idx]


def reference_tables(p: int, dim: int, nq: Optional[int] = None):
    """Tensor-product basis values/gradients at Gauss points: (xi_q, w_q, Phi, [G_d])."""
    n = p + 1
    nq = nq or n
    xq, wq = basis.gauss(nq)
    nodes = basis.gauss_lobatto(n)
    V, D = basis.lagrange(nodes, xq)
    if dim == 2:
        Phi = np.kron(V, V)
        G = [np.kron(V, D), np.kron(D, V)]
        W = np.kron(wq, wq)
        qg = np.meshgrid(xq, xq, indexing="ij")
        xi = np.stack([qg[1].ravel(), qg[0].ravel()], axis=1)
    else:
        Phi = np.kron(V, np.kron(V, V))
        G = [np.kron(V, np.kron(V, D)), np.kron(V, np.kron(D, V)), np.kron(D, np.kron(V, V))]
        W = np.kron(wq, np.kron(wq, wq))
        qg = np.meshgrid(xq, xq, xq, indexing="ij")
        xi = np.stack([qg[2].ravel(), qg[1].ravel(), qg[0].ravel()], axis=1)
    return xi, W, Phi, G


def jacobians(space: Space, xi: np.ndarray, cells: Optional[np.ndarray] = None) -> np.ndarray:
    """J[c, q] = d x / d xi (dim x dim) of the multilinear cell map at reference points xi
    (every cell, or the listed cells)."""
    X = space.cell_vertices()                     # (nc, 2^d, d)
    if cells is not None:
        X = X[cells]
    d = space.dim
    nv = 2 ** d
    dN = np.zeros((xi.shape[0], nv, d))
    for v in range(nv):
        bits = [(v >> e) & 1 for e in range(d)]
        for j in range(d):
            val = np.ones(xi.shape[0])
            for e in range(d):
                if e == j:
                    val = val * (1.0 if bits[e] else -1.0)
                else:
                    val = val * (xi[:, e] if bits[e] else 1.0 - xi[:, e])
            dN[:, v, j] = val
    return np.einsum("cvi,qvj->cqij", X, dN)


def cell_matrices(space: Space, cells: Optional[np.ndarray] = None):
    """Element mass and stiffness matrices, each (n_cells, n_s, n_s), by Gauss quadrature
    (every cell, or only the listed linear cell indices, in that order)."""
    xi, W, Phi, G = reference_tables(space.p, space.dim)
    J = jacobians(space, xi, cells)
    det = np.linalg.det(J)
    if np.any(det <= 0):
        raise ValueError("inverted cell")
    Jinv = np.linalg.inv(J)
    K = np.einsum("cqik,cqjk->cqij", Jinv, Jinv)       # J^{-1} J^{-T}
    rho = space.coef_at(xi, cells)
    wdet = W[None, :] * det
    Mk = np.einsum("qa,cq,qb->cab", Phi, wdet, Phi)
    Ak = np.zeros_like(Mk)
    for i in range(space.dim):
        for j in range(space.dim):
            Ak += np.einsum("qa,cq,qb->cab", G[i], wdet * rho * K[:, :, i, j], G[j])
    return Mk, Ak


def assemble(space: Space):
    """Assembled (M_h, A_h) over all lattice nodes (boundary included), CSR."""
    Mk, Ak = cell_matrices(space)
    dofs = space.cell_dofs()
    ns = dofs.shape[1]
    rows = np.repeat(dofs, ns, axis=1).ravel()
    cols = np.tile(dofs, (1, ns)).ravel()
    N = space.n_x
    M = sp.csr_matrix((Mk.ravel(), (rows, cols)), shape=(N, N))
    A = sp.csr_matrix((Ak.ravel(), (rows, cols)), shape=(N, N))
    M.sum_duplicates()
    A.sum_duplicates()
    return M, A


def dirichlet_restrict(mat: sp.spmatrix, bmask: np.ndarray) -> sp.csr_matrix:
    """Zero boundary rows and columns (the operator keeps only interior couplings)."""
    keep = sp.diags((~bmask).astype(np.float64))
    return (keep @ mat @ keep).tocsr()


def node_coordinates(space: Space) -> np.ndarray:
    """Physical position of every lattice node, shape (N_x, dim)."""
    n = space.n
    nodes1 = basis.gauss_lobatto(n)
    ref = np.meshgrid(*[nodes1] * space.dim, indexing="ij")
    ref = np.stack([g.ravel() for g in ref[::-1]], axis=1)          # (n_s, d), x fastest
    X = space.cell_vertices()
    d = space.dim
    Nv = np.ones((ref.shape[0], 2 ** d))
    for v in range(2 ** d):
        for e in range(d):
            Nv[:, v] *= ref[:, e] if (v >> e) & 1 else 1.0 - ref[:, e]
    pos = np.einsum("sv,cvi->csi", Nv, X)
    out = np.zeros((space.n_x, d))
    out[space.cell_dofs().ravel()] = pos.reshape(-1, d)
    return out
