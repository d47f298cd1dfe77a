"""Single entries of the slab operator and of one additive Schwarz step, for problems whose
assembled space-time matrices do not fit in host memory (test infrastructure, like the
rest of this package).

Each entry is computed from its definition by cell-local assembly.

Operator (eq. lin-sys, S = M_T (x) A_h + N_T (x) M_h with Dirichlet rows kept as identity):
  (S x)[i, g] = sum over cells K that contain node g, sum over j of
                (M_T)_ij (A_K x_K^j)_g + (N_T)_ij (M_K x_K^j)_g        (g interior)
  (S x)[i, g] = x[i, g]                                                (g on the boundary)
where x_K^j is temporal plane j of x on the nodes of K with Dirichlet values read as zero.

One additive Schwarz step from u = 0 (eqs. vanka0, vanka):
  u[i, g] = omega * sum over cells K that contain g of (B_K^{-1} R_{K,m} r)[i - m n_c, g]
with m the time cell of temporal DoF i, n_c temporal DoFs per time cell, and
B_K = M_tau (x) (A_h)_KK + Ntilde (x) (M_h)_KK, the principal submatrix of the assembled
operator on the interior nodes of K times one time cell; (A_h)_KK and (M_h)_KK are summed
from the cell matrices of K and of every cell that shares nodes with K.  A Dirichlet DoF is
its own 1x1 identity block: u = omega r there.
"""
from __future__ import annotations

from typing import Dict, Iterable, List, Tuple

import numpy as np

from . import mg, spacetime, spatial, temporal


class Sampler:
    """Cell matrices on demand for one configuration (finest level)."""

    def __init__(self, cfg, verts, coef):
        self.cfg = cfg
        self.space = spacetime.fine_space(cfg, verts, coef)
        self.slab = temporal.slab(cfg.problem, cfg.time_method, cfg.k, cfg.n_time_cells, cfg.tau, cfg.t0)
        self._cache: Dict[int, Tuple[np.ndarray, np.ndarray]] = {}
        self._fdm = None
        self._levels = None

    # node and cell numbering (computed per cell: the full tables would not fit at 10^8 nodes)
    def is_boundary(self, g: int) -> bool:
        return any(x == 0 or x == m - 1 for x, m in zip(self.node_coords(g), self.space.nodes))

    def cell_nodes(self, K: int) -> np.ndarray:
        """Global node index of each cell-local node (x fastest), like spatial.Space.cell_dofs."""
        p, n, dim = self.space.p, self.space.p + 1, self.space.dim
        cc = []
        k = K
        for m in self.space.cells:
            cc.append(k % m)
            k //= m
        loc = np.indices((n,) * dim).reshape(dim, -1)[::-1]        # rows: lx, ly(, lz), x fastest
        idx = np.zeros(loc.shape[1], dtype=np.int64)
        stride = 1
        for d in range(dim):
            idx += (cc[d] * p + loc[d]) * stride
            stride *= self.space.nodes[d]
        return idx

    def node_boundary(self, nodes: np.ndarray) -> np.ndarray:
        out = np.zeros(len(nodes), dtype=bool)
        rest = nodes.copy()
        for m in self.space.nodes:
            x = rest % m
            rest //= m
            out |= (x == 0) | (x == m - 1)
        return out

    # lattice helpers -----------------------------------------------------------------------
    def node_coords(self, g: int) -> List[int]:
        out = []
        for m in self.space.nodes:
            out.append(g % m)
            g //= m
        return out

    def cell_index(self, cc) -> int:
        idx, stride = 0, 1
        for d, c in enumerate(cc):
            idx += c * stride
            stride *= self.space.cells[d]
        return idx

    def cells_of_node(self, g: int) -> List[int]:
        p = self.space.p
        per_dim = []
        for d, x in enumerate(self.node_coords(g)):
            cand = [x // p - 1, x // p] if x % p == 0 else [x // p]
            per_dim.append([c for c in cand if 0 <= c < self.space.cells[d]])
        out = [[]]
        for opts in per_dim:
            out = [o + [c] for o in out for c in opts]
        return [self.cell_index(cc) for cc in out]

    def neighbours(self, K: int) -> List[int]:
        cc = []
        k = K
        for m in self.space.cells:
            cc.append(k % m)
            k //= m
        out = [[]]
        for d, c in enumerate(cc):
            out = [o + [c + e] for o in out for e in (-1, 0, 1) if 0 <= c + e < self.space.cells[d]]
        return [self.cell_index(v) for v in out]

    def matrices(self, cells: Iterable[int]):
        need = sorted(set(int(c) for c in cells) - set(self._cache))
        if need:
            M, A = spatial.cell_matrices(self.space, np.array(need, dtype=np.int64))
            for c, m, a in zip(need, M, A):
                self._cache[c] = (m, a)
        return [self._cache[int(c)] for c in cells]

    # sampled operator rows -------------------------------------------------------------------
    def operator_entries(self, x: np.ndarray, samples) -> np.ndarray:
        """(S x)[i, g] for each (i, g) in samples; x of shape (n_t, N_x)."""
        x = x.reshape(self.slab.n_t, self.space.n_x)
        out = np.zeros(len(samples))
        self.matrices([K for _, g in samples if not self.is_boundary(g) for K in self.cells_of_node(g)])
        for s, (i, g) in enumerate(samples):
            if self.is_boundary(g):
                out[s] = x[i, g]
                continue
            val = 0.0
            cells = self.cells_of_node(g)
            for K, (Mk, Ak) in zip(cells, self.matrices(cells)):
                d = self.cell_nodes(K)
                a = int(np.nonzero(d == g)[0][0])
                xK = x[:, d] * (~self.node_boundary(d))[None, :]   # (n_t, n_s)
                Ax = xK @ Ak[a]                                     # (A_K x^j)_g for every j
                Mx = xK @ Mk[a]
                val += self.slab.M_T[i] @ Ax + self.slab.N_T[i] @ Mx
            out[s] = val
        return out

    # sampled additive Schwarz step -----------------------------------------------------------
    def local_blocks(self, K: int):
        """Interior node list of K and (A_h)_KK, (M_h)_KK on it (principal submatrices)."""
        dK = self.cell_nodes(K)
        inner = dK[~self.node_boundary(dK)]
        pos = {int(g): t for t, g in enumerate(inner)}
        n = len(inner)
        A = np.zeros((n, n))
        M = np.zeros((n, n))
        nb = self.neighbours(K)
        for K2, (Mk, Ak) in zip(nb, self.matrices(nb)):
            d2 = self.cell_nodes(K2)
            loc = np.array([pos.get(int(g), -1) for g in d2])
            sel = np.nonzero(loc >= 0)[0]
            if len(sel) == 0:
                continue
            ix = np.ix_(loc[sel], loc[sel])
            A[ix] += Ak[np.ix_(sel, sel)]
            M[ix] += Mk[np.ix_(sel, sel)]
        return inner, A, M

    def separable_blocks(self, K: int):
        """Interior node list of K and the separable surrogate (A~, M~) (oracle.mg.fdm_cell)."""
        if self._fdm is None:
            self._fdm = mg.fdm_setup(self.space)
        dK = self.cell_nodes(K)
        inner = dK[~self.node_boundary(dK)]
        cc = []
        k = K
        for m in self.space.cells:
            cc.append(k % m)
            k //= m
        Mt, At = mg.fdm_cell(self.space, cc, *self._fdm)
        return inner, At, Mt

    def asm_entries(self, r: np.ndarray, omega: float, samples, separable: bool = False) -> np.ndarray:
        """u[i, g] after one additive Schwarz step u = omega * ASM(r) from u = 0 (exact cell
        blocks, or the separable surrogate blocks of oracle.mg.fdm_blocks)."""
        r = r.reshape(self.slab.n_t, self.space.n_x)
        nc = self.slab.nt_cell
        out = np.zeros(len(samples))
        if not separable:
            self.matrices([K2 for _, g in samples if not self.is_boundary(g) for K in self.cells_of_node(g)
                           for K2 in self.neighbours(K)])
        for s, (i, g) in enumerate(samples):
            if self.is_boundary(g):
                out[s] = omega * r[i, g]
                continue
            m, il = divmod(i, nc)
            val = 0.0
            for K in self.cells_of_node(g):
                inner, A, M = self.local_blocks(K) if not separable else self.separable_blocks(K)
                B = np.kron(self.slab.M_tau, A) + np.kron(self.slab.N_tilde, M)
                rhs = r[m * nc:(m + 1) * nc][:, inner].ravel()          # [temporal][node]
                sol = np.linalg.solve(B, rhs).reshape(nc, len(inner))
                val += sol[il, int(np.nonzero(inner == g)[0][0])]
            out[s] = omega * val
        return out


    # sampled grid transfers (Section 3.2) ------------------------------------------------------
    def level_spaces(self) -> List[spatial.Space]:
        """Spatial levels, finest (index 0) first, as in oracle.mg.level_spaces."""
        if self._levels is None:
            self._levels = mg.level_spaces(self.space)
        return self._levels

    def transfer_factors(self, level: int) -> List[np.ndarray]:
        """Per direction, the 1D prolongation from level + 1 to level (dense, nodes_f x nodes_c).

        The prolongation evaluates a coarse basis function at a fine node in the reference
        coordinates of one coarse cell per direction, so its value is the product over the
        directions of 1D values: P = P_{d-1} (x) ... (x) P_0 on the x-fastest node numbering.
        Each factor is oracle.mg.prolongation on the 1D lattice of that direction."""
        fine, coarse = self.level_spaces()[level], self.level_spaces()[level + 1]
        out = []
        for d in range(fine.dim):
            f1 = spatial.Space(dim=1, cells=(fine.cells[d],), p=fine.p, verts=None, lo=(0.0,), hi=(1.0,),
                               coef_fine=np.ones(1), fine_cells=(fine.cells[d],))
            c1 = spatial.Space(dim=1, cells=(coarse.cells[d],), p=coarse.p, verts=None, lo=(0.0,), hi=(1.0,),
                               coef_fine=np.ones(1), fine_cells=(fine.cells[d],))
            out.append(mg.prolongation(c1, f1).toarray())
        return out

    @staticmethod
    def _coords(g: int, nodes) -> List[int]:
        out = []
        for m in nodes:
            out.append(g % m)
            g //= m
        return out

    def prolong_entries(self, ec: np.ndarray, level: int, samples) -> np.ndarray:
        """(P e_c)[i, g] at fine-level nodes: e_c of shape (n_t, N_x of level + 1), Dirichlet
        values of e_c read as zero, zero at fine Dirichlet nodes (oracle.mg.Hierarchy.prolong)."""
        fine, coarse = self.level_spaces()[level], self.level_spaces()[level + 1]
        ec = ec.reshape(-1, coarse.n_x)
        P1 = self.transfer_factors(level)
        out = np.zeros(len(samples))
        for s, (i, g) in enumerate(samples):
            xf = self._coords(g, fine.nodes)
            if any(x == 0 or x == m - 1 for x, m in zip(xf, fine.nodes)):
                continue
            cols = [np.nonzero(P1[d][xf[d]])[0] for d in range(fine.dim)]
            val = 0.0
            for cc in np.array(np.meshgrid(*cols, indexing="ij")).reshape(fine.dim, -1).T:
                if any(c == 0 or c == m - 1 for c, m in zip(cc, coarse.nodes)):
                    continue
                w, gc, stride = 1.0, 0, 1
                for d in range(fine.dim):
                    w *= P1[d][xf[d], cc[d]]
                    gc += int(cc[d]) * stride
                    stride *= coarse.nodes[d]
                val += w * ec[i, gc]
            out[s] = val
        return out

    def restrict_entries(self, rf: np.ndarray, level: int, samples) -> np.ndarray:
        """(P^T r_f)[i, g] at nodes of level + 1: r_f of shape (n_t, N_x of level), Dirichlet
        values of r_f read as zero, zero at coarse Dirichlet nodes (oracle.mg.Hierarchy.restrict)."""
        fine, coarse = self.level_spaces()[level], self.level_spaces()[level + 1]
        rf = rf.reshape(-1, fine.n_x)
        P1 = self.transfer_factors(level)
        out = np.zeros(len(samples))
        for s, (i, g) in enumerate(samples):
            xc = self._coords(g, coarse.nodes)
            if any(x == 0 or x == m - 1 for x, m in zip(xc, coarse.nodes)):
                continue
            rows = [np.nonzero(P1[d][:, xc[d]])[0] for d in range(fine.dim)]
            val = 0.0
            for ff in np.array(np.meshgrid(*rows, indexing="ij")).reshape(fine.dim, -1).T:
                if any(f == 0 or f == m - 1 for f, m in zip(ff, fine.nodes)):
                    continue
                w, gf, stride = 1.0, 0, 1
                for d in range(fine.dim):
                    w *= P1[d][ff[d], xc[d]]
                    gf += int(ff[d]) * stride
                    stride *= fine.nodes[d]
                val += w * rf[i, gf]
            out[s] = val
        return out


def sample_points(cfg, n_inner: int, n_boundary: int, seed: int):
    """(temporal DoF, node) pairs on the finest level: interior nodes of every kind (cell
    corners, edges, faces, cell interiors) and a few Dirichlet nodes, drawn from a seeded
    generator."""
    return lattice_points(cfg.p, cfg.n_cells[: cfg.dim], cfg.n_t, n_inner, n_boundary, seed)


def lattice_points(p: int, cells, n_t: int, n_inner: int, n_boundary: int, seed: int):
    """Like sample_points for any Q_p lattice of `cells` cells per direction and n_t planes."""
    rng = np.random.default_rng(seed)
    dim = len(cells)
    nodes = [p * c + 1 for c in cells]
    out = []
    for t in range(n_inner):
        kind = t % 4          # number of coordinates that sit on a cell boundary (0..3, capped at dim)
        coords = []
        for d in range(dim):
            on = d < min(kind, dim)
            while True:
                x = int(rng.integers(1, nodes[d] - 1))
                if (x % p == 0) == on or p == 1:
                    break
            coords.append(x)
        g, stride = 0, 1
        for d in range(dim):
            g += coords[d] * stride
            stride *= nodes[d]
        out.append((int(rng.integers(0, n_t)), g))
    for _ in range(n_boundary):
        coords = [int(rng.integers(0, m)) for m in nodes]
        d = int(rng.integers(0, dim))
        coords[d] = 0 if rng.random() < 0.5 else nodes[d] - 1
        g, stride = 0, 1
        for dd in range(dim):
            g += coords[dd] * stride
            stride *= nodes[dd]
        out.append((int(rng.integers(0, n_t)), g))
    return out
