"""Space-time multigrid: hierarchy, transfers, cell-wise additive Schwarz, V-cycle.

Section 3 of the paper.  Readings where the paper is silent:
  * hierarchy (Alg. mg-sequence, spatial levels only): halve p while p > min_p
    (4 -> 2 -> 1, 3 -> 1, 2 -> 1), then halve the cell count per direction while
    it stays even and >= 2 * coarse_cells; coarse h-levels use the even-index
    vertex subset and re-discretise (coefficient lookup in spatial.Space).
  * transfers (Section 3.2): prolongation evaluates the coarse Q_p function at
    the fine nodes through the fine node's reference coordinates in its coarse
    parent cell (the L2 embedding of nested spaces); restriction is the exact
    transpose.  Both act on interior nodes only (Dirichlet rows/columns dropped).
  * smoother (eqs. vanka0, vanka): blocks are the interior DoFs of one spatial
    cell times the temporal DoFs of one time cell; the block matrix is the
    principal submatrix of the assembled level operator, inverted densely; every
    Dirichlet DoF is its own 1x1 identity block.  One step is
    u <- u + omega * sum_T R_T^T S_TT^{-1} R_T (f - S u).
  * vertex-patch smoother (Section 5, named there as the extension of the cell-wise
    smoother that gives robustness in p): one block per interior vertex v of the
    level, on the lattice nodes strictly inside the 2^d cells around v, times the
    temporal DoFs of one time cell; exact (principal submatrix) or separable
    (Kronecker product of the per-axis principal submatrices of the assembled 1D
    matrices, with the mean coefficient of the patch).  Summed like the cell blocks.
  * omega (eq. relaxation): 2 / (lambda_max + lambda_min) from real parts of the
    Ritz values of 15 Arnoldi steps on ASM * S, clamped to (0, 1].  Optional
    alternative (omega_rule < 0): |omega_rule| / lambda_max.
  * coarsest level: exact sparse LU.  V-cycle: Alg. stmg with nu1 = nu2 = n_smooth
    and zero initial guesses.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import basis, spatial, spacetime, temporal


# --------------------------------------------------------------------------- hierarchy

def level_spaces(fine: spatial.Space, min_p: int = 1, coarse_cells: int = 2) -> List[spatial.Space]:
    """Spaces from finest to coarsest."""
    out = [fine]
    cur = fine
    while cur.p > min_p:
        cur = spatial.Space(dim=cur.dim, cells=cur.cells, p=max(min_p, cur.p // 2), verts=cur.verts,
                            lo=cur.lo, hi=cur.hi, coef_fine=cur.coef_fine,
                            fine_cells=cur.fine_cells, ratio=cur.ratio)
        out.append(cur)
    while all(c % 2 == 0 and c // 2 >= coarse_cells for c in cur.cells):
        verts = None
        if cur.verts is not None:
            sl = tuple(slice(None, None, 2) for _ in range(cur.dim)) + (slice(None),)
            verts = np.ascontiguousarray(cur.verts[sl])
        cur = spatial.Space(dim=cur.dim, cells=tuple(c // 2 for c in cur.cells), p=cur.p,
                            verts=verts, lo=cur.lo, hi=cur.hi, coef_fine=cur.coef_fine,
                            fine_cells=cur.fine_cells, ratio=cur.ratio * 2)
        out.append(cur)
    return out


def _node_reference(space: spatial.Space):
    """Per lattice node of `space`: a containing cell (coords) and the reference coordinate."""
    nodes1 = basis.gauss_lobatto(space.n)
    per_dim = []
    for d in range(space.dim):
        g = np.arange(space.nodes[d])
        cell = np.minimum(g // space.p, space.cells[d] - 1)
        loc = g - cell * space.p
        per_dim.append((cell, nodes1[loc]))
    return per_dim


def prolongation(coarse: spatial.Space, fine: spatial.Space) -> sp.csr_matrix:
    """P[g_f, g_c] = coarse basis function g_c evaluated at fine node g_f (all lattice nodes)."""
    if coarse.cells == fine.cells:
        h_ratio = 1
    else:
        h_ratio = fine.cells[0] // coarse.cells[0]
    cnodes = basis.gauss_lobatto(coarse.n)
    fref = _node_reference(fine)
    rows_1d = []
    for d in range(fine.dim):
        fcell, fxi = fref[d]
        ccell = np.minimum(fcell // h_ratio, coarse.cells[d] - 1)
        cxi = ((fcell - ccell * h_ratio) + fxi) / h_ratio
        V, _ = basis.lagrange(cnodes, cxi)                          # (N_f_d, p_c + 1)
        rows_1d.append((ccell, V))
    # d-dimensional evaluation: product of 1D factors over the coarse cell's nodes
    Nf = fine.nodes
    Nc = coarse.nodes
    grids = np.meshgrid(*[np.arange(m) for m in Nf[::-1]], indexing="ij")
    gf = [g.ravel() for g in grids[::-1]]
    nloc = coarse.n
    locs = np.meshgrid(*[np.arange(nloc)] * fine.dim, indexing="ij")
    locs = [l.ravel() for l in locs[::-1]]
    rows, cols, vals = [], [], []
    fidx = np.zeros(len(gf[0]), dtype=np.int64)
    stride = 1
    for d in range(fine.dim):
        fidx += gf[d] * stride
        stride *= Nf[d]
    for a in range(len(locs[0])):
        val = np.ones(len(gf[0]))
        cidx = np.zeros(len(gf[0]), dtype=np.int64)
        stride = 1
        for d in range(fine.dim):
            ccell, V = rows_1d[d]
            val = val * V[gf[d], locs[d][a]]
            cidx += (ccell[gf[d]] * coarse.p + locs[d][a]) * stride
            stride *= Nc[d]
        nz = np.abs(val) > 0
        rows.append(fidx[nz])
        cols.append(cidx[nz])
        vals.append(val[nz])
    P = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(fine.n_x, coarse.n_x))
    # a fine node on a coarse cell interface receives the same value from both sides;
    # the construction above visits exactly one coarse cell per fine node.
    return P


# --------------------------------------------------------------------------- smoother

@dataclass
class Level:
    op: spacetime.SlabOperator
    S: sp.csr_matrix
    blocks: list = field(default_factory=list)       # (index array, dense inverse)
    omega: float = 1.0
    P: Optional[sp.csr_matrix] = None                # from the next coarser level to this one
    Pt: Optional[np.ndarray] = None                  # temporal prolongation instead of P
    lu: object = None


def asm_blocks(op: spacetime.SlabOperator, S: sp.csr_matrix):
    """(indices, inverse of the principal submatrix) for every space-time cell K x I_m."""
    space, sl = op.space, op.slab
    dofs = space.cell_dofs()
    bm = op.bmask
    nc = sl.nt_cell
    c = sl.n_t // nc
    Nx = space.n_x
    S = S.tocsr()
    out = []
    for K in range(space.n_cells):
        sdofs = dofs[K][~bm[dofs[K]]]
        if len(sdofs) == 0:
            continue
        for m in range(c):
            idx = np.concatenate([(m * nc + i) * Nx + sdofs for i in range(nc)])
            B = S[idx][:, idx].toarray()
            out.append((idx, np.linalg.inv(B)))
    return out


def _assembled_1d(n_cells: int, p: int, h: float):
    """Assembled 1D Q_p mass and stiffness matrices ((p+1)-point Gauss, GLL nodes) on a
    uniform line of n_cells cells of length h (all nodes, no boundary condition)."""
    xq, wq = basis.gauss(p + 1)
    V, D = basis.lagrange(basis.gauss_lobatto(p + 1), xq)
    Me = h * (V.T * wq) @ V
    Ae = (D.T * wq) @ D / h
    N = p * n_cells + 1
    M = np.zeros((N, N))
    A = np.zeros((N, N))
    for c in range(n_cells):
        sl = slice(c * p, c * p + p + 1)
        M[sl, sl] += Me
        A[sl, sl] += Ae
    return M, A


def fdm_cell(space: spatial.Space, cc, one_d, coef) -> tuple:
    """Separable surrogate (M~, A~) of cell cc on its interior nodes (see fdm_blocks)."""
    d, p, r = space.dim, space.p, space.ratio
    Ms, As = [], []
    for a in range(d):
        g0 = cc[a] * p
        idx = [g0 + l for l in range(p + 1) if 0 < g0 + l < p * space.cells[a]]
        M1, A1 = one_d[a]
        Ms.append(M1[np.ix_(idx, idx)])
        As.append(A1[np.ix_(idx, idx)])
    box = tuple(slice(cc[a] * r, (cc[a] + 1) * r) for a in reversed(range(d)))
    rho = float(np.mean(coef[box]))
    if d == 2:
        Mt = np.kron(Ms[1], Ms[0])
        At = rho * (np.kron(As[1], Ms[0]) + np.kron(Ms[1], As[0]))
    else:
        Mt = np.kron(Ms[2], np.kron(Ms[1], Ms[0]))
        At = rho * (np.kron(As[2], np.kron(Ms[1], Ms[0])) + np.kron(Ms[2], np.kron(As[1], Ms[0]))
                    + np.kron(Ms[2], np.kron(Ms[1], As[0])))
    return Mt, At


def fdm_setup(space: spatial.Space):
    """Per-axis assembled 1D matrices and the finest coefficient array of a Cartesian level."""
    if space.verts is not None:
        raise ValueError("the separable surrogate needs a Cartesian level")
    one_d = [_assembled_1d(space.cells[a], space.p, (space.hi[a] - space.lo[a]) / space.cells[a])
             for a in range(space.dim)]
    return one_d, space.coef_fine.reshape(tuple(space.fine_cells[::-1]))


def fdm_blocks(op: spacetime.SlabOperator):
    """Separable surrogate blocks of the additive Schwarz smoother (Cartesian levels only).

    For cell K the spatial blocks are replaced by Kronecker products of per-axis principal
    submatrices of the assembled 1D matrices on K's interior nodes,
      M~ = M_z (x) M_y (x) M_x,   A~ = rho_K (A_z (x) M_y (x) M_x + M_z (x) A_y (x) M_x + M_z (x) M_y (x) A_x),
    with rho_K the mean coefficient of the cell; the block is M_tau (x) A~ + Ntilde (x) M~ for
    every time cell.  With a constant coefficient this is the exact principal block.
    Returns (indices, inverse) pairs in the layout of asm_blocks."""
    space, sl = op.space, op.slab
    one_d, coef = fdm_setup(space)
    dofs = space.cell_dofs()
    bm = op.bmask
    nc = sl.nt_cell
    c = sl.n_t // nc
    Nx = space.n_x
    out = []
    for K, cc in enumerate(space.cell_coords()):
        sdofs = dofs[K][~bm[dofs[K]]]
        if len(sdofs) == 0:
            continue
        Mt, At = fdm_cell(space, cc, one_d, coef)
        inv = np.linalg.inv(np.kron(sl.M_tau, At) + np.kron(sl.N_tilde, Mt))
        for m in range(c):
            idx = np.concatenate([(m * nc + i) * Nx + sdofs for i in range(nc)])
            out.append((idx, inv))
    return out


def vertex_patches(space: spatial.Space):
    """(vertex, nodes) for every interior vertex of the cell lattice: vertex coordinates v with
    1 <= v_a <= cells_a - 1, and the global indices of the lattice nodes strictly inside the 2^d
    cells around v (p (v_a - 1) < g_a < p (v_a + 1) per axis, x fastest)."""
    d, p = space.dim, space.p
    N = space.nodes
    ranges = [range(1, space.cells[a]) for a in range(d)]
    out = []
    for v in np.array(np.meshgrid(*ranges[::-1], indexing="ij")).reshape(d, -1).T[:, ::-1]:
        axes = [np.arange(p * (v[a] - 1) + 1, p * (v[a] + 1)) for a in range(d)]
        g = np.zeros(1, dtype=np.int64)
        stride = 1
        for a in range(d):
            g = (g[None, :] + axes[a][:, None] * stride).ravel()
            stride *= N[a]
        out.append((tuple(int(x) for x in v), np.sort(g)))
    return out


def patch_blocks(op: spacetime.SlabOperator, S: sp.csr_matrix):
    """Exact vertex-patch blocks: (indices, inverse of the principal submatrix) for every interior
    vertex patch times every time cell."""
    sl = op.slab
    nc = sl.nt_cell
    c = sl.n_t // nc
    Nx = op.space.n_x
    S = S.tocsr()
    out = []
    for _, nodes in vertex_patches(op.space):
        for m in range(c):
            idx = np.concatenate([(m * nc + i) * Nx + nodes for i in range(nc)])
            out.append((idx, np.linalg.inv(S[idx][:, idx].toarray())))
    return out


def fdm_patch_blocks(op: spacetime.SlabOperator):
    """Separable vertex-patch blocks (Cartesian levels): per axis the principal submatrix of the
    assembled 1D matrices on the patch's 2p - 1 inner nodes, M~ = M_z (x) M_y (x) M_x,
    A~ = rho_v (A_z (x) M_y (x) M_x + M_z (x) A_y (x) M_x + M_z (x) M_y (x) A_x) with rho_v the mean
    finest coefficient over the patch's 2^d cells; block M_tau (x) A~ + Ntilde (x) M~.  With a
    constant coefficient this is the exact patch block."""
    space, sl = op.space, op.slab
    one_d, coef = fdm_setup(space)
    d, p, r = space.dim, space.p, space.ratio
    nc = sl.nt_cell
    c = sl.n_t // nc
    Nx = space.n_x
    out = []
    for v, nodes in vertex_patches(space):
        Ms, As = [], []
        for a in range(d):
            idx = np.arange(p * (v[a] - 1) + 1, p * (v[a] + 1))
            Ms.append(one_d[a][0][np.ix_(idx, idx)])
            As.append(one_d[a][1][np.ix_(idx, idx)])
        box = tuple(slice((v[a] - 1) * r, (v[a] + 1) * r) for a in reversed(range(d)))
        rho = float(np.mean(coef[box]))
        if d == 2:
            Mt = np.kron(Ms[1], Ms[0])
            At = rho * (np.kron(As[1], Ms[0]) + np.kron(Ms[1], As[0]))
        else:
            Mt = np.kron(Ms[2], np.kron(Ms[1], Ms[0]))
            At = rho * (np.kron(As[2], np.kron(Ms[1], Ms[0])) + np.kron(Ms[2], np.kron(As[1], Ms[0]))
                        + np.kron(Ms[2], np.kron(Ms[1], As[0])))
        inv = np.linalg.inv(np.kron(sl.M_tau, At) + np.kron(sl.N_tilde, Mt))
        for m in range(c):
            idx = np.concatenate([(m * nc + i) * Nx + nodes for i in range(nc)])
            out.append((idx, inv))
    return out


def smoother_blocks(op: spacetime.SlabOperator, S: sp.csr_matrix, asm_variant: int):
    """Blocks of the additive Schwarz smoother: 0 exact cell blocks, 1 separable cell blocks,
    2 separable vertex patches, 3 exact vertex patches."""
    if asm_variant == 0:
        return asm_blocks(op, S)
    if asm_variant == 1:
        return fdm_blocks(op)
    if asm_variant == 2:
        return fdm_patch_blocks(op)
    if asm_variant == 3:
        return patch_blocks(op, S)
    raise ValueError("asm_variant must be 0..3")


def asm_apply(level: Level, r: np.ndarray) -> np.ndarray:
    """sum_T R_T^T S_TT^{-1} R_T r, plus the identity on Dirichlet DoFs."""
    r = r.ravel()
    z = np.zeros_like(r)
    for idx, inv in level.blocks:
        z[idx] += inv @ r[idx]
    nt = level.op.n_t
    bfull = np.tile(level.op.bmask, nt)
    z[bfull] += r[bfull]
    return z


def smooth(level: Level, f: np.ndarray, u: np.ndarray, steps: int, omega: Optional[float] = None):
    w = level.omega if omega is None else omega
    f = f.ravel()
    u = u.ravel().copy()
    for _ in range(steps):
        u = u + w * asm_apply(level, f - level.S @ u)
    return u


def arnoldi_start(n_t: int, bmask: np.ndarray) -> np.ndarray:
    """Deterministic start vector 1 + sin(0.7 g + 1.3 i + 0.1)/2 on interior DoFs."""
    g = np.arange(len(bmask), dtype=np.float64)
    i = np.arange(n_t, dtype=np.float64)
    v = 1.0 + 0.5 * np.sin(0.7 * g[None, :] + 1.3 * i[:, None] + 0.1)
    v[:, bmask] = 0.0
    return v.ravel()


def estimate_omega(level: Level, steps: int = 15, rule: float = 0.0) -> float:
    """omega = 2/(lambda_max + lambda_min) from Arnoldi Ritz values of ASM * S (eq. relaxation).

    rule < 0 selects |rule| / lambda_max instead: the paper's rule balances the extreme
    eigenvalues, which for high p leaves the top of the spectrum almost undamped
    (factor close to -1); scaling by the largest Ritz value damps it.
    """
    v = arnoldi_start(level.op.n_t, level.op.bmask)
    n = len(v)
    V = np.zeros((steps + 1, n))
    H = np.zeros((steps + 1, steps))
    V[0] = v / np.linalg.norm(v)
    m = steps
    for j in range(steps):
        w = asm_apply(level, level.S @ V[j])
        # Gram-Schmidt twice: Ritz values are eigenvalue estimates only for an orthonormal
        # basis, and one pass loses orthogonality on clustered, non-normal spectra
        for _ in range(2):
            for i in range(j + 1):
                c = V[i] @ w
                H[i, j] += c
                w = w - c * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] < 1e-14:
            m = j + 1
            break
        V[j + 1] = w / H[j + 1, j]
    ev = np.linalg.eigvals(H[:m, :m]).real
    om = -rule / ev.max() if rule < 0 else 2.0 / (ev.max() + ev.min())
    return float(min(max(om, 1e-3), 1.0))


# --------------------------------------------------------------------------- hierarchy object

class Hierarchy:
    """Levels ordered coarsest (index 0) to finest (index L), as in Alg. stmg."""

    def __init__(self, fine_op: spacetime.SlabOperator, min_p: int = 1, coarse_cells: int = 2,
                 omegas: Optional[List[float]] = None, n_smooth: int = 1, omega_rule: float = 0.0,
                 asm_variant: int = 0, time_mg: bool = False):
        spaces = level_spaces(fine_op.space, min_p, coarse_cells)[::-1]
        # (space, slab) per level, coarsest first: with time_mg, temporal levels on the coarsest
        # spatial mesh come below the spatial ones ("first in space, then in time")
        pairs = [(sp, fine_op.slab) for sp in spaces]
        # no temporal levels when the coarsest spatial mesh has no interior node (nothing to coarsen)
        if time_mg and all(n >= 3 for n in spaces[0].nodes):
            for sl in temporal.time_levels(fine_op.slab):
                pairs.insert(0, (spaces[0], sl))
        self.n_smooth = n_smooth
        self.levels: List[Level] = []
        for i, (space, sl) in enumerate(pairs):
            op = fine_op if i == len(pairs) - 1 else spacetime.build(space, sl)
            lev = Level(op=op, S=op.matrix())
            if i == 0:
                lev.lu = spla.splu(lev.S.tocsc())
            else:
                lev.blocks = smoother_blocks(op, lev.S, asm_variant)
                if pairs[i - 1][1] is not sl:
                    lev.Pt = temporal.prolongation(sl, pairs[i - 1][1])
                else:
                    lev.P = prolongation(pairs[i - 1][0], space)
            self.levels.append(lev)
        for i, lev in enumerate(self.levels):
            if i == 0:
                continue
            if omegas is not None:
                lev.omega = omegas[i]
            else:
                lev.omega = estimate_omega(lev, rule=omega_rule)

    @property
    def omegas(self):
        return [lev.omega for lev in self.levels]

    def prolong(self, i: int, ec: np.ndarray) -> np.ndarray:
        """Level i-1 -> level i on interior nodes, applied to every temporal row."""
        lev, coarse = self.levels[i], self.levels[i - 1]
        E = ec.reshape(coarse.op.n_t, coarse.op.n_x) * (~coarse.op.bmask)[None, :]
        out = lev.Pt @ E if lev.Pt is not None else (lev.P @ E.T).T
        out[:, lev.op.bmask] = 0.0
        return out.ravel()

    def restrict(self, i: int, r: np.ndarray) -> np.ndarray:
        """Level i -> level i-1: the transpose of prolong."""
        lev, coarse = self.levels[i], self.levels[i - 1]
        R = r.reshape(lev.op.n_t, lev.op.n_x) * (~lev.op.bmask)[None, :]
        out = lev.Pt.T @ R if lev.Pt is not None else (lev.P.T @ R.T).T
        out[:, coarse.op.bmask] = 0.0
        return out.ravel()

    def vcycle(self, f: np.ndarray, i: Optional[int] = None) -> np.ndarray:
        """Alg. stmg with zero initial guess: returns u ~ S_i^{-1} f."""
        if i is None:
            i = len(self.levels) - 1
        lev = self.levels[i]
        f = f.ravel()
        if i == 0:
            return lev.lu.solve(f)
        u = np.zeros_like(f)
        u = smooth(lev, f, u, self.n_smooth)
        r = f - lev.S @ u
        ec = self.vcycle(self.restrict(i, r), i - 1)
        u = u + self.prolong(i, ec)
        u = smooth(lev, f, u, self.n_smooth)
        return u
