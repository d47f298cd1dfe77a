"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the space-time method itself: it only
describes problem configurations and draws random numbers (mesh vertex
perturbations, cell coefficients, right-hand-side vectors and smooth source
coefficients).  Both the CPU oracle and the GPU library consume what it
produces, so neither side depends on the other.

Draw order for one configuration (one ``numpy.random.Generator(PCG64(seed))``):
vertex perturbation, then cell coefficients, then source coefficients.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np

HEAT, WAVE = 0, 1
DG, CGP = 0, 1
PREC_FP64, PREC_FP32, PREC_LEARNED = 0, 1, 2


@dataclass
class Config:
    """One slab problem: domain [lo, hi]^d, n_cells Q_p cells, c time cells of length tau."""

    dim: int = 3
    problem: int = HEAT          # 0 heat, 1 acoustic wave (first-order system, condensed)
    time_method: int = DG        # 0 dG(k), 1 cGP(k)
    p: int = 2                   # spatial degree Q_p
    k: int = 1                   # temporal degree
    n_time_cells: int = 4        # c: time cells batched into one slab
    n_cells: Tuple[int, int, int] = (8, 8, 1)
    t0: float = 0.0
    tau: float = 0.25
    lo: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    hi: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    n_smooth: int = 1
    min_p: int = 1
    coarse_cells: int = 2
    omega: float = 0.0           # > 0 fixed; 0: eq. relaxation per level; < 0: |omega| / lambda_max per level
    precision: int = PREC_FP64
    restart: int = 30
    max_iter: int = 200
    rtol: float = 1e-8
    seed: int = 1
    # input recipe (not part of the solver configuration)
    perturb: float = 0.0         # interior vertex displacement, fraction of h, uniform per component
    coef: str = "one"            # "one" | "lognormal" | "lognormal_checker" | "shm" | "shm_rough"
    coef_sigma: float = 0.0
    name: str = ""

    def replace(self, **kw) -> "Config":
        return dataclasses.replace(self, **kw)

    @property
    def cells(self) -> Tuple[int, ...]:
        return tuple(self.n_cells[: self.dim])

    @property
    def n_t(self) -> int:
        per = self.k + 1 if self.time_method == DG else self.k
        return self.n_time_cells * per

    @property
    def nodes(self) -> Tuple[int, ...]:
        return tuple(self.p * n + 1 for n in self.cells)

    @property
    def n_x(self) -> int:
        return int(np.prod(self.nodes))

    @property
    def n_st(self) -> int:
        return self.n_x * self.n_t

    @property
    def h(self) -> Tuple[float, ...]:
        return tuple((self.hi[i] - self.lo[i]) / self.cells[i] for i in range(self.dim))


def paper_config(idx: int) -> Config:
    """The five benchmark configurations (1-based), with tau = h/2 where the paper is silent."""
    if idx == 1:
        return Config(dim=2, problem=HEAT, time_method=DG, p=2, k=1, n_time_cells=4,
                      n_cells=(8, 8, 1), tau=0.25, coef="one", seed=1,
                      name="heat2d_8x8_Q2_dG1_c4")
    if idx == 2:
        return Config(dim=3, problem=HEAT, time_method=DG, p=4, k=2, n_time_cells=8,
                      n_cells=(32, 32, 32), tau=0.5 / 32, perturb=0.1, coef="one", seed=2,
                      name="heat3d_32cube_Q4_perturbed_dG2_c8")
    if idx == 3:
        return Config(dim=3, problem=WAVE, time_method=CGP, p=3, k=2, n_time_cells=4,
                      n_cells=(64, 64, 64), tau=0.5 / 64, coef="lognormal_checker",
                      coef_sigma=1.0, precision=PREC_FP32, seed=3,
                      name="wave3d_64cube_Q3_cGP2_c4")
    if idx == 4:
        return Config(dim=3, problem=HEAT, time_method=DG, p=4, k=1, n_time_cells=2,
                      n_cells=(128, 128, 128), tau=0.5 / 128, coef="lognormal",
                      coef_sigma=0.5, precision=PREC_FP32, restart=10, seed=4,
                      name="heat3d_128cube_Q4_dG1_c2")
    if idx == 5:
        return Config(dim=3, problem=HEAT, time_method=DG, p=2, k=1, n_time_cells=4,
                      n_cells=(64, 64, 64), tau=0.5 / 64, coef="lognormal", coef_sigma=1.0,
                      precision=PREC_LEARNED, seed=5,
                      name="heat3d_64cube_Q2_dG1_c4")
    raise ValueError(idx)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def vertex_lattice(cfg: Config, rng: Optional[np.random.Generator] = None) -> Optional[np.ndarray]:
    """Vertex positions, shape (nz+1, ny+1, nx+1, 3) in 3D or (ny+1, nx+1, 2) in 2D.

    Returns None for an unperturbed (Cartesian) mesh.  Interior vertices move by
    U[-perturb*h_i, perturb*h_i] in each component i; boundary vertices stay.
    """
    if cfg.perturb == 0.0:
        return None
    d = cfg.dim
    cells = cfg.cells
    axes = [np.linspace(cfg.lo[i], cfg.hi[i], cells[i] + 1) for i in range(d)]
    grids = np.meshgrid(*axes[::-1], indexing="ij")          # slowest first
    pos = np.stack(grids[::-1], axis=-1)                      # [..., x, y, z]
    if rng is None:
        rng = _rng(cfg.seed)
    h = np.array(cfg.h)
    disp = rng.uniform(-1.0, 1.0, size=pos.shape) * (cfg.perturb * h)
    interior = np.ones(pos.shape[:-1], dtype=bool)
    for ax in range(d):
        sl = [slice(None)] * d
        sl[ax] = 0
        interior[tuple(sl)] = False
        sl[ax] = -1
        interior[tuple(sl)] = False
    pos = pos + disp * interior[..., None]
    return np.ascontiguousarray(pos)


def cell_coefficients(cfg: Config, rng: Optional[np.random.Generator] = None) -> np.ndarray:
    """One positive coefficient (kappa or c^2) per finest cell, cell order x fastest."""
    shape = tuple(cfg.cells[::-1])
    if cfg.coef == "one":
        return np.ones(shape, dtype=np.float64).ravel()
    if cfg.coef in ("shm", "shm_rough"):
        # layered medium of the structural-health-monitoring example (Section 4.2, eq. rho),
        # evaluated at cell centres; the layer interfaces y = 0.2, z = 0.2 lie on cell faces
        # for 5 * 2^r cells on [-1, 1]; "shm_rough" multiplies by c ~ U[0.4, 1.6] drawn per
        # cell of the 5 x 5 x 5 initial mesh
        h = np.array(cfg.h)
        idx = np.indices(shape)                          # (z, y, x) cell indices
        yc = cfg.lo[1] + (idx[1] + 0.5) * h[1]
        zc = cfg.lo[2] + (idx[0] + 0.5) * h[2]
        val = np.where(yc < 0.2, 1.0, np.where(zc < 0.2, 9.0, 16.0))
        if cfg.coef == "shm_rough":
            if rng is None:
                rng = _rng(cfg.seed)
            c = rng.uniform(0.4, 1.6, size=(5, 5, 5))
            sub = [np.minimum((idx[a] * 5) // shape[a], 4) for a in range(3)]
            val = val * c[sub[0], sub[1], sub[2]]
        return np.ascontiguousarray(val.ravel())
    if rng is None:
        rng = _rng(cfg.seed)
    g = rng.standard_normal(shape)
    val = np.exp(cfg.coef_sigma * g)
    if cfg.coef == "lognormal_checker":
        idx = np.indices(shape)
        par = sum(i // 8 for i in idx) % 2
        val = val * np.where(par == 1, 100.0, 1.0)
    return np.ascontiguousarray(val.ravel())


def shm_config(r: int = 3, p: int = 3, k: int = 2, n_time_cells: int = 4, rough: bool = False,
               seed: int = 7) -> Config:
    """Structural-health-monitoring wave example (Section 4.2) on [-1, 1]^3 with 5 * 2^r cells per
    direction, cGP(k) in time with tau = h / 2 (the paper refines time once more than space),
    homogeneous Dirichlet data (the paper does not state the boundary condition)."""
    n = 5 * 2 ** r
    h = 2.0 / n
    return Config(dim=3, problem=WAVE, time_method=CGP, p=p, k=k, n_time_cells=n_time_cells,
                  n_cells=(n, n, n), tau=h / 2, lo=(-1.0, -1.0, -1.0), hi=(1.0, 1.0, 1.0),
                  coef="shm_rough" if rough else "shm", precision=PREC_FP32, seed=seed,
                  name=f"shm_wave3d_{n}cube_Q{p}_cGP{k}_c{n_time_cells}" + ("_rough" if rough else ""))


def shm_initial_values(xyz: np.ndarray, s: float = 0.01) -> np.ndarray:
    """Initial displacement of the example (eq. initial-shm) at the given points (N, 3):
    exp(-|x/s|^2) (1 - |x/s|^2) for |x/s| < 1, else 0."""
    q = np.sum((np.asarray(xyz) / s) ** 2, axis=1)
    return np.where(q < 1.0, np.exp(-q) * (1.0 - q), 0.0)


SHM_POINTS = np.array([[0.75, 0.0, 0.0], [0.0, 0.0, 0.75], [0.75, 0.1, 0.75]])   # goal-quantity points


def draw_problem(cfg: Config):
    """Vertices (or None) and cell coefficients, drawn in the documented order."""
    rng = _rng(cfg.seed)
    verts = vertex_lattice(cfg, rng) if cfg.perturb != 0.0 else None
    coef = cell_coefficients(cfg, rng) if cfg.coef != "one" else cell_coefficients(cfg)
    return verts, coef


def source_coefficients(seed: int, modes: int = 4, tdeg: int = 2, dim: int = 3) -> np.ndarray:
    """gamma[a,b,c,q] ~ N(0,1)/(a^2+b^2+c^2) for a smooth random source
    f = sum gamma * prod sin(a pi x_i) * P_q(time); shape (modes,)*dim + (tdeg+1,)."""
    rng = _rng(seed)
    shape = (modes,) * dim + (tdeg + 1,)
    g = rng.standard_normal(shape)
    idx = np.indices(shape[:-1]) + 1
    den = sum(i.astype(np.float64) ** 2 for i in idx)
    return g / den[..., None]


def random_slab_vector(cfg: Config, seed: int, boundary_zero: bool = True) -> np.ndarray:
    """A standard-normal space-time vector [n_t, N_x] (x fastest), zero on the domain boundary."""
    rng = _rng(seed)
    nodes = cfg.nodes
    v = rng.standard_normal((cfg.n_t,) + tuple(nodes[::-1]))
    if boundary_zero:
        for ax in range(1, cfg.dim + 1):
            sl = [slice(None)] * (cfg.dim + 1)
            sl[ax] = 0
            v[tuple(sl)] = 0.0
            sl[ax] = -1
            v[tuple(sl)] = 0.0
    return np.ascontiguousarray(v.reshape(cfg.n_t, -1))


def small_configs():
    """Small cases the oracle finishes in seconds; they span several cells and both time methods."""
    out = [paper_config(1)]
    out.append(Config(dim=3, problem=HEAT, time_method=DG, p=2, k=1, n_time_cells=2,
                      n_cells=(4, 4, 4), tau=0.125, perturb=0.1, coef="lognormal",
                      coef_sigma=0.5, seed=11, name="heat3d_4cube_Q2_perturbed_dG1_c2"))
    out.append(Config(dim=3, problem=WAVE, time_method=CGP, p=3, k=2, n_time_cells=2,
                      n_cells=(4, 4, 4), tau=0.125, coef="lognormal_checker",
                      coef_sigma=1.0, seed=12, name="wave3d_4cube_Q3_cGP2_c2"))
    return out
