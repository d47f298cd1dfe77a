"""Shared helpers of the GPU parity tests (oracle on the CPU, library through the C ABI)."""
import numpy as np

import stmg_inputs as si
from oracle import mg, spacetime

# cases that the oracle assembles in seconds but that span several cells, levels and a ragged mix
# of Dirichlet and interior nodes
CASES = {
    "heat2d_q2_dg1": si.paper_config(1),
    "heat2d_q4_cgp2_pert": si.Config(dim=2, problem=0, time_method=1, p=4, k=2, n_time_cells=3,
                                     n_cells=(6, 4, 1), tau=0.05, perturb=0.15, coef="lognormal",
                                     coef_sigma=1.0, seed=21),
    "wave2d_q3_dg2": si.Config(dim=2, problem=1, time_method=0, p=3, k=2, n_time_cells=2,
                               n_cells=(4, 4, 1), tau=0.05, coef="lognormal", coef_sigma=0.7, seed=22),
    "heat3d_q2_dg1_pert": si.small_configs()[1],
    "wave3d_q3_cgp2": si.small_configs()[2],
    "heat3d_q4_dg2_pert": si.Config(dim=3, problem=0, time_method=0, p=4, k=2, n_time_cells=2,
                                    n_cells=(2, 2, 2), tau=0.05, perturb=0.1, coef="lognormal",
                                    coef_sigma=0.5, seed=23),
    "heat3d_q1_dg0": si.Config(dim=3, problem=0, time_method=0, p=1, k=0, n_time_cells=3,
                               n_cells=(4, 4, 4), tau=0.1, coef="lognormal", coef_sigma=1.0, seed=24),
    "wave3d_q2_cgp1_ragged": si.Config(dim=3, problem=1, time_method=1, p=2, k=1, n_time_cells=2,
                                       n_cells=(3, 2, 5), tau=0.05, perturb=0.1, seed=25),
    # n_t >= 8: the smoother runs on the matrix cores
    "heat3d_q4_dg2_c4_pert": si.Config(dim=3, problem=0, time_method=0, p=4, k=2, n_time_cells=4,
                                       n_cells=(2, 3, 2), tau=0.05, perturb=0.1, coef="lognormal",
                                       coef_sigma=0.8, seed=26),
    "wave3d_q3_cgp2_c4": si.Config(dim=3, problem=1, time_method=1, p=3, k=2, n_time_cells=4,
                                   n_cells=(3, 2, 2), tau=0.05, coef="lognormal", coef_sigma=1.0, seed=27),
    "heat3d_q2_dg1_c8_ragged": si.Config(dim=3, problem=0, time_method=0, p=2, k=1, n_time_cells=8,
                                         n_cells=(3, 4, 2), tau=0.05, perturb=0.1, seed=28),
    # Cartesian boxes with one coefficient per cell (brick operator): several bricks per direction
    # with a ragged last brick, non-cubic cells
    "heat3d_q4_dg1_brick": si.Config(dim=3, problem=0, time_method=0, p=4, k=1, n_time_cells=2,
                                     n_cells=(5, 4, 3), tau=0.02, hi=(1.0, 0.8, 1.2), coef="lognormal",
                                     coef_sigma=0.5, seed=29),
    "heat3d_q2_dg1_c4_brick": si.Config(dim=3, problem=0, time_method=0, p=2, k=1, n_time_cells=4,
                                        n_cells=(9, 6, 5), tau=0.03, coef="lognormal", coef_sigma=1.0,
                                        seed=30),
    "wave3d_q3_cgp2_brick": si.Config(dim=3, problem=1, time_method=1, p=3, k=2, n_time_cells=2,
                                      n_cells=(4, 5, 3), tau=0.02, hi=(1.0, 1.3, 0.9),
                                      coef="lognormal_checker", coef_sigma=1.0, seed=31),
    # long in x: many bricks along x
    "heat3d_q2_dg1_long": si.Config(dim=3, problem=0, time_method=0, p=2, k=1, n_time_cells=1,
                                    n_cells=(44, 3, 2), tau=0.01, hi=(4.0, 0.3, 0.2), coef="lognormal",
                                    coef_sigma=0.7, seed=32),
}

# Cartesian cases with at least two cells per direction (vertex-patch smoother)
PATCH_CASES = ["heat2d_q2_dg1", "wave2d_q3_dg2", "heat3d_q1_dg0", "wave3d_q3_cgp2_c4", "heat3d_q4_dg1_brick",
               "heat3d_q2_dg1_c4_brick"]

# Cartesian 3D cases whose operator runs on the brick kernel by default
BRICK_CASES = ["heat3d_q4_dg1_brick", "heat3d_q2_dg1_c4_brick", "wave3d_q3_cgp2_brick", "heat3d_q1_dg0",
               "wave3d_q3_cgp2_c4", "heat3d_q2_dg1_long"]


def problem(name):
    cfg = CASES[name]
    verts, coef = si.draw_problem(cfg)
    return cfg, verts, coef


def oracle_op(cfg, verts, coef):
    return spacetime.from_config(cfg, verts, coef)


def rel_err(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))
