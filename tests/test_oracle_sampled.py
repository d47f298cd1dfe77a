"""Pins of the oracle's single-entry evaluation (oracle.sampled) against the assembled oracle."""
import numpy as np
import pytest

import stmg_inputs as si
from oracle import mg, sampled, spacetime

CFGS = [
    si.Config(dim=3, problem=0, time_method=0, p=2, k=1, n_time_cells=2, n_cells=(3, 4, 3), tau=0.05,
              perturb=0.12, coef="lognormal", coef_sigma=1.0, seed=41),
    si.Config(dim=3, problem=1, time_method=1, p=3, k=2, n_time_cells=2, n_cells=(2, 3, 2), tau=0.04,
              coef="lognormal_checker", coef_sigma=0.5, seed=42),
    si.Config(dim=2, problem=1, time_method=0, p=4, k=2, n_time_cells=2, n_cells=(3, 3, 1), tau=0.05,
              perturb=0.1, coef="lognormal", coef_sigma=0.8, seed=43),
]


@pytest.mark.parametrize("cfg", CFGS, ids=["heat3d_q2_dg1", "wave3d_q3_cgp2", "wave2d_q4_dg2"])
def test_sampled_operator_and_asm_match_assembled(cfg):
    verts, coef = si.draw_problem(cfg)
    op = spacetime.from_config(cfg, verts, coef)
    S = op.matrix()
    smp = sampled.Sampler(cfg, verts, coef)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((cfg.n_t, op.n_x))
    pts = sampled.sample_points(cfg, 24, 6, seed=7)
    y = op.apply(x)
    ys = smp.operator_entries(x, pts)
    ref = np.array([y[i, g] for i, g in pts])
    assert np.allclose(ys, ref, rtol=1e-12, atol=1e-12 * np.abs(y).max())
    lev = mg.Level(op=op, S=S, blocks=mg.asm_blocks(op, S))
    u = 0.37 * mg.asm_apply(lev, x.ravel()).reshape(cfg.n_t, op.n_x)
    us = smp.asm_entries(x, 0.37, pts)
    ref = np.array([u[i, g] for i, g in pts])
    assert np.allclose(us, ref, rtol=1e-10, atol=1e-10 * np.abs(u).max())


def test_sample_points_cover_node_kinds():
    cfg = CFGS[0]
    pts = sampled.sample_points(cfg, 40, 8, seed=1)
    smp = sampled.Sampler(cfg, *si.draw_problem(cfg))
    counts = sorted({len(smp.cells_of_node(g)) for _, g in pts if not smp.is_boundary(g)})
    assert counts == [1, 2, 4, 8]
    assert sum(smp.is_boundary(g) for _, g in pts) == 8
    # per-cell numbering agrees with the full tables of spatial.Space
    dofs = smp.space.cell_dofs()
    bm = smp.space.boundary_mask()
    for K in (0, 5, smp.space.n_cells - 1):
        assert np.array_equal(smp.cell_nodes(K), dofs[K])
        assert np.array_equal(smp.node_boundary(dofs[K]), bm[dofs[K]])


def test_sampled_separable_step_matches_blocks():
    cfg = si.Config(dim=3, problem=0, time_method=0, p=3, k=1, n_time_cells=2, n_cells=(3, 2, 4), tau=0.05,
                    coef="lognormal", coef_sigma=1.0, seed=44)
    verts, coef = si.draw_problem(cfg)
    op = spacetime.from_config(cfg, verts, coef)
    lev = mg.Level(op=op, S=op.matrix(), blocks=mg.fdm_blocks(op))
    x = np.random.default_rng(9).standard_normal((cfg.n_t, op.n_x))
    u = 0.4 * mg.asm_apply(lev, x.ravel()).reshape(cfg.n_t, op.n_x)
    smp = sampled.Sampler(cfg, verts, coef)
    pts = sampled.sample_points(cfg, 20, 4, seed=3)
    got = smp.asm_entries(x, 0.4, pts, separable=True)
    ref = np.array([u[i, g] for i, g in pts])
    assert np.allclose(got, ref, rtol=1e-10, atol=1e-10 * np.abs(u).max())


@pytest.mark.parametrize("cfg", [
    si.Config(dim=3, problem=0, time_method=0, p=4, k=1, n_time_cells=2, n_cells=(4, 6, 4), tau=0.05,
              perturb=0.1, coef="lognormal", coef_sigma=1.0, seed=45),
    si.Config(dim=3, problem=1, time_method=1, p=3, k=2, n_time_cells=1, n_cells=(4, 4, 8), tau=0.04,
              coef="lognormal", coef_sigma=0.5, seed=46),
    si.Config(dim=2, problem=0, time_method=0, p=2, k=0, n_time_cells=2, n_cells=(8, 4, 1), tau=0.05,
              coef="lognormal", coef_sigma=0.5, seed=47),
], ids=["heat3d_q4_perturbed", "wave3d_q3", "heat2d_q2"])
def test_sampled_transfers_match_hierarchy(cfg):
    """Single entries of P e and P^T r on every level pair (p- and h-transfers) equal those of the
    assembled transfers of oracle.mg.Hierarchy."""
    verts, coef = si.draw_problem(cfg)
    op = spacetime.from_config(cfg, verts, coef)
    H = mg.Hierarchy(op, omegas=[1.0] * 16)
    smp = sampled.Sampler(cfg, verts, coef)
    spaces = smp.level_spaces()
    L = len(H.levels)
    assert len(spaces) == L and L >= 3
    rng = np.random.default_rng(11)
    kinds = set()
    for l in range(L - 1):
        io = L - 1 - l
        fine, coarse = spaces[l], spaces[l + 1]
        assert H.levels[io].op.n_x == fine.n_x and H.levels[io - 1].op.n_x == coarse.n_x
        kinds.add("p" if fine.cells == coarse.cells else "h")
        ec = rng.standard_normal((cfg.n_t, coarse.n_x))
        rf = rng.standard_normal((cfg.n_t, fine.n_x))
        pe = H.prolong(io, ec.ravel()).reshape(cfg.n_t, fine.n_x)
        rr = H.restrict(io, rf.ravel()).reshape(cfg.n_t, coarse.n_x)
        ptf = sampled.lattice_points(fine.p, fine.cells, cfg.n_t, 40, 8, seed=l)
        ptc = sampled.lattice_points(coarse.p, coarse.cells, cfg.n_t, 40, 8, seed=100 + l)
        got = smp.prolong_entries(ec, l, ptf)
        assert np.allclose(got, [pe[i, g] for i, g in ptf], rtol=1e-13, atol=1e-13 * np.abs(pe).max())
        got = smp.restrict_entries(rf, l, ptc)
        assert np.allclose(got, [rr[i, g] for i, g in ptc], rtol=1e-13, atol=1e-13 * np.abs(rr).max())
    assert kinds == {"p", "h"}
