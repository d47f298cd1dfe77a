"""Structural-health-monitoring wave example (Section 4.2) on one GPU: slab-by-slab time
marching of the acoustic wave equation on [-1, 1]^3 x [0, T] with the layered medium of
eq. rho (optionally perturbed per initial-mesh cell), the pulse of eq. initial-shm, cGP(k) in
time and Q_p in space; the point values of the displacement at the three goal points are
recorded at every temporal DoF.

Every step runs in the library: stmg_slab_rhs (coupling to the previous slab), stmg_solve
(FGMRES with the FP32 V-cycle), stmg_wave_velocity, stmg_point_values.

CLI:  python -m paper_2408_04372_amd.shm --level 3 --p 3 --k 2 --c 4 --T 2.0 [--rough]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(cfg, T: float, precision: int = 1, rtol: float = 1e-8, max_slabs: int = 10 ** 9, log=None, **kw):
    """March from t = 0 to T in slabs of cfg.n_time_cells cells.  Returns (times, values,
    per-slab info, final (u, v) as host arrays)."""
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import torch
    import stmg_inputs as si
    from paper_2408_04372_amd import Handle, _lib
    verts, coef = si.draw_problem(cfg)
    h = Handle(cfg, verts, coef, precision=precision, rtol=rtol, omega=-1.5,
               vcycle_dtypes=2 if precision == 1 else 3, **kw)
    n_t, nx = cfg.n_t, h.info["n_x"][0]
    dev = torch.device("cuda:0")
    u0 = torch.from_numpy(si.shm_initial_values(h.node_coordinates())).to(dev).contiguous()
    v0 = torch.zeros_like(u0)
    zero = torch.zeros_like(u0)
    b = torch.empty(n_t * nx, dtype=torch.float64, device=dev)
    U = torch.zeros_like(b)
    V = torch.empty_like(b)
    slab_len = cfg.n_time_cells * cfg.tau
    n_slabs = min(int(round(T / slab_len)), max_slabs)
    times, values, infos = [], [], []
    t0 = 0.0
    wall = time.perf_counter()
    for sl in range(n_slabs):
        h.slab_rhs(b, None, zero, u0, v0)
        U.zero_()
        info = h.solve(b, U, raise_on_noconv=True)
        h.wave_velocity(U, V, u0, v0)
        vals = h.point_values(U, si.SHM_POINTS)          # (n_t, 3)
        # the library's temporal DoF times of this slab (cGP: the last k Gauss-Lobatto points per cell)
        slab_times = _lib.temporal_dof_times(cfg.problem, cfg.time_method, cfg.k, cfg.n_time_cells, cfg.tau, t0)
        for i in range(n_t):
            times.append(float(slab_times[i]))
            values.append(vals[i].tolist())
        u0 = U.view(n_t, nx)[-1].clone()
        v0 = V.view(n_t, nx)[-1].clone()
        infos.append({"slab": sl, "iterations": info["iterations"], "seconds": info["seconds"],
                      "rel_residual": info["rel_residual"]})
        if log:
            log(f"slab {sl}: t = {t0 + slab_len:.4f}, {info['iterations']} it, {info['seconds']:.3f} s")
        t0 += slab_len
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall
    out_u, out_v = u0.cpu().numpy(), v0.cpu().numpy()
    summary = {"workload": cfg.name, "n_st_per_slab": n_t * nx, "slabs": n_slabs, "wall_s": wall,
               "dofs_per_s": n_t * nx * n_slabs / wall, "iterations_mean": float(np.mean([i["iterations"] for i in infos]))}
    h.close()
    return np.array(times), np.array(values), infos, summary, (out_u, out_v)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--level", type=int, default=3)
    ap.add_argument("--p", type=int, default=3)
    ap.add_argument("--k", type=int, default=2)
    ap.add_argument("--c", type=int, default=4)
    ap.add_argument("--T", type=float, default=2.0)
    ap.add_argument("--rough", action="store_true")
    ap.add_argument("--max-slabs", type=int, default=10 ** 9)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import stmg_inputs as si
    cfg = si.shm_config(args.level, args.p, args.k, args.c, rough=args.rough)
    times, values, infos, summary, _ = run(cfg, args.T, max_slabs=args.max_slabs,
                                           log=lambda m: print(m, file=sys.stderr, flush=True))
    print(json.dumps(summary))
    if args.out:
        np.savez(args.out, times=times, values=values)


if __name__ == "__main__":
    main()
