"""Relaxation study on the oracle (CPU, minutes per case): FGMRES(30) iterations to a 1e-8 true
relative residual with one oracle V-cycle per iteration, for several choices of omega_l in
eq. vanka, on small members of the benchmark families:
  * omega_l = 1;
  * eq. relaxation, 2 / (lambda_max + lambda_min), from 80 Arnoldi steps (close to the extreme
    eigenvalues) and from the 15 steps the library uses;
  * eq. relaxation with lambda_min := lambda_max / 3, i.e. omega_l = 1.5 / lambda_max;
  * omega_l = 1 / lambda_max.
The cell blocks are applied in batches (same arithmetic as oracle.mg.asm_apply, grouped by block
size) so that the 1e5-DoF cases finish.  Not collected by pytest; run
    python tests/omega_study.py c2 c2b c4 q2 q3
"""
import os
import sys
import time
import numpy as np
sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import stmg_inputs as si
from oracle import mg, spacetime, krylov

def fast_blocks(lev):
    groups = {}
    for idx, inv in lev.blocks:
        groups.setdefault(len(idx), []).append((idx, inv))
    out = []
    for n, lst in groups.items():
        I = np.stack([a for a, _ in lst]); B = np.stack([b for _, b in lst])
        out.append((I, B))
    lev._fast = out
    nt = lev.op.n_t
    lev._bfull = np.tile(lev.op.bmask, nt)

def asm_apply_fast(level, r):
    r = r.ravel(); z = np.zeros_like(r)
    for I, B in level._fast:
        v = np.einsum('bij,bj->bi', B, r[I])
        np.add.at(z, I.ravel(), v.ravel())
    z[level._bfull] += r[level._bfull]
    return z
mg.asm_apply = asm_apply_fast

def ritz(lev, steps):
    v = mg.arnoldi_start(lev.op.n_t, lev.op.bmask)
    n = len(v); V = np.zeros((steps + 1, n)); H = np.zeros((steps + 1, steps))
    V[0] = v / np.linalg.norm(v); m = steps
    for j in range(steps):
        w = asm_apply_fast(lev, lev.S @ V[j])
        for _ in range(2):
            c = V[:j+1] @ w; H[:j+1, j] += c; w = w - V[:j+1].T @ c
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] < 1e-14: m = j + 1; break
        V[j + 1] = w / H[j + 1, j]
    ev = np.linalg.eigvals(H[:m, :m]).real
    return ev.min(), ev.max()

def run(name, cfg, rhs_seed=11, restart=30, maxit=150):
    verts, coef = si.draw_problem(cfg)
    op = spacetime.from_config(cfg, verts, coef)
    t0 = time.time()
    H = mg.Hierarchy(op, omegas=[1.0] * 32, asm_variant=0)
    L = len(H.levels)
    est = {}
    for l in range(1, L):
        fast_blocks(H.levels[l])
        est[l] = dict(n=int(H.levels[l].S.shape[0]), r15=ritz(H.levels[l], 15), r80=ritz(H.levels[l], 80))
    print(f"== {name}: levels {L}, N_st {cfg.n_st}, setup {time.time()-t0:.0f}s", flush=True)
    for l in range(1, L):
        e = est[l]
        print(f"  level {l} n={e['n']}: ritz15 [{e['r15'][0]:.4f}, {e['r15'][1]:.4f}]  ritz80 [{e['r80'][0]:.4f}, {e['r80'][1]:.4f}]", flush=True)
    b = si.random_slab_vector(cfg, rhs_seed).ravel()
    settings = {
        "omega=1": lambda e: 1.0,
        "eq.relaxation, 80-step Ritz": lambda e: 2.0 / (e["r80"][0] + e["r80"][1]),
        "eq.relaxation, 15-step Ritz": lambda e: 2.0 / (e["r15"][0] + e["r15"][1]),
        "1.5/lmax (lmin := lmax/3)": lambda e: 1.5 / e["r15"][1],
        "1/lmax": lambda e: 1.0 / e["r15"][1],
    }
    for sname, f in settings.items():
        for l in range(1, L):
            H.levels[l].omega = f(est[l])
        t1 = time.time()
        x, it, rr = krylov.fgmres(op.apply, b, H.vcycle, rtol=1e-8, restart=restart, max_iter=maxit)
        print(f"  {sname:30s}: it {it:4d} res {rr:.1e} omega {[round(H.levels[l].omega, 4) for l in range(1, L)]} ({time.time()-t1:.0f}s)", flush=True)

if __name__ == "__main__":
    which = sys.argv[1:]
    if "c2" in which:
        run("config-2 family (Q4 perturbed 10%, dG(2), c=8, tau=h/2) 4^3", si.paper_config(2).replace(n_cells=(4, 4, 4), tau=1 / 8))
    if "c2b" in which:
        run("config-2 family (Q4 perturbed 10%, dG(2), c=8, tau=h/2) 2^3", si.paper_config(2).replace(n_cells=(2, 2, 2), tau=1 / 4))
    if "q2" in which:
        run("config-5 family (Q2 dG(1) c=4, lognormal 1) 8^3", si.paper_config(5).replace(n_cells=(8, 8, 8), tau=1 / 16))
    if "c4" in which:
        run("config-4 family (Q4 dG(1) c=2, lognormal 0.5) 4^3", si.paper_config(4).replace(n_cells=(4, 4, 4), tau=1 / 8))
    if "q3" in which:
        run("config-3 family (wave Q3 cGP(2) c=4) 4^3", si.paper_config(3).replace(n_cells=(4, 4, 4), tau=1 / 8))
