"""Benchmark: space-time DoFs/s per V-cycle and time to a 1e-8 relative residual.

One step = one stmg_solve of the all-at-once slab system from x0 = 0 to a true
relative residual of 1e-8 with FP64 FGMRES and one space-time multigrid V-cycle
per iteration (operator, cell-wise additive Schwarz smoother, h/p transfers,
coarse solve, Krylov updates: the whole hot path).  Default workload: heat
equation on the unit cube, 128^3 Cartesian Q4 cells, lognormal conductivity
(sigma 0.5) per cell, dG(1), 2 time cells per slab (5.40e8 space-time DoFs
including Dirichlet nodes), plain FP64 V-cycle with the separable cell-block
smoother, FGMRES(10).  Inputs are seeded and synthetic.

value = N_st * (V-cycles in the timed steps) / (timed seconds).

Extras: the same solve with an FP32 V-cycle (time, iterations, difference to the
FP64 solution), operator and V-cycle rates, and the other single-GPU workloads
(32^3 Q4 perturbed dG(2); 64^3 Q3 wave cGP(2); 64^3 Q2 dG(1) with the learned stage).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 4] [--no-cpu-baseline]
       [--no-extras] [--no-learned] [--extra-configs 2,3,5]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VALU_PEAK_TFLOPS = 78.6     # 256 CUs x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
FP64_MFMA_PEAK_TFLOPS = 78.6

# solver settings per workload: the separable cell blocks where exact factors do not fit
LAUNCH = {
    2: dict(asm_variant=0, restart=30),
    3: dict(asm_variant=0, restart=30),
    4: dict(asm_variant=1, restart=10),
    5: dict(asm_variant=0, restart=30),
}
OMEGA = -1.5   # omega_l = 1.5 / lambda_max of ASM * S_l per level

# committed FETCH_SIZE / WRITE_SIZE summaries of the finest-level kernels, per workload
TRAFFIC_PROFILES = {
    ("heat3d_32cube_Q4_perturbed_dG2_c8", "operator"):
        ("st_apply3_heat3d_q4_dg2_c8_hbm_traffic.md", ("op_apply.hip", "blas.hip", "device.hpp")),
    ("heat3d_32cube_Q4_perturbed_dG2_c8", "smoother"):
        ("k_asm_mfma_heat3d_q4_dg2_c8_hbm_traffic.md", ("asm.hip", "blas.hip", "device.hpp")),
    ("heat3d_128cube_Q4_dG1_c2", "operator"):
        ("st_apply3_brick_heat3d_128cube_q4_dg1_c2_hbm_traffic.md", ("op_brick.hip", "brick.hpp", "device.hpp")),
    ("heat3d_128cube_Q4_dG1_c2", "smoother"):
        ("k_asm_fdm_brick_heat3d_128cube_q4_dg1_c2_hbm_traffic.md", ("asm_brick.hip", "brick.hpp", "device.hpp")),
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def code_hash(*paths):
    """sha256 (16 hex digits) of source files with // comments and blank lines removed."""
    import hashlib
    import re
    h = hashlib.sha256()
    for path in paths:
        lines = [re.sub(r"//.*", "", ln).rstrip() for ln in open(path).read().splitlines()]
        h.update("\n".join(ln for ln in lines if ln.strip()).encode())
    return h.hexdigest()[:16]


def kernel_traffic(cfg, key, dtype="f64"):
    """HBM bytes per finest-level apply of kernel `key` ("operator" or "smoother") from its committed
    FETCH_SIZE/WRITE_SIZE summary, or None when no summary covers this workload or the kernel source
    changed since it was measured."""
    ent = TRAFFIC_PROFILES.get((cfg.name, key))
    if ent is None:
        return None
    path = os.path.join(ROOT, "profiles", ent[0])
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            if k.strip() in ("traffic_bytes_per_apply", "source_sha256_16", "dtype"):
                vals[k.strip()] = v.strip()
    cur = code_hash(*[os.path.join(ROOT, "paper_2408_04372_amd", "csrc", f) for f in ent[1]])
    if vals.get("source_sha256_16") != cur or "traffic_bytes_per_apply" not in vals:
        return None
    if vals.get("dtype", "f64") != dtype:
        return None
    return float(vals["traffic_bytes_per_apply"])


def algorithmic_terms(h, cfg, asm_variant, dtype_bytes=8):
    """Algorithmic bytes and flops of one finest-level apply of the operator and of the smoother.

    operator: read x and write y once (2 N_st s) plus per-cell data (rho_K, vertices);
    flops per (cell, temporal DoF): on Cartesian meshes (one coefficient per cell, the brick
    kernel) 8 separable 1D sweeps of n^(d+1) FMA, otherwise 12 sum-factorisation sweeps of
    n^(d+1) FMA and 10 FMA per quadrature point; plus the temporal mixing at the n^d nodes.
    smoother: read r, read and write u (3 N_st s) plus stored cell factors (exact blocks) or
    rho_K (separable blocks)."""
    info = h.info
    n_t = info["n_t"]
    nst = n_t * info["n_x"][0]
    d = cfg.dim
    ncells = int(np.prod(cfg.n_cells[:d]))
    n = cfg.p + 1
    ns = n ** d
    nt_cell = info["nt_cell"]
    c = n_t // nt_cell
    meta = ncells * dtype_bytes + (int(np.prod([v + 1 for v in cfg.n_cells[:d]])) * d * 8 if cfg.perturb else 0)
    op_bytes = 2 * nst * dtype_bytes + meta
    if d == 3 and not cfg.perturb:
        op_flops = ncells * (n_t * 2 * 8 * n ** (d + 1) + 2 * info["temporal_nnz"] * n ** d)
    else:
        op_flops = ncells * (n_t * (2 * 12 * n ** (d + 1) + 2 * 10 * n ** d) + 2 * info["temporal_nnz"] * n ** d)
    if asm_variant == 0:
        asm_bytes = 3 * nst * dtype_bytes + ncells * (ns * ns + ns * nt_cell * nt_cell) * dtype_bytes
        asm_flops = ncells * (4 * ns * ns * n_t + 2 * ns * c * nt_cell * nt_cell)
        asm_peak = FP64_MFMA_PEAK_TFLOPS
    else:
        asm_bytes = 3 * nst * dtype_bytes + ncells * dtype_bytes
        asm_flops = ncells * (n_t * 2 * 2 * d * n ** (d + 1) + ns * c * (nt_cell ** 3 + 2 * nt_cell ** 2))
        asm_peak = FP64_VALU_PEAK_TFLOPS
    return {"operator": (op_bytes, op_flops, FP64_VALU_PEAK_TFLOPS),
            "smoother": (asm_bytes, asm_flops, asm_peak)}


def kernel_roofline(h, cfg, asm_variant, ks):
    """Achieved rates of the finest-level operator and smoother (HIP-event averages over the
    timed solves) against their algorithmic bytes and flops, and the resource that bounds each."""
    terms = algorithmic_terms(h, cfg, asm_variant)
    out = {}
    for key, cnt, tt in (("operator", ks["n_operator"], ks["t_operator"]),
                         ("smoother", ks["n_smoother"], ks["t_smoother"])):
        if not cnt:
            continue
        nb, fl, peak_f = terms[key]
        t = tt / cnt
        t_mem, t_fl = nb / (HBM_PEAK_GBS * 1e9), fl / (peak_f * 1e12)
        alu = "mfma" if (key == "smoother" and asm_variant == 0) else "alu"
        out[key] = {"avg_s": t, "launches": cnt, "bytes": nb, "flops": fl, "GBs": nb / t / 1e9,
                    "TFLOPs": fl / t / 1e12, "frac_hbm": nb / t / 1e9 / HBM_PEAK_GBS,
                    "frac_flops": fl / t / 1e12 / peak_f,
                    "bound": alu if t_fl > t_mem else "hbm",
                    "peak_flops": peak_f, "traffic": kernel_traffic(cfg, key),
                    "speed_of_light_s": max(t_mem, t_fl)}
    return out


# ------------------------------------------------------------------------------ CPU baseline

def _oracle_worker(args):
    """One host core: the oracle's V-cycle on the sample, repeated for budget_s seconds."""
    cfg_idx, cells, budget_s, seed = args
    from threadpoolctl import threadpool_limits
    import stmg_inputs as si
    from oracle import mg, spacetime
    with threadpool_limits(limits=1):
        cfg = si.paper_config(cfg_idx)
        hh = cfg.h[0]
        cfg = cfg.replace(n_cells=(cells,) * 3, hi=(cells * hh,) * 3)
        verts, coef = si.draw_problem(cfg)
        op = spacetime.from_config(cfg, verts, coef)
        H = mg.Hierarchy(op, omegas=[0.5] * 16, asm_variant=LAUNCH[cfg_idx]["asm_variant"])
        r = si.random_slab_vector(cfg, seed).ravel()
        H.vcycle(r)
        n = 0
        t0 = time.time()
        while time.time() - t0 < budget_s:
            H.vcycle(r)
            n += 1
        return cfg.n_st, n, time.time() - t0


def cpu_baseline(cfg_idx: int, cells: int = 4, budget_s: float = 15.0):
    """The oracle's V-cycle on a bounded sample of the same workload (cells^3 cells of the same
    mesh width, degrees, time step and coefficient law), one independent copy per host core
    (at most 16), each single-threaded; value = summed DoFs per V-cycle per second."""
    import multiprocessing as mp
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    cores = max(1, min(ncpu, 16))
    ctx = mp.get_context("fork")          # before any GPU work in this process
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_worker, [(cfg_idx, cells, budget_s, 3 + i) for i in range(cores)])
    rate = sum(nst * n / t for nst, n, t in res)
    nst = res[0][0]
    n_tot = sum(n for _, n, _ in res)
    return {"value": rate, "unit": "space-time DoFs/s per V-cycle", "cores": cores, "kind": "oracle",
            "sample": f"oracle V-cycle (assembled sparse operator, dense cell-block ASM inverses "
                      f"({'separable' if LAUNCH[cfg_idx]['asm_variant'] else 'exact'} blocks as on the GPU), "
                      f"sparse transfers, LU coarse solve) on {cells}^3 cells of the same workload (same h, p, k, "
                      f"c, tau, coefficient law; {nst} DoFs), one single-threaded copy per core on {cores} "
                      f"cores, {n_tot} V-cycles in {budget_s:.0f} s per core, setup excluded"}


def copy_probe(nbytes: int = 1 << 30, reps: int = 10):
    """Plain device-to-device copy of a known size: its FETCH_SIZE / WRITE_SIZE readings per
    dispatch calibrate the counters against nbytes read and nbytes written."""
    import torch
    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    print(json.dumps({"copy_bytes": nbytes, "avg_s": t, "GBs_read_plus_write": 2 * nbytes / t / 1e9}), flush=True)


# ------------------------------------------------------------------------------ GPU parts

def rates(h, dev, nst, n_op=20, n_vc=5):
    """DoFs/s of one operator apply and of one V-cycle, FP64 and FP32 (HIP events on the
    handle's stream)."""
    import torch
    out = {}
    for dt in (torch.float64, torch.float32):
        xv = torch.randn(nst, dtype=dt, device=dev)
        yv = torch.empty_like(xv)
        for _ in range(2):
            h.vmult(xv, yv)
            h.vcycle(xv, yv)
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(h.stream)
        for _ in range(n_op):
            h.vmult(xv, yv)
        e1.record(h.stream)
        for _ in range(n_vc):
            h.vcycle(xv, yv)
        e2.record(h.stream)
        torch.cuda.synchronize()
        key = "fp64" if dt == torch.float64 else "fp32"
        out[f"vmult_dofs_per_s_{key}"] = nst / (e0.elapsed_time(e1) / (n_op * 1e3))
        out[f"vcycle_dofs_per_s_{key}"] = nst / (e1.elapsed_time(e2) / (n_vc * 1e3))
        del xv, yv
    return out


def solve_modes(h, b, x, precisions=(0, 1)):
    """Time to 1e-8 per preconditioner precision (after one warm-up solve each); returns the
    infos and the solutions (host) for the error of each path against the FP64 one."""
    import torch
    res, sols = {}, {}
    for prec in precisions:
        h.set_precision(prec)
        x.zero_()
        h.solve(b, x)
        x.zero_()
        inf = h.solve(b, x)
        res[prec] = inf
        sols[prec] = x.clone()
    h.set_precision(0)
    ref = sols[0]
    nref = torch.linalg.norm(ref).item()
    for prec in precisions:
        res[prec]["rel_diff_vs_fp64"] = torch.linalg.norm(sols[prec] - ref).item() / nref
    del sols
    return res


def smoother_variants(cfg, verts, coef, b, idx):
    """FP64 time to 1e-8 with the cell-wise exact, cell-wise separable and separable vertex-patch
    smoothers (asm_variant 0, 1, 2) on one workload: set-up, iterations, solve time and the
    finest-level smoother time per application."""
    import torch
    from paper_2408_04372_amd import Handle
    out = {}
    for av, key in ((0, "cell_exact"), (1, "cell_separable"), (2, "vertex_patch_separable")):
        kw = dict(LAUNCH[idx])
        kw["asm_variant"] = av
        t0 = time.time()
        h = Handle(cfg, verts, coef, vcycle_dtypes=1, precision=0, rtol=1e-8, max_iter=400, omega=OMEGA, **kw)
        setup = time.time() - t0
        x = torch.zeros_like(b)
        h.solve(b, x)
        x.zero_()
        h.kernel_stats(reset=True)
        inf = h.solve(b, x)
        ks = h.kernel_stats(reset=True)
        out[key] = {"setup_s": setup, "iterations": inf["iterations"], "seconds": inf["seconds"],
                    "rel_residual": inf["rel_residual"],
                    "smoother_ms_per_application": 1e3 * ks["t_smoother"] / max(1, ks["n_smoother"])}
        h.close()
        del x
        torch.cuda.empty_cache()
    return out


def extra_config(idx, dev, learned_on, train_solves):
    """Time to 1e-8 (FP64 and FP32 V-cycle, learned stage on the 64^3 Q2 workload) and the
    operator / V-cycle rates of another single-GPU workload."""
    import torch
    import stmg_inputs as si
    from paper_2408_04372_amd import Handle
    cfg = si.paper_config(idx)
    verts, coef = si.draw_problem(cfg)
    t0 = time.time()
    h = Handle(cfg, verts, coef, vcycle_dtypes=3, precision=0, rtol=1e-8, max_iter=400, omega=OMEGA,
               **LAUNCH[idx])
    setup = time.time() - t0
    b = torch.from_numpy(si.random_slab_vector(cfg, 1001)).to(dev).reshape(-1).contiguous()
    x = torch.zeros_like(b)
    nst = h.size(0)
    modes = solve_modes(h, b, x)
    out = {"workload": cfg.name, "n_st": nst, "setup_s": setup, "levels": h.info["n_levels"],
           "device_GB": h.info["device_bytes"] / 1e9, "eig_resolves": h.info["eig_resolves"],
           "fp64": {k: modes[0][k] for k in ("iterations", "seconds", "rel_residual")},
           "fp32_vcycle": {k: modes[1][k] for k in ("iterations", "seconds", "rel_residual", "rel_diff_vs_fp64")}}
    out.update(rates(h, dev, nst))
    if idx == 5:
        h.close()
        torch.cuda.empty_cache()
        out["smoother_variants"] = smoother_variants(cfg, verts, coef, b, idx)
        log(f"smoother variants ({cfg.name}): {json.dumps(out['smoother_variants'])}")
        h = None
    if learned_on and idx == 5:
        # the learned stage: trained on seeded plain-multigrid solves (seeds 1001, 1002, ...) on a
        # 16^3-cell box of the same mesh width, degrees, time step and coefficient law, then
        # evaluated on the full workload on held-out right-hand sides (seeds 3001-3003) against the
        # plain FP64 and FP32-V-cycle solves
        from paper_2408_04372_amd import learned
        tl = time.time()
        theta, ch, losses = learned.train_for_config(idx, solves=train_solves, epochs=2, lr=2e-3, cells=16,
                                                     log=log)
        t_train = time.time() - tl
        if h is not None:
            h.close()
        torch.cuda.empty_cache()
        res = learned.gain(cfg, verts, coef, theta, ch, seeds=[3001, 3002, 3003], omega=OMEGA, rtol=1e-8,
                           max_iter=400, **LAUNCH[idx])
        out["learned"] = {"eval_seeds": [3001, 3002, 3003], "train_s": t_train, "train_solves": train_solves,
                          "train_seeds": [1001, 1000 + train_solves], "train_box_cells": 16,
                          "train_pairs": 4 * train_solves, "train_epochs": 2,
                          "train_loss_first_last": [losses[0], losses[-1]], "channels": ch}
        out["learned"].update(res)
        del b, x
        torch.cuda.empty_cache()
        return out
    if idx == 2:
        # temporal levels below the spatial ones (k to its minimum, then tau doubled)
        h.close()
        t1 = time.time()
        htm = Handle(cfg, verts, coef, vcycle_dtypes=1, precision=0, rtol=1e-8, max_iter=400, omega=OMEGA,
                     time_mg=1, **LAUNCH[idx])
        tm_setup = time.time() - t1
        x.zero_()
        htm.solve(b, x)
        x.zero_()
        inftm = htm.solve(b, x)
        out["time_mg"] = {"levels": htm.info["n_levels"], "n_t_level": htm.info["n_t_level"],
                          "coarse_unknowns": htm.info["coarse_unknowns"], "setup_s": tm_setup,
                          "iterations": inftm["iterations"], "seconds": inftm["seconds"],
                          "rel_residual": inftm["rel_residual"]}
        htm.close()
    elif h is not None:
        h.close()
    del b, x
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--extra-configs", default="2,3,5")
    ap.add_argument("--train-solves", type=int, default=2000)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run 10 device copies of 1 GiB (calibration of hardware byte counters)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the slab solver is a single-GPU build); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    cpu = None
    if not args.no_cpu_baseline:
        # the oracle runs first, in forked workers, before this process touches the GPU
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(args.config)
        log(f"cpu baseline: {cpu['value']:.3e} DoFs/s per V-cycle on {cpu['cores']} cores")

    import torch
    import stmg_inputs as si
    from paper_2408_04372_amd import Handle

    cfg = si.paper_config(args.config)
    launch = LAUNCH[args.config]
    verts, coef = si.draw_problem(cfg)
    log(f"workload {cfg.name}: N_st={cfg.n_st} n_t={cfg.n_t}")
    dev = torch.device("cuda:0")
    t0 = time.time()
    # relaxation per level: 1.5 / lambda_max of ASM * S_l (Arnoldi estimate)
    h = Handle(cfg, verts, coef, vcycle_dtypes=3, precision=0, rtol=1e-8, max_iter=400, omega=OMEGA, **launch)
    setup_s = time.time() - t0
    log(f"setup {setup_s:.1f} s, levels {h.info['n_levels']}, omega {np.round(h.info['omega'], 4).tolist()}, "
        f"device bytes {h.info['device_bytes'] / 1e9:.1f} GB, eigen-solve repeats {h.info['eig_resolves']}")
    b = torch.from_numpy(si.random_slab_vector(cfg, 1001)).to(dev).reshape(-1).contiguous()
    x = torch.zeros_like(b)
    nst = h.size(0)

    for i in range(args.warmup):
        x.zero_()
        inf = h.solve(b, x)
        log(f"warmup {i}: {inf['iterations']} it, res {inf['rel_residual']:.2e}, {inf['seconds']:.3f} s")
    h.kernel_stats(reset=True)
    torch.cuda.synchronize()
    iters = 0
    infos = []
    t_start = time.perf_counter()
    for i in range(args.steps):
        x.zero_()
        inf = h.solve(b, x)
        iters += inf["iterations"]
        infos.append(inf)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ks = h.kernel_stats(reset=True)
    for i, inf in enumerate(infos):
        log(f"step {i}: {inf['iterations']} it, res {inf['rel_residual']:.2e}, {inf['seconds']:.3f} s, "
            f"smoother {inf['t_smoother']:.3f} gmg {inf['t_gmg_other']:.3f} op {inf['t_operator']:.3f} "
            f"other {inf['t_other']:.3f}")
    value = nst * iters / elapsed
    kr = kernel_roofline(h, cfg, launch["asm_variant"], ks)
    dominant = max(kr, key=lambda k: kr[k]["avg_s"] * kr[k]["launches"])
    d = kr[dominant]
    if d["bound"] == "hbm":
        ach, peak, unit, frac = d["GBs"], HBM_PEAK_GBS, "GB/s", d["frac_hbm"]
    else:
        ach, peak, unit, frac = d["TFLOPs"], d["peak_flops"], "TFLOP/s", d["frac_flops"]
    brick = cfg.dim == 3 and not cfg.perturb
    names = {"operator": ("operator (st_apply3_brick, 8 brick colours, finest level, FP64)" if brick else
                          "operator (st_apply3 over all cells + gather, finest level, FP64)"),
             "smoother": ("smoother (k_asm_fdm_brick, 8 brick colours, finest level, FP64)"
                          if (launch["asm_variant"] and brick) else
                          "smoother (k_asm_mfma over all cells + gather, finest level, FP64)")}
    roofline = {"kernel": names[dominant], "bound": d["bound"], "achieved": ach, "peak": peak, "unit": unit,
                "frac": frac, "traffic": d["traffic"],
                "avg_launch_s": d["avg_s"], "bytes_per_launch": d["bytes"], "flops_per_launch": d["flops"],
                "frac_hbm": d["frac_hbm"], "frac_flops": d["frac_flops"]}
    extras = {"kernels": kr, "kernel_counts": ks,
              "buckets_s": {k: float(np.mean([i[k] for i in infos]))
                            for k in ("t_smoother", "t_gmg_other", "t_operator", "t_other")},
              "device_GB": h.info["device_bytes"] / 1e9, "eig_resolves": h.info["eig_resolves"],
              "omega": list(h.info["omega"][:h.info["n_levels"]])}
    if not args.no_extras:
        modes = solve_modes(h, b, x)
        extras["time_to_solution_s"] = {"fp64": elapsed / args.steps, "fp32_vcycle": modes[1]["seconds"]}
        extras["iterations"] = {"fp64": iters / args.steps, "fp32_vcycle": modes[1]["iterations"]}
        extras["fp32_vcycle_rel_diff_vs_fp64"] = modes[1]["rel_diff_vs_fp64"]
        extras["fp32_vcycle_rel_residual"] = modes[1]["rel_residual"]
        extras.update(rates(h, dev, nst))
        log(f"extras ({cfg.name}): {json.dumps({k: v for k, v in extras.items() if k not in ('kernels',)})}")
    h.close()
    del b, x
    torch.cuda.empty_cache()
    if not args.no_extras:
        others = {}
        for idx in [int(v) for v in args.extra_configs.split(",") if v.strip()]:
            if idx == args.config or idx not in LAUNCH:
                continue
            log(f"extra workload {idx} ...")
            others[si.paper_config(idx).name] = extra_config(idx, dev, not args.no_learned, args.train_solves)
            log(f"extra workload {idx}: {json.dumps(others[si.paper_config(idx).name])}")
        extras["other_workloads"] = others
    out = {
        "metric": "space-time DoFs/s per V-cycle + time-to-1e-8 residual (plain FP64 vs FP32/learned)",
        "value": value,
        "unit": "space-time DoFs/s per V-cycle",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg.name, "n_cells": list(cfg.n_cells), "p": cfg.p, "k": cfg.k,
                   "time_method": "dG" if cfg.time_method == 0 else "cGP", "n_time_cells": cfg.n_time_cells,
                   "n_st": nst, "perturbation": cfg.perturb, "coefficient": f"{cfg.coef} sigma={cfg.coef_sigma}",
                   "rtol": 1e-8, "restart": launch["restart"], "n_smooth": 1,
                   "smoother": "separable cell blocks" if launch["asm_variant"] else "exact cell blocks",
                   "vcycle": "fp64", "omega_rule": "1.5/lambda_max per level", "setup_s": setup_s},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
