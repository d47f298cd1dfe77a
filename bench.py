"""Benchmark: space-time DoFs/s per V-cycle and time to a 1e-8 relative residual.

One step = one stmg_solve of the all-at-once slab system from x0 = 0 to a true
relative residual of 1e-8 with FP64 FGMRES and one space-time multigrid V-cycle
per iteration (operator, cell-wise additive Schwarz smoother, h/p transfers,
coarse solve, Krylov updates: the whole hot path).  Workload: heat equation on
the unit cube, 32^3 Q4 cells with vertices displaced by up to 10% of h, dG(2),
8 time cells per slab (51.5 M space-time DoFs including Dirichlet nodes),
plain FP64 V-cycle; inputs are seeded and synthetic.

value = N_st * (V-cycles in the timed steps) / (timed seconds).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
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


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


FP64_VALU_PEAK_TFLOPS = 78.6     # 256 CUs x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
FP64_MFMA_PEAK_TFLOPS = 78.6
# committed FETCH_SIZE / WRITE_SIZE summaries of the finest-level kernels at the default workload
TRAFFIC_PROFILES = {
    "operator": (os.path.join(ROOT, "profiles", "st_apply3_heat3d_q4_dg2_c8_hbm_traffic.md"),
                 ("op_apply.hip", "blas.hip", "device.hpp")),
    "smoother": (os.path.join(ROOT, "profiles", "k_asm_mfma_heat3d_q4_dg2_c8_hbm_traffic.md"),
                 ("asm.hip", "blas.hip", "device.hpp")),
}


def code_hash(*paths):
    """sha256 (16 hex digits) of source files with // comments and blank lines removed."""
    import hashlib
    import re
    h = hashlib.sha256()
    for path in paths:
        lines = [re.sub(r"//.*", "", ln).rstrip() for ln in open(path).read().splitlines()]
        h.update("\n".join(ln for ln in lines if ln.strip()).encode())
    return h.hexdigest()[:16]


def kernel_traffic(cfg, key):
    """HBM bytes per finest-level apply of kernel `key` ("operator" or "smoother") from its committed
    FETCH_SIZE/WRITE_SIZE summary, or None when the workload differs or the kernel source changed
    since it was measured."""
    path, src = TRAFFIC_PROFILES[key]
    if cfg.name != "heat3d_32cube_Q4_perturbed_dG2_c8" or not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.split(":")[0].strip() in ("traffic_bytes_per_apply", "source_sha256_16"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    cur = code_hash(*[os.path.join(ROOT, "paper_2408_04372_amd", "csrc", f) for f in src])
    if vals.get("source_sha256_16") != cur or "traffic_bytes_per_apply" not in vals:
        return None
    return float(vals["traffic_bytes_per_apply"])


def kernel_roofline(h, cfg, ks, dtype_bytes=8):
    """Algorithmic bytes and flops per launch (one apply = all colour dispatches) of the
    finest-level operator and smoother kernels, and the resource that bounds each."""
    info = h.info
    n_t = info["n_t"]
    nx = info["n_x"][0]
    nst = n_t * nx
    d = cfg.dim
    ncells = int(np.prod(cfg.n_cells[:d]))
    n = cfg.p + 1
    ns = n ** d
    nt_cell = info["nt_cell"]
    c = n_t // nt_cell
    meta = ncells * 8 + (int(np.prod([v + 1 for v in cfg.n_cells[:d]])) * d * 8 if cfg.perturb else 0)
    out = {}
    # operator: read x, read and write y, cell data; flops per (cell, temporal DoF): 12 sum-factorisation
    # sweeps of n^(d+1) FMA, 10 FMA per quadrature point, temporal mixing at the n^d nodes
    op_bytes = 3 * nst * dtype_bytes + meta
    op_flops = ncells * (n_t * (2 * 12 * n ** (d + 1) + 2 * 10 * n ** d) + 2 * info["temporal_nnz"] * n ** d)
    # smoother: read r, read and write u, read Q_K and the temporal inverses; two GEMMs with Q_K
    asm_bytes = 3 * nst * dtype_bytes + ncells * (ns * ns + ns * nt_cell * nt_cell) * dtype_bytes
    asm_flops = ncells * (4 * ns * ns * n_t + 2 * ns * c * nt_cell * nt_cell)
    for key, nb, fl, peak_f, cnt, tt in (
            ("operator", op_bytes, op_flops, FP64_VALU_PEAK_TFLOPS, ks["n_operator"], ks["t_operator"]),
            ("smoother", asm_bytes, asm_flops, FP64_MFMA_PEAK_TFLOPS, ks["n_smoother"], ks["t_smoother"])):
        if not cnt:
            continue
        t = tt / cnt
        t_mem, t_fl = nb / (HBM_PEAK_GBS * 1e9), fl / (peak_f * 1e12)
        out[key] = {"avg_s": t, "launches": cnt, "bytes": nb, "flops": fl, "GBs": nb / t / 1e9,
                    "TFLOPs": fl / t / 1e12, "frac_hbm": nb / t / 1e9 / HBM_PEAK_GBS,
                    "frac_flops": fl / t / 1e12 / peak_f,
                    "bound": ("alu" if key == "operator" else "mfma") if t_fl > t_mem else "hbm",
                    "peak_flops": peak_f, "traffic": kernel_traffic(cfg, key),
                    "speed_of_light_s": max(t_mem, t_fl)}
    return out


def cpu_baseline(budget_s: float = 15.0):
    """The oracle's V-cycle on a bounded sample of the same workload (2^3 cells, same p, k, c)."""
    import stmg_inputs as si
    from oracle import mg, spacetime
    cfg = si.paper_config(2).replace(n_cells=(2, 2, 2))
    verts, coef = si.draw_problem(cfg)
    t0 = time.time()
    op = spacetime.from_config(cfg, verts, coef)
    H = mg.Hierarchy(op, omegas=[1.0] * 8)
    for lev in H.levels[1:]:
        lev.omega = 0.5
    setup = time.time() - t0
    r = si.random_slab_vector(cfg, 3).ravel()
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):          # the oracle runs single-threaded: report 1 core
        H.vcycle(r)
        n = 0
        t0 = time.time()
        while time.time() - t0 < budget_s:
            H.vcycle(r)
            n += 1
        dt = (time.time() - t0) / n
    threads = 1
    return {"value": cfg.n_st / dt, "unit": "space-time DoFs/s per V-cycle", "cores": threads,
            "kind": "oracle",
            "sample": f"oracle V-cycle (assembled sparse operator, dense principal-block ASM inverses, "
                      f"sparse transfers, LU coarse solve) on 2^3 cells of the same Q4/dG(2)/c=8 "
                      f"perturbed heat problem ({cfg.n_st} DoFs), {n} V-cycles in {n * dt:.1f} s, "
                      f"setup {setup:.1f} s excluded"}


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
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

    import torch
    import stmg_inputs as si
    from paper_2408_04372_amd import Handle

    cfg = si.paper_config(args.config)
    verts, coef = si.draw_problem(cfg)
    log(f"workload {cfg.name}: N_st={cfg.n_st} n_t={cfg.n_t}")
    dev = torch.device("cuda:0")
    t0 = time.time()
    # relaxation per level: 1.5 / lambda_max of ASM * S_l (Arnoldi estimate); the literal
    # eq.-relaxation value (about 2 / lambda_max) stalls FGMRES at Q4 (top of the spectrum
    # left undamped)
    h = Handle(cfg, verts, coef, vcycle_dtypes=3, precision=0, rtol=1e-8, restart=30, max_iter=300,
               omega=-1.5)
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
    kr = kernel_roofline(h, cfg, ks)
    dominant = max(kr, key=lambda k: kr[k]["avg_s"] * kr[k]["launches"])
    d = kr[dominant]
    if d["bound"] == "hbm":
        ach, peak, unit, frac = d["GBs"], HBM_PEAK_GBS, "GB/s", d["frac_hbm"]
    else:
        ach, peak, unit, frac = d["TFLOPs"], d["peak_flops"], "TFLOP/s", d["frac_flops"]
    roofline = {"kernel": "smoother (k_asm_mfma over all cells + gather, finest level)" if dominant == "smoother"
                else "operator (st_apply3 over all cells + gather, finest level)",
                "bound": d["bound"], "achieved": ach, "peak": peak, "unit": unit, "frac": frac,
                "traffic": kernel_traffic(cfg, dominant),
                "avg_launch_s": d["avg_s"], "bytes_per_launch": d["bytes"], "flops_per_launch": d["flops"],
                "frac_hbm": d["frac_hbm"], "frac_flops": d["frac_flops"]}
    extras = {"kernels": kr, "kernel_counts": ks}
    if not args.no_extras:
        # time to 1e-8 with the FP32 V-cycle inside FP64 FGMRES
        h.set_precision(1)
        x.zero_()
        h.solve(b, x)
        x.zero_()
        inf32 = h.solve(b, x)
        h.set_precision(0)
        extras["time_to_solution_s"] = {"fp64": elapsed / args.steps, "fp32_vcycle": inf32["seconds"]}
        extras["iterations"] = {"fp64": iters / args.steps, "fp32_vcycle": inf32["iterations"]}
        # temporal levels below the spatial ones (k to its minimum, then tau doubled)
        t1 = time.time()
        htm = Handle(cfg, verts, coef, vcycle_dtypes=1, precision=0, rtol=1e-8, restart=30, max_iter=300,
                     omega=-1.5, time_mg=1)
        tm_setup = time.time() - t1
        x.zero_()
        htm.solve(b, x)
        x.zero_()
        inftm = htm.solve(b, x)
        extras["time_mg"] = {"levels": htm.info["n_levels"], "n_t_level": htm.info["n_t_level"],
                             "coarse_unknowns": htm.info["coarse_unknowns"], "setup_s": tm_setup,
                             "iterations": inftm["iterations"], "seconds": inftm["seconds"],
                             "rel_residual": inftm["rel_residual"],
                             "spatial_only": {"levels": h.info["n_levels"],
                                              "coarse_unknowns": h.info["coarse_unknowns"]}}
        htm.close()
        if not args.no_learned:
            # learned stage: a network trained on the GPU on plain-STMG pairs of an 8^3-cell box
            # with the same mesh width, degrees and time step, then used on the full problem
            from paper_2408_04372_amd import learned
            tl = time.time()
            theta, ch, losses = learned.train_for_config(args.config, solves=60, epochs=3, lr=2e-3, cells=8,
                                                         log=log)
            t_train = time.time() - tl
            h.cnn_create(ch)
            h.cnn_set_params(theta)
            h.set_precision(2)
            x.zero_()
            h.solve(b, x)
            x.zero_()
            infl = h.solve(b, x)
            h.set_precision(0)
            extras["time_to_solution_s"]["learned"] = infl["seconds"]
            extras["iterations"]["learned"] = infl["iterations"]
            extras["learned"] = {"cnn_used": infl["cnn_used"], "cnn_fallbacks": infl["cnn_fallbacks"],
                                 "rel_residual": infl["rel_residual"], "train_s": t_train,
                                 "train_loss_first_last": [losses[0], losses[-1]], "channels": ch,
                                 "train_solves": 60}
        # operator and V-cycle alone, event-timed
        for dt in (torch.float64, torch.float32):
            xv = torch.randn(nst, dtype=dt, device=dev)
            yv = torch.empty_like(xv)
            for _ in range(3):
                h.vmult(xv, yv)
                h.vcycle(xv, yv)
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            e0.record(h.stream)
            for _ in range(20):
                h.vmult(xv, yv)
            e1.record(h.stream)
            for _ in range(5):
                h.vcycle(xv, yv)
            e2.record(h.stream)
            torch.cuda.synchronize()
            key = "fp64" if dt == torch.float64 else "fp32"
            extras[f"vmult_dofs_per_s_{key}"] = nst / (e0.elapsed_time(e1) / 20e3)
            extras[f"vcycle_dofs_per_s_{key}"] = nst / (e1.elapsed_time(e2) / 5e3)
        log(f"extras: {json.dumps({k: v for k, v in extras.items() if k not in ('kernels',)})}")
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline()
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
                   "time_method": "dG", "n_time_cells": cfg.n_time_cells, "n_st": nst,
                   "perturbation": cfg.perturb, "rtol": 1e-8, "restart": 30, "n_smooth": 1,
                   "omega_rule": "1.5/lambda_max per level",
                   "setup_s": setup_s},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extras": extras,
    }
    extras["eig_resolves"] = h.info["eig_resolves"]
    print(json.dumps(out), flush=True)
    h.close()


if __name__ == "__main__":
    main()
