"""What the trained network gains over plain space-time multigrid.

A network is trained on the GPU (library kernels, Adam) on (residual, error) pairs from
plain STMG iterations of the heat problem with Q2 cells, dG(1), 4 time cells, tau = h/2
and a lognormal (sigma = 1) cell coefficient on an 8^3-cell box; it is then used inside
FGMRES on held-out right-hand sides on a 16^3-cell box of the same mesh width.  The test
reports iterations and time of the FP32-V-cycle method with and without the learned
stage and checks that
  - training lowers the loss,
  - every learned solve reaches the 1e-8 true relative residual,
  - the learned stage never costs more than one extra FGMRES iteration (rejected stages
    reduce to the plain V-cycle, so only accepted ones change the iteration);
and prints the measured accepted-stage fraction, the iteration difference and the time ratio.
"""
import json

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import stmg_inputs as si

pytestmark = pytest.mark.gpu


def test_trained_network_gain():
    from paper_2408_04372_amd import learned
    theta, ch, losses = learned.train_for_config(5, solves=150, epochs=3, lr=2e-3, cells=8, log=print)
    print("losses", losses)
    assert losses[-1] < losses[0]
    cfg = learned.training_config(5, 16)
    verts, coef = si.draw_problem(cfg.replace(seed=cfg.seed + 100))
    res = learned.gain(cfg, verts, coef, theta, ch, seeds=[3001, 3002, 3003], omega=-1.0, rtol=1e-8,
                       max_iter=300)
    print("gain", json.dumps(res))
    for key in ("fp64", "fp32_vcycle", "learned"):
        assert res[key]["rel_residual_max"] <= 1e-8
    lr, pl = res["learned"], res["fp32_vcycle"]
    stages = lr["cnn_used"] + lr["cnn_fallbacks"]
    assert stages == 3 * lr["iterations_mean"]
    accepted = lr["cnn_used"] / stages
    delta = lr["iterations_mean"] - pl["iterations_mean"]
    print(f"learned stage: {accepted:.1%} of {stages} stages accepted, iterations {lr['iterations_mean']:.2f} "
          f"vs {pl['iterations_mean']:.2f} (delta {delta:+.2f}), time ratio vs FP32 V-cycle "
          f"{1.0 / res['speedup_time_vs_fp32']:.3f}")
    assert 0.0 <= accepted <= 1.0
    assert delta <= 1.0
