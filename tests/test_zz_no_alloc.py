"""stmg_vmult_noalloc: the operator through the library's static per-device scratch (no device
memory allocated by the call), against stmg_vmult on the same handle and the oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import stmg_inputs as si
from tests.gpu_common import oracle_op, problem, rel_err

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _np(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


@pytest.mark.parametrize("path", [0, 1])
@pytest.mark.parametrize("name", ["heat3d_q4_dg1_brick", "heat2d_q2_dg1", "heat3d_q2_dg1_pert",
                                  "wave3d_q3_cgp2_brick"])
def test_vmult_noalloc_matches_vmult(name, path):
    """Two calls in a row, the second on a smaller input (the next coarser level); on the per-cell
    path (1) stmg_vmult runs the same kernels and must agree bitwise, on the default path to a few
    ulps; level 0 also against the oracle."""
    from paper_2408_04372_amd import Handle
    cfg, verts, coef = problem(name)
    print(f"case {name} path {path}", flush=True)
    op = oracle_op(cfg, verts, coef)
    rng = np.random.default_rng(61)
    with Handle(cfg, verts, coef, omega=0.5, vcycle_dtypes=3, kernel_path=path) as h:
        L = h.info["n_levels"]
        assert L >= 2
        for level in (0, 1):
            n = h.size(level)
            xh = rng.standard_normal(n)
            for dt, tol in ((torch.float64, 1e-12), (torch.float32, 2e-5)):
                x = torch.from_numpy(xh).to(DEV, dtype=dt)
                y_ref = torch.empty_like(x)
                h.vmult(x, y_ref, level=level)
                y = torch.full_like(x, float("nan"))
                h.vmult_noalloc(x, y, level=level)
                if path == 1:
                    assert torch.equal(y, y_ref), (level, dt)
                assert rel_err(_np(y), _np(y_ref)) < tol, (level, dt)
                if level == 0:
                    ref = op.apply(xh.reshape(cfg.n_t, cfg.n_x))
                    assert rel_err(_np(y), ref) < tol, dt


def test_vmult_noalloc_rejects_levels_beyond_the_scratch():
    """32^3 Q4 cells, 4 temporal DoFs: the FP64 per-cell slots need 131 MB (> 64 MiB) and are
    rejected; the FP32 slots (65.5 MB) fit and agree with stmg_vmult."""
    from paper_2408_04372_amd import Handle, StmgError
    cfg = si.Config(dim=3, problem=0, time_method=0, p=4, k=1, n_time_cells=2, n_cells=(32, 32, 32),
                    tau=1 / 64, coef="lognormal", coef_sigma=0.5, seed=62)
    verts, coef = si.draw_problem(cfg)
    with Handle(cfg, verts, coef, omega=0.5, vcycle_dtypes=3, asm_variant=1) as h:
        n = h.size(0)
        x = torch.randn(n, dtype=torch.float64, device=DEV)
        y = torch.empty_like(x)
        with pytest.raises(StmgError) as e:
            h.vmult_noalloc(x, y)
        assert "scratch" in str(e.value)
        x32 = x.float()
        y32 = torch.empty_like(x32)
        ref32 = torch.empty_like(x32)
        h.vmult_noalloc(x32, y32)
        h.vmult(x32, ref32)
        assert rel_err(_np(y32), _np(ref32)) < 2e-5
