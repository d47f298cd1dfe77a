"""Oracle study of the vertex-patch smoother (not collected by pytest): FGMRES(30) iterations to
1e-8 with the V-cycle of the oracle hierarchy for four smoothers (cell blocks exact / separable,
vertex patches exact / separable) on heat dG(1), c = 2, omega_l = 1.5 / lambda_max, for p = 1..4
(2D, 8^2 cells) and p = 1..3 (3D, 4^3 cells).

    python tests/patch_study.py one          # constant coefficient
    python tests/patch_study.py lognormal    # lognormal, sigma = 0.5
"""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import stmg_inputs as si
from oracle import krylov, mg, spacetime


def main(coef: str):
    for dim, cells in ((2, (8, 8, 1)), (3, (4, 4, 4))):
        for p in (1, 2, 3, 4):
            if dim == 3 and p == 4:
                continue
            cfg = si.Config(dim=dim, problem=0, time_method=0, p=p, k=1, n_time_cells=2, n_cells=cells,
                            tau=0.5 / cells[0], coef=coef, coef_sigma=0.5, seed=7)
            verts, cf = si.draw_problem(cfg)
            op = spacetime.from_config(cfg, verts, cf)
            b = si.random_slab_vector(cfg, 3).ravel()
            its = []
            for variant in (0, 1, 3, 2):
                H = mg.Hierarchy(op, asm_variant=variant, omega_rule=-1.5)
                _, it, _ = krylov.fgmres(op.apply, b, H.vcycle, rtol=1e-8, restart=30, max_iter=200)
                its.append(it)
            print(f"{dim}D p={p} DoFs={op.n_t * op.n_x}: cell exact {its[0]}, cell separable {its[1]}, "
                  f"patch exact {its[2]}, patch separable {its[3]}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "lognormal")
