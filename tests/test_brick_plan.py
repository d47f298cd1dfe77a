"""Host logic of the brick tiling (csrc/brick.hpp): the brick planner's choices for the workloads it
was tuned on, its limits over a sweep of levels, and the colour launches' coverage of the bricks.
The header is compiled for the host with hipcc (no GPU call is made).  CPU only."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2408_04372_amd", "csrc")
HIPCC = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")

DRIVER = r"""
#include <cstdio>
#include <vector>
#include "brick.hpp"
using namespace stmg;

static GeomDesc level(int p, int n0, int n1, int n2) {
  GeomDesc g;
  g.dim = 3; g.p = p; g.n = p + 1;
  g.nc[0] = n0; g.nc[1] = n1; g.nc[2] = n2;
  for (int d = 0; d < 3; ++d) g.nn[d] = g.nc[d] * p + 1;
  return g;
}

int main() {
  // documented choices: operator FP64 Q4 / FP32 Q4 / FP64 Q2, smoother FP64 Q4 (n_t = 4, 128^3)
  struct Case { const char* name; int p, nt, ipc, lanes, elem, scr; long extra; int vgprs; bool inbox, lng; };
  const Case cases[] = {
      {"op64_q4", 4, 4, 4, 5, 8, 50, 300, 217, true, true},
      {"op32_q4", 4, 4, 4, 5, 4, 50, 150, 117, true, false},
      {"op64_q2", 2, 4, 4, 3, 8, 18, 300, 94, true, true},
      {"fdm64_q4", 4, 4, 2, 10, 8, 50, 8 * (12 * 30 + 1), 183, false, false},
  };
  for (const Case& c : cases) {
    BrickPlan pl;
    const bool ok = plan_brick(level(c.p, 128, 128, 128), c.nt, c.ipc, c.lanes, c.elem, c.scr, c.extra, c.vgprs, pl,
                               c.inbox, c.lng);
    std::printf("case %s %d %d %d %d %d %zu\n", c.name, ok, pl.B[0], pl.B[1], pl.B[2], pl.waves, pl.lds);
  }
  // limits over a sweep
  long checked = 0, bad = 0;
  for (int p = 1; p <= 4; ++p)
    for (int nt : {1, 2, 3, 4, 8, 24})
      for (int nc : {1, 2, 3, 5, 16, 64})
        for (int elem : {4, 8})
          for (int vg : {64, 128, 217, 256})
            for (int inbox = 0; inbox < 2; ++inbox) {
              const int lanes = p + 1;
              BrickPlan pl;
              GeomDesc g = level(p, nc, nc + 1, nc);
              if (!plan_brick(g, nt, nt, lanes, elem, 2 * lanes * lanes, 300, vg, pl, inbox != 0, inbox != 0)) continue;
              ++checked;
              const int tpw = 64 / lanes;
              const long items = (long)pl.B[0] * pl.B[1] * pl.B[2] * nt;
              if (pl.waves > 8 || pl.lds > 72 * 1024 || items > (long)pl.waves * tpw) ++bad;
              for (int d = 0; d < 3; ++d)
                if (pl.B[d] < 1 || pl.B[d] > g.nc[d]) ++bad;
              // every brick is launched by exactly one colour
              BrickLaunch L[8];
              brick_launches(g, pl, L);
              std::vector<int> hit((size_t)L[0].nbt[0] * L[0].nbt[1] * L[0].nbt[2], 0);
              for (int col = 0; col < 8; ++col)
                for (int lb = 0; lb < L[col].nblocks; ++lb) {
                  const int ib[3] = {lb % L[col].nbc[0], (lb / L[col].nbc[0]) % L[col].nbc[1],
                                     lb / (L[col].nbc[0] * L[col].nbc[1])};
                  int b[3];
                  for (int d = 0; d < 3; ++d) b[d] = 2 * ib[d] + ((col >> d) & 1);
                  ++hit[((size_t)b[2] * L[0].nbt[1] + b[1]) * L[0].nbt[0] + b[0]];
                }
              for (int h : hit)
                if (h != 1) ++bad;
            }
  std::printf("sweep %ld %ld\n", checked, bad);
  return 0;
}
"""


def test_brick_planner_choices_and_limits():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "plan.cpp")
        open(src, "w").write(DRIVER)
        exe = os.path.join(d, "plan")
        r = subprocess.run([HIPCC, "-std=c++17", "-x", "hip", "--offload-arch=gfx950", "-O1", "-I", CSRC,
                            "-I", os.path.join(ROOT, "include"), src, "-o", exe], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        assert out.returncode == 0, out.stderr[-2000:]
    lines = out.stdout.split("\n")
    got = {ln.split()[1]: [int(v) for v in ln.split()[2:]] for ln in lines if ln.startswith("case")}
    # (ok, B_x, B_y, B_z, waves, LDS bytes)
    assert got["op64_q4"][:5] == [1, 6, 2, 1, 4] and got["op64_q4"][5] < 40 * 1024   # exchange slices in the box
    assert got["op32_q4"][:5] == [1, 6, 2, 1, 4]                                    # no long bricks in FP32
    assert got["op64_q2"][:4] == [1, 6, 3, 2]                                       # a long brick for Q2
    assert got["fdm64_q4"][:5] == [1, 6, 2, 1, 4]
    checked, bad = [int(v) for v in next(ln for ln in lines if ln.startswith("sweep")).split()[1:]]
    assert checked > 500 and bad == 0
