"""The library's host-side set-up numerics (csrc/hostmath.cpp: quadrature, Lagrange bases, the
dG/cGP temporal matrices of Sections 2.1-2.2, temporal prolongations, small dense inverses and
generalised eigen-solves) built with g++ under AddressSanitizer and UndefinedBehaviorSanitizer and
run over the ranges the library uses.  The driver also checks a few identities, so a silent
out-of-bounds read that changes a value fails as well.  CPU only."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2408_04372_amd", "csrc")

DRIVER = r"""
#include <cmath>
#include <cstdio>
#include <stdexcept>
#include "hostmath.hpp"
using namespace stmg::hm;

static int bad = 0;
static void check(bool ok, const char* what, int a, int b) {
  if (!ok) { std::printf("FAIL %s %d %d\n", what, a, b); ++bad; }
}
static bool finite(const Mat& m) {
  for (double v : m.a) if (!std::isfinite(v)) return false;
  return true;
}

int main() {
  Vec x, w;
  for (int n = 1; n <= 8; ++n) {
    gauss(n, x, w);
    double s = 0;
    for (int i = 0; i < n; ++i) { s += w[i]; check(x[i] > 0 && x[i] < 1, "gauss node", n, i); }
    check(std::fabs(s - 1) < 1e-13, "gauss weights", n, 0);
    Vec r = gauss_radau_right(n);
    check((int)r.size() == n && std::fabs(r[n - 1] - 1) < 1e-14, "radau", n, 0);
    if (n >= 2) {
      Vec l = gauss_lobatto(n);
      check((int)l.size() == n && std::fabs(l[0]) < 1e-14 && std::fabs(l[n - 1] - 1) < 1e-14, "lobatto", n, 0);
      Mat val, der;
      lagrange(l, l, val, der);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) check(std::fabs(val(i, j) - (i == j)) < 1e-12, "lagrange", i, j);
      for (int i = 0; i < n; ++i) {
        double d = 0;
        for (int j = 0; j < n; ++j) d += der(i, j);
        check(std::fabs(d) < 1e-9, "lagrange derivative of 1", n, i);
      }
    }
  }
  for (int problem = 0; problem < 2; ++problem)
    for (int method = 0; method < 2; ++method)
      for (int k = method; k <= 4; ++k)
        for (int c : {1, 2, 3, 4, 8}) {
          Temporal t = temporal(problem, method, k, c, 0.05);
          const int per = method == 0 ? k + 1 : k;
          check(t.n_t == c * per && t.nt_cell == per, "n_t", k, c);
          check(t.M_T.r == t.n_t && t.N_T.r == t.n_t && finite(t.M_T) && finite(t.N_T) && finite(t.A_T),
                "slab matrices", k, c);
          check(finite(t.M_tau) && finite(t.N_tilde), "cell factors", k, c);
          check((int)dof_positions(t).size() == per, "dof positions", k, c);
          if (k > method) {
            Mat P = temporal_prolongation(t, temporal(problem, method, k - 1, c, 0.05));
            check(P.r == t.n_t && finite(P), "k prolongation", k, c);
          }
          if (c % 2 == 0) {
            Mat P = temporal_prolongation(t, temporal(problem, method, k, c / 2, 0.1));
            check(P.r == t.n_t && finite(P), "tau prolongation", k, c);
          }
        }
  // dense inverse and the generalised symmetric eigenproblem on seeded SPD pairs
  unsigned s = 12345u;
  auto rnd = [&]() { s = s * 1103515245u + 12345u; return ((s >> 8) & 0xffff) / 65536.0 - 0.5; };
  for (int n = 1; n <= 9; ++n) {
    Mat B(n, n), C(n, n);
    for (double& v : B.a) v = rnd();
    for (double& v : C.a) v = rnd();
    Mat A = matmul(B, B), M = matmul(C, C);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double a = 0, m = 0;
        for (int l = 0; l < n; ++l) { a += B(i, l) * B(j, l); m += C(i, l) * C(j, l); }
        A(i, j) = a + (i == j ? 1.0 : 0.0);
        M(i, j) = m + (i == j ? 1.0 : 0.0);
      }
    Mat Ai = inverse(A), I = matmul(Ai, A);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) check(std::fabs(I(i, j) - (i == j)) < 1e-10, "inverse", i, j);
    Mat Q;
    Vec lam;
    sym_gen_eig(A, M, Q, lam);
    Mat MQ = matmul(M, Q), AQ = matmul(A, Q);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) check(std::fabs(AQ(i, j) - lam[j] * MQ(i, j)) < 1e-9, "eigenpair", i, j);
  }
  bool threw = false;
  try {
    Mat Z(3, 3);
    inverse(Z);
  } catch (const std::exception&) {
    threw = true;
  }
  check(threw, "singular inverse throws", 0, 0);
  if (bad == 0) std::printf("ok\n");
  return bad == 0 ? 0 : 1;
}
"""


def test_host_numerics_under_asan_and_ubsan():
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    with tempfile.TemporaryDirectory() as d:
        drv = os.path.join(d, "driver.cpp")
        open(drv, "w").write(DRIVER)
        exe = os.path.join(d, "driver")
        cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-I", CSRC,
               os.path.join(CSRC, "hostmath.cpp"), drv, "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert r.returncode == 0 and r.stdout.strip().endswith("ok"), (r.stdout[-2000:], r.stderr[-4000:])
