"""The library's host-side temporal set-up (C++) against the oracle (Python), on the CPU: slab
matrices M_T, A_T, N_T for both problems and both methods (Sections 2.1-2.2), and the temporal
prolongations between the k- and tau-levels of the temporal hierarchy (Section 3.2).  The two
implementations share no code; the library calls are host only."""
import os

import numpy as np
import pytest

from oracle import temporal

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2408_04372_amd",
                   "libstmg.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libstmg.so not built")


def _lib():
    from paper_2408_04372_amd import _lib
    return _lib


@pytest.mark.parametrize("problem", [0, 1])
@pytest.mark.parametrize("method,k", [(0, 0), (0, 1), (0, 3), (1, 1), (1, 2), (1, 4)])
@pytest.mark.parametrize("c", [1, 3])
def test_slab_matrices_match_oracle(problem, method, k, c):
    tau = 0.07
    M, A, N = _lib().temporal_matrices(problem, method, k, c, tau)
    s = temporal.slab(problem, method, k, c, tau)
    for got, ref in ((M, s.M_T), (A, s.A_T), (N, s.N_T)):
        assert got.shape == ref.shape
        assert np.allclose(got, ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("problem", [0, 1])
@pytest.mark.parametrize("method,k,c", [(0, 2, 8), (0, 3, 4), (1, 2, 8), (1, 4, 2)])
def test_temporal_prolongations_match_oracle(problem, method, k, c):
    tau = 0.05
    fine = temporal.slab(problem, method, k, c, tau)
    T = c * tau
    cur = fine
    levels = temporal.time_levels(fine)
    assert levels
    for co in levels:
        kf, cf = temporal.degree(cur), cur.n_t // cur.nt_cell
        kc, cc = temporal.degree(co), co.n_t // co.nt_cell
        P = _lib().temporal_prolongation(problem, method, kf, cf, kc, cc, T)
        ref = temporal.prolongation(cur, co)
        assert P.shape == ref.shape
        assert np.allclose(P, ref, rtol=0, atol=1e-13), (kf, cf, kc, cc)
        cur = co


def test_host_queries_reject_bad_arguments():
    L = _lib()
    with pytest.raises(L.StmgError):
        L.temporal_matrices(2, 0, 1, 1, 0.1)           # problem
    with pytest.raises(L.StmgError):
        L.temporal_matrices(0, 1, 0, 1, 0.1)           # cGP(0)
    with pytest.raises(L.StmgError):
        L.temporal_matrices(0, 0, 1, 1, -0.1)          # tau
    with pytest.raises(L.StmgError):
        L.temporal_prolongation(0, 0, 1, 4, 2, 2, 1.0)  # coarse degree above fine
    with pytest.raises(L.StmgError):
        L.temporal_prolongation(0, 0, 1, 4, 1, 3, 1.0)  # 3 does not divide 4


@pytest.mark.parametrize("problem", [0, 1])
@pytest.mark.parametrize("method,k", [(0, 0), (0, 2), (1, 1), (1, 3)])
def test_smoother_temporal_factors_are_the_diagonal_time_cell_blocks(problem, method, k):
    # every time cell's local block of the smoother uses the diagonal time-cell blocks of M_T and
    # N_T (eq. vanka0); they are the same for every cell of the slab
    tau, c = 0.04, 4
    Mt, Nt = _lib().temporal_cell_factors(problem, method, k, tau)
    s = temporal.slab(problem, method, k, c, tau)
    n = s.nt_cell
    assert Mt.shape == (n, n)
    for m in range(c):
        blk = slice(m * n, (m + 1) * n)
        assert np.allclose(Mt, s.M_T[blk, blk], rtol=1e-12, atol=1e-14)
        assert np.allclose(Nt, s.N_T[blk, blk], rtol=1e-12, atol=1e-13 * np.abs(s.N_T).max())
