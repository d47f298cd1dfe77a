"""Pins of the oracle's temporal matrices (Sections 2.1-2.2) against closed forms."""
import math

import numpy as np
import pytest

from oracle import basis, temporal


def pade_exp_neg(m: int, n: int, z):
    """(m, n) Pade approximant of exp(-z): degree-m numerator over degree-n denominator."""
    num = sum(math.factorial(m + n - j) * math.factorial(m)
              / (math.factorial(m + n) * math.factorial(j) * math.factorial(m - j)) * (-z) ** j
              for j in range(m + 1))
    den = sum(math.factorial(m + n - j) * math.factorial(n)
              / (math.factorial(m + n) * math.factorial(j) * math.factorial(n - j)) * z ** j
              for j in range(n + 1))
    return num / den


ZS = [0.3, 2.0, 17.0, 0.5 + 3.0j, 40.0]


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_dg_is_radau_iia_pade(k):
    # dG(k) with right Radau nodes reproduces the (k, k+1) Pade approximant of exp(-z)
    for z in ZS:
        assert abs(temporal.amplification(0, temporal.DG, k, z) - pade_exp_neg(k, k + 1, z)) < 1e-12


@pytest.mark.parametrize("k", [1, 2, 3])
def test_cgp_is_diagonal_pade(k):
    # cGP(k) reproduces the (k, k) Pade approximant (k = 1: Crank-Nicolson)
    for z in ZS:
        assert abs(temporal.amplification(0, temporal.CGP, k, z) - pade_exp_neg(k, k, z)) < 1e-12


def test_dg1_hand_values():
    # dG(1): right Radau nodes {1/3, 1}; basis l1 = 3(1-t)/2, l2 = (3t-1)/2 (worked by hand)
    M, A, alpha, nodes = temporal.dg_local(1, 2.0)
    assert np.allclose(nodes, [1 / 3, 1.0], atol=1e-15)
    assert np.allclose(M, 2.0 * np.diag([3 / 4, 1 / 4]), atol=1e-14)
    assert np.allclose(A, [[9 / 8, 3 / 8], [-9 / 8, 5 / 8]], atol=1e-14)
    assert np.allclose(alpha, [3 / 2, -1 / 2], atol=1e-14)


def test_dg0_is_backward_euler():
    M, A, alpha, _ = temporal.dg_local(0, 0.7)
    assert np.allclose(M, [[0.7]]) and np.allclose(A, [[1.0]]) and np.allclose(alpha, [1.0])


def test_cgp_hand_values():
    # cGP(1): M = tau/2, A = 1, beta = tau/2, alpha = -1 (trapezoidal rule)
    M, A, alpha, beta, _ = temporal.cgp_local(1, 0.4)
    assert np.allclose(M, [[0.2]]) and np.allclose(A, [[1.0]])
    assert np.allclose(beta, [0.2]) and np.allclose(alpha, [-1.0])
    # cGP(2): GL nodes {0, 1/2, 1}; test basis linear at {1/2, 1} (worked by hand)
    M, A, alpha, beta, trial = temporal.cgp_local(2, 1.0)
    assert np.allclose(trial, [0, 0.5, 1])
    assert np.allclose(M, np.diag([2 / 3, 1 / 6]), atol=1e-14)
    assert np.allclose(A, [[4 / 3, 1 / 3], [-4 / 3, 2 / 3]], atol=1e-14)
    assert np.allclose(beta, [1 / 3, -1 / 6], atol=1e-14)
    assert np.allclose(alpha, [-5 / 3, 2 / 3], atol=1e-14)


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
def test_dg_invariants(k):
    tau = 0.37
    M, A, alpha, _ = temporal.dg_local(k, tau)
    # the time derivative of a constant vanishes: only the jump term xi_i(0) survives
    assert np.allclose(A @ np.ones(k + 1), alpha, atol=1e-12)
    # nodal basis at the quadrature nodes: diagonal mass with the Radau weights, total tau
    assert np.allclose(M, np.diag(np.diag(M)), atol=1e-13)
    assert abs(M.sum() - tau) < 1e-13


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_cgp_invariants(k):
    tau = 0.37
    M, A, alpha, beta, _ = temporal.cgp_local(k, tau)
    assert np.allclose(A @ np.ones(k) + alpha, 0.0, atol=1e-12)
    assert np.allclose(M, np.diag(np.diag(M)), atol=1e-13)
    assert abs(M.sum() + beta.sum() - tau) < 1e-13


def test_radau_and_lobatto_nodes():
    r = basis.gauss_radau_right(3)
    assert np.allclose(r, [(4 - math.sqrt(6)) / 10, (4 + math.sqrt(6)) / 10, 1.0], atol=1e-14)
    l = basis.gauss_lobatto(5)
    assert np.allclose(l, [0, (1 - math.sqrt(3 / 7)) / 2, 0.5, (1 + math.sqrt(3 / 7)) / 2, 1], atol=1e-14)


@pytest.mark.parametrize("method,k", [(temporal.DG, 1), (temporal.DG, 2), (temporal.CGP, 2)])
def test_slab_equals_sequential_steps(method, k):
    # scalar heat y' = -lam y: the c-cell slab system reproduces c single-step solves
    lam, tau, c = 3.0, 0.2, 5
    sl = temporal.slab(temporal.HEAT, method, k, c, tau)
    S = sl.M_T * lam + sl.N_T
    y0 = 1.0
    if method == temporal.DG:
        rhs = sl.a * y0
    else:
        rhs = -(sl.a + lam * sl.b_beta) * y0
    U = np.linalg.solve(S, rhs)
    ends = U[sl.nt_cell - 1::sl.nt_cell]
    R = temporal.amplification(0, method, k, lam * tau)
    assert np.allclose(ends, [R ** (m + 1) for m in range(c)], rtol=1e-12)


def test_wave_slab_factor():
    # N_T = A_T M_T^{-1} A_T; its diagonal blocks are all equal to A_tau M_tau^{-1} A_tau
    sl = temporal.slab(temporal.WAVE, temporal.CGP, 2, 4, 0.1)
    M, A, _, _, _ = temporal.cgp_local(2, 0.1)
    loc = A @ np.linalg.solve(M, A)
    for m in range(4):
        s = slice(2 * m, 2 * m + 2)
        assert np.allclose(sl.N_T[s, s], loc, rtol=1e-12)
    assert np.allclose(np.triu(sl.N_T, 2), 0.0)


@pytest.mark.parametrize("method", [0, 1])
def test_temporal_prolongation_reproduces_coarse_functions(method):
    # the embedding of the coarse temporal space: a polynomial of the coarse degree (vanishing at
    # t0 for cGP, whose initial value is constrained) is reproduced exactly at the fine DoF times
    s = temporal.slab(0, method, 3, 4, 0.2, t0=1.0)
    g = lambda t: (t - 1.0) * (2.0 - 0.5 * (t - 1.0))          # degree 2, zero at t0
    cur = s
    for c in temporal.time_levels(s):
        P = temporal.prolongation(cur, c)
        if temporal.degree(c) >= 2:
            assert np.allclose(P @ g(c.times), g(cur.times), atol=1e-12)
        if temporal.degree(c) >= 1:
            lin = lambda t: 3.0 * (t - 1.0)
            assert np.allclose(P @ lin(c.times), lin(cur.times), atol=1e-12)
        else:                                   # dG(0): piecewise constants
            assert np.allclose(P @ np.ones(c.n_t), np.ones(cur.n_t), atol=1e-12)
        cur = c
    assert temporal.degree(cur) == (0 if method == 0 else 1) and cur.n_t // cur.nt_cell == 1


@pytest.mark.parametrize("k,c", [(1, 4), (2, 8), (3, 2), (4, 6)])
def test_dg_prolongation_is_galerkin(k, c):
    # dG: trial and test spaces coincide and the coarse spaces are nested in the fine ones
    # (Section 3.2), so the coarse slab matrices are the Galerkin products of the embedding;
    # a wrong node, weight or cell offset in the embedding breaks this
    s = temporal.slab(0, temporal.DG, k, c, 0.1, t0=0.5)
    cur = s
    levels = temporal.time_levels(s)
    assert levels
    for co in levels:
        P = temporal.prolongation(cur, co)
        for name in ("M_T", "A_T"):
            F, C = getattr(cur, name), getattr(co, name)
            assert np.allclose(P.T @ F @ P, C, rtol=0, atol=1e-13 * np.abs(C).max()), (name, co.n_t)
        cur = co
