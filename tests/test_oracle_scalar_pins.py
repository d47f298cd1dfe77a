"""Pins of the slab systems on one spatial degree of freedom (CPU only).

With a "spatial" mesh of one node, M_h = mu and A_h = kappa are positive scalars and every
slab system of Sections 2.1-2.2 becomes a small temporal system whose exact behaviour is known:

  * wave (eqs. wave-cg-dg-at-once, wave-cg-cg-at-once): mu u'' + kappa u = 0 is the first-order
    system Y' = J Y, Y = (u, v), J = [[0, 1], [-kappa/mu, 0]].  dG(k) on the first-order system is
    the (k, k+1) Pade approximant of exp(tau J) at every time-cell end, cGP(k) the (k, k) one.
    The slab solves the condensed system for U and recovers V (eqs. wave-cg-dg-ade,
    wave-cg-cg-ade), so these pins check N_T = A_T M_T^{-1} A_T, the u0 / v0 coupling terms of the
    right-hand side and the velocity recovery, with nonzero u0 and v0.
  * heat: mu u' + kappa u = 0 gives the scalar Pade functions of exp(-tau kappa/mu) (pinned
    elsewhere through the one-cell amplification); here through the whole slab and its
    right-hand side with c > 1 cells.
  * loads: a solution that is linear in time, u = a + b t, lies in every trial space with k >= 1
    and the node rules integrate its load exactly, so the slab reproduces it at every temporal
    DoF (and v = b for the wave problem).  This pins the load term (M_T (x) I) F and, for cGP,
    the start-value load F0 against the coupling terms.

The Pade approximants are written from their closed-form coefficients, independently of the
oracle's temporal matrices.
"""
from math import factorial
from types import SimpleNamespace

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import rhs, spacetime, temporal


def pade(m: int, n: int, Z: np.ndarray) -> np.ndarray:
    """R_{m,n}(Z) = Q_n(Z)^{-1} P_m(Z), the (m, n) Pade approximant of exp at a square matrix Z."""
    I = np.eye(Z.shape[0])
    P = np.zeros_like(Z)
    Q = np.zeros_like(Z)
    Zj = I.copy()
    for j in range(max(m, n) + 1):
        if j <= m:
            P = P + factorial(m + n - j) * factorial(m) / (factorial(m + n) * factorial(j) * factorial(m - j)) * Zj
        if j <= n:
            Q = Q + factorial(m + n - j) * factorial(n) / (factorial(m + n) * factorial(j) * factorial(n - j)) \
                * (-1) ** j * Zj
        Zj = Zj @ Z
    return np.linalg.solve(Q, P)


def scalar_operator(problem: int, method: int, k: int, c: int, tau: float, mu: float, kappa: float,
                    t0: float = 0.0):
    """Slab operator on one spatial DoF: M_h = mu, A_h = kappa (no Dirichlet node)."""
    sl = temporal.slab(problem, method, k, c, tau, t0)
    M = sp.csr_matrix([[mu]])
    A = sp.csr_matrix([[kappa]])
    return spacetime.SlabOperator(space=SimpleNamespace(n_x=1), slab=sl, M=M, A=A, Mi=M, Ai=A,
                                  bmask=np.array([False]))


def test_pade_closed_form_is_exp_to_its_order():
    # the coefficient formula itself: R_{m,n}(z) - exp(z) = O(z^(m+n+1))
    for m, n in ((1, 2), (2, 2), (2, 3), (3, 3), (3, 4)):
        # exp(z) - R_{m,n}(z) = (-1)^n m! n! / ((m+n)! (m+n+1)!) z^(m+n+1) + O(z^(m+n+2))
        lead = (-1) ** n * factorial(m) * factorial(n) / (factorial(m + n) * factorial(m + n + 1))
        z = 0.1
        err = np.exp(z) - pade(m, n, np.array([[z]]))[0, 0]
        assert err / (lead * z ** (m + n + 1)) == pytest.approx(1.0, rel=0.2)
    # (1, 1) is the trapezoidal rule, (0, 1) backward Euler
    z = 0.37
    assert pade(1, 1, np.array([[z]]))[0, 0] == pytest.approx((1 + z / 2) / (1 - z / 2), rel=1e-15)
    assert pade(0, 1, np.array([[z]]))[0, 0] == pytest.approx(1 / (1 - z), rel=1e-15)


@pytest.mark.parametrize("method,k", [(temporal.DG, 0), (temporal.DG, 1), (temporal.DG, 2), (temporal.DG, 3),
                                      (temporal.CGP, 1), (temporal.CGP, 2), (temporal.CGP, 3)])
@pytest.mark.parametrize("omega_tau", [0.3, 1.7, 6.0])
def test_wave_slab_is_pade_of_the_oscillator(method, k, omega_tau):
    mu, kappa, c = 2.5, 2.5 * 9.0, 3                 # omega^2 = kappa / mu = 9
    tau = omega_tau / 3.0
    op = scalar_operator(temporal.WAVE, method, k, c, tau, mu, kappa)
    u0, v0 = np.array([0.8]), np.array([-1.3])
    F = np.zeros((op.n_t, 1))
    b = rhs.rhs(op, F, F0=np.zeros(1), u0=u0, v0=v0)
    U = op.solve(b)
    V = rhs.velocity(op, U, u0=u0, v0=v0)
    J = np.array([[0.0, 1.0], [-kappa / mu, 0.0]])
    m, n = (k, k + 1) if method == temporal.DG else (k, k)
    R = pade(m, n, tau * J)
    Y = np.array([u0[0], v0[0]])
    nc = op.slab.nt_cell
    for cell in range(c):
        Y = R @ Y
        last = (cell + 1) * nc - 1
        got = np.array([U[last, 0], V[last, 0]])
        assert np.abs(got - Y).max() <= 1e-12 * max(1.0, np.abs(Y).max()), (cell, got, Y)


@pytest.mark.parametrize("method,k", [(temporal.DG, 0), (temporal.DG, 2), (temporal.CGP, 1), (temporal.CGP, 3)])
def test_heat_slab_is_pade_of_the_decay(method, k):
    mu, kappa, c, tau = 0.5, 3.0, 4, 0.21
    op = scalar_operator(temporal.HEAT, method, k, c, tau, mu, kappa)
    u0 = np.array([1.7])
    b = rhs.rhs(op, np.zeros((op.n_t, 1)), F0=np.zeros(1), u0=u0)
    U = op.solve(b)
    m, n = (k, k + 1) if method == temporal.DG else (k, k)
    r = pade(m, n, np.array([[-tau * kappa / mu]]))[0, 0]
    nc = op.slab.nt_cell
    for cell in range(c):
        assert U[(cell + 1) * nc - 1, 0] == pytest.approx(u0[0] * r ** (cell + 1), rel=1e-12)


@pytest.mark.parametrize("problem", [temporal.HEAT, temporal.WAVE])
@pytest.mark.parametrize("method,k", [(temporal.DG, 1), (temporal.DG, 3), (temporal.CGP, 1), (temporal.CGP, 2)])
def test_linear_in_time_solution_is_reproduced(problem, method, k):
    # mu u' + kappa u = f (heat) or mu u'' + kappa u = f (wave) with u = a + b t
    mu, kappa, c, tau, t0 = 1.3, 4.0, 3, 0.17, 0.4
    a, bb = 0.6, -2.2
    op = scalar_operator(problem, method, k, c, tau, mu, kappa, t0=t0)
    u = lambda t: a + bb * t
    f = (lambda t: mu * bb + kappa * u(t)) if problem == temporal.HEAT else (lambda t: kappa * u(t))
    F = f(op.slab.times)[:, None]
    u0, v0 = np.array([u(t0)]), np.array([bb])
    b = rhs.rhs(op, F, F0=np.array([f(t0)]), u0=u0, v0=v0)
    U = op.solve(b)
    assert np.abs(U[:, 0] - u(op.slab.times)).max() <= 1e-12
    if problem == temporal.WAVE:
        V = rhs.velocity(op, U, u0=u0, v0=v0)
        assert np.abs(V[:, 0] - bb).max() <= 1e-12


def test_pins_catch_planted_coupling_errors():
    # a sign error in the u0 coupling of the wave dG right-hand side, or in the velocity
    # recovery, breaks the oscillator pin
    mu, kappa, tau = 1.0, 4.0, 0.3
    op = scalar_operator(temporal.WAVE, temporal.DG, 1, 2, tau, mu, kappa)
    s = op.slab
    u0, v0 = np.array([1.0]), np.array([0.5])
    g_a = s.A_T @ np.linalg.solve(s.M_T, s.a)
    b_bad = np.outer(s.a, v0) - np.outer(g_a, u0)           # wrong sign on the u0 term
    U = op.solve(b_bad)
    V = rhs.velocity(op, U, u0=u0, v0=v0)
    R = pade(1, 2, tau * np.array([[0.0, 1.0], [-kappa / mu, 0.0]]))
    Y = R @ np.array([1.0, 0.5])
    assert np.abs(np.array([U[1, 0], V[1, 0]]) - Y).max() > 1e-2
    U = op.solve(rhs.rhs(op, np.zeros((op.n_t, 1)), u0=u0, v0=v0))
    V_bad = np.linalg.solve(s.M_T, s.A_T @ U + np.outer(s.a, u0))   # wrong sign in the recovery
    assert abs(V_bad[1, 0] - Y[1]) > 1e-2
