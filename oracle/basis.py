"""1D node sets, quadrature rules and Lagrange bases on the reference interval [0, 1].

Section 2 defines Q_p through a nodal Lagrange basis without naming the nodes;
the reading used here is Gauss-Lobatto-Legendre (GLL) nodes.  Section 2.1 puts
the dG(k) temporal basis at the k+1 Gauss-Radau points (right-sided: the last
node is t = 1, which the slab coupling through the previous end value needs);
Section 2.2 puts the cGP(k) trial basis at the k+1 Gauss-Lobatto points.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as L


def gauss(n: int):
    """n-point Gauss-Legendre rule on [0, 1]: (points, weights)."""
    x, w = L.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def gauss_lobatto(n: int) -> np.ndarray:
    """n >= 2 Gauss-Lobatto points on [0, 1] (endpoints plus roots of P'_{n-1})."""
    if n < 2:
        raise ValueError("Gauss-Lobatto needs at least two points")
    inner = L.Legendre.basis(n - 1).deriv().roots() if n > 2 else np.array([])
    x = np.concatenate(([-1.0], np.sort(np.real(inner)), [1.0]))
    return 0.5 * (x + 1.0)


def gauss_radau_right(n: int) -> np.ndarray:
    """n-point Gauss-Radau points on [0, 1] that include t = 1.

    On [-1, 1] they are the roots of P_{n-1}(x) - P_n(x) (x = 1 is one of them).
    """
    if n == 1:
        return np.array([1.0])
    c = np.zeros(n + 1)
    c[n - 1] = 1.0
    c[n] = -1.0
    r = np.sort(np.real(L.legroots(c)))
    r[-1] = 1.0
    return 0.5 * (r + 1.0)


def lagrange(nodes: np.ndarray, x: np.ndarray):
    """Values and first derivatives of the Lagrange basis on `nodes` at points x.

    Returns (V, D) with V[q, i] = l_i(x_q) and D[q, i] = l_i'(x_q), from the
    product formula (no barycentric shortcuts).
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    V = np.ones((len(x), n))
    D = np.zeros((len(x), n))
    for i in range(n):
        others = [j for j in range(n) if j != i]
        den = np.prod([nodes[i] - nodes[j] for j in others]) if others else 1.0
        num = np.ones_like(x)
        for j in others:
            num = num * (x - nodes[j])
        V[:, i] = num / den
        dsum = np.zeros_like(x)
        for m in others:
            term = np.ones_like(x)
            for j in others:
                if j != m:
                    term = term * (x - nodes[j])
            dsum = dsum + term
        D[:, i] = dsum / den
    return V, D
