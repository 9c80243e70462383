"""One-dimensional nodal basis, Gauss quadrature and line operators (oracle).

TEST INFRASTRUCTURE ONLY: part of the plain FP64 CPU oracle.  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it.

Follows Section 2.1 (nodes ``0 = s_0 < ... < s_p = 1``, Lagrange basis, the
line mass matrix of eq. ``reqn``) and Section 2.2 (Gauss-Legendre rule with
``ceil((3p+1)/2)`` points, i.e. exact for degree 3p; the pre-factorised mass
matrix; the test-function derivative tabulated at the Gauss points).
"""
from __future__ import annotations

import math

import numpy as np


def _legendre_pair(n: int, x: np.ndarray):
    """Return (P_n(x), P_{n-1}(x)) by the three-term recurrence."""
    pm = np.ones_like(x)
    if n == 0:
        return pm, np.zeros_like(x)
    pc = x.copy()
    for k in range(2, n + 1):
        pm, pc = pc, ((2 * k - 1) * x * pc - (k - 1) * pm) / k
    return pc, pm


def gll_nodes(p: int) -> np.ndarray:
    """Nodes s_i: Gauss-Lobatto-Legendre points on [0,1] (s_0 = 0, s_p = 1).

    The paper only asks for an increasing sequence with fixed end points; the
    Lobatto family is the reading taken here.  Interior nodes are the zeros of
    P_p', found by Newton's method with P_p'' from Legendre's equation.
    """
    x = -np.cos(math.pi * np.arange(p + 1) / p)
    inner = x[1:-1].copy()
    for _ in range(60):
        if inner.size == 0:
            break
        P, Pm = _legendre_pair(p, inner)
        d1 = p * (Pm - inner * P) / (1 - inner ** 2)
        d2 = (2 * inner * d1 - p * (p + 1) * P) / (1 - inner ** 2)
        step = d1 / d2
        inner -= step
        if np.max(np.abs(step)) < 1e-17:
            break
    x = np.concatenate([[-1.0], np.sort(inner), [1.0]])
    return 0.5 * (x + 1.0)


def n_gauss(p: int) -> int:
    """Number of Gauss points: ceil((3p+1)/2) (Section 2.2)."""
    return int(math.ceil((3 * p + 1) / 2))


def gauss_legendre(n: int):
    """Gauss-Legendre nodes and weights on [0,1] (zeros of P_n by Newton)."""
    x = np.cos(math.pi * (np.arange(n) + 0.75) / (n + 0.5))
    for _ in range(100):
        P, Pm = _legendre_pair(n, x)
        dP = n * (Pm - x * P) / (1 - x ** 2)
        step = P / dP
        x -= step
        if np.max(np.abs(step)) < 1e-17:
            break
    P, Pm = _legendre_pair(n, x)
    dP = n * (Pm - x * P) / (1 - x ** 2)
    w = 2.0 / ((1 - x ** 2) * dP ** 2)
    order = np.argsort(x)
    return 0.5 * (x[order] + 1.0), 0.5 * w[order]


def lagrange(s: np.ndarray, x: np.ndarray) -> np.ndarray:
    """phi[q, i] = phi_i(x_q) = prod_{j != i} (x_q - s_j) / (s_i - s_j)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = s.size
    out = np.ones((x.size, n))
    for i in range(n):
        for j in range(n):
            if j != i:
                out[:, i] *= (x - s[j]) / (s[i] - s[j])
    return out


def lagrange_deriv(s: np.ndarray, x: np.ndarray) -> np.ndarray:
    """dphi[q, i] = phi_i'(x_q), by the product rule on the product formula."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = s.size
    out = np.zeros((x.size, n))
    for i in range(n):
        for k in range(n):
            if k == i:
                continue
            term = np.full(x.size, 1.0 / (s[i] - s[k]))
            for j in range(n):
                if j != i and j != k:
                    term *= (x - s[j]) / (s[i] - s[j])
            out[:, i] += term
    return out


class LineOps:
    """The constant 1-D operators of one line (Section 2.2).

    Attributes
    ----------
    s      : nodes, shape [p+1]
    xg, wg : Gauss points / weights on [0,1], shape [ng]
    I      : I[g, i] = phi_i(xg)   (interpolation to Gauss points)
    Dg     : Dg[g, i] = phi_i'(xg) (test-function derivative at Gauss points)
    M      : mass matrix M[i, j] = int phi_i phi_j = sum_g w_g I[g,i] I[g,j]
    Mchol  : lower Cholesky factor of M (the paper pre-factorises M)
    Dn     : Dn[i, j] = phi_j'(s_i) (nodal differentiation, for the mapping)
    """

    def __init__(self, p: int, nodes: str = "gll"):
        self.p = p
        self.n1 = p + 1
        if nodes == "gll":
            self.s = gll_nodes(p)
        elif nodes == "equispaced":
            self.s = np.linspace(0.0, 1.0, p + 1)
        else:
            raise ValueError(nodes)
        self.ng = n_gauss(p)
        self.xg, self.wg = gauss_legendre(self.ng)
        self.I = lagrange(self.s, self.xg)
        self.Dg = lagrange_deriv(self.s, self.xg)
        self.M = self.I.T @ (self.wg[:, None] * self.I)
        self.Mchol = np.linalg.cholesky(self.M)
        self.Dn = lagrange_deriv(self.s, self.s)

    def solve_mass(self, b: np.ndarray) -> np.ndarray:
        """Solve M r = b (first axis) with the Cholesky factor."""
        y = np.linalg.solve(self.Mchol, b)
        return np.linalg.solve(self.Mchol.T, y)
