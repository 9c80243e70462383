"""Pins for the oracle's 1-D basis, quadrature and line operators (Sections 2.1-2.2)."""
import math

import numpy as np
import pytest

from oracle.basis import LineOps, gauss_legendre, gll_nodes, n_gauss


def test_gll_closed_forms():
    # Lobatto points on [0,1] for p = 1..4 (interior points are zeros of P_p')
    assert np.allclose(gll_nodes(1), [0, 1], atol=1e-15)
    assert np.allclose(gll_nodes(2), [0, 0.5, 1], atol=1e-15)
    r5 = 1 / math.sqrt(5)
    assert np.allclose(gll_nodes(3), [0, (1 - r5) / 2, (1 + r5) / 2, 1], atol=1e-15)
    r37 = math.sqrt(3 / 7)
    assert np.allclose(gll_nodes(4), [0, (1 - r37) / 2, 0.5, (1 + r37) / 2, 1], atol=1e-15)


@pytest.mark.parametrize("p", range(1, 9))
def test_gauss_rule(p):
    ng = n_gauss(p)
    assert ng == math.ceil((3 * p + 1) / 2)
    x, w = gauss_legendre(ng)
    # library routine on [-1,1]
    xl, wl = np.polynomial.legendre.leggauss(ng)
    assert np.allclose(x, (xl + 1) / 2, atol=1e-15)
    assert np.allclose(w, wl / 2, atol=1e-15)
    assert abs(w.sum() - 1) < 1e-14
    # exact for every monomial up to degree 2 ng - 1 >= 3p
    for k in range(2 * ng):
        assert abs((w * x ** k).sum() - 1.0 / (k + 1)) < 1e-14
    assert 2 * ng - 1 >= 3 * p


@pytest.mark.parametrize("p", range(1, 8))
def test_mass_matrix_properties(p):
    o = LineOps(p)
    assert np.allclose(o.M, o.M.T, atol=1e-16)
    assert np.all(np.linalg.eigvalsh(o.M) > 0)
    # row sums are the integrals of the basis functions; they sum to the length 1
    xg, wg = gauss_legendre(30)
    from oracle.basis import lagrange
    ints = (wg[:, None] * lagrange(o.s, xg)).sum(0)
    assert np.allclose(o.M.sum(1), ints, atol=1e-14)
    assert abs(ints.sum() - 1) < 1e-14
    # Cholesky factor reproduces M
    assert np.allclose(o.Mchol @ o.Mchol.T, o.M, atol=1e-15)


def test_p1_closed_form():
    o = LineOps(1)
    assert np.allclose(o.M, [[1 / 3, 1 / 6], [1 / 6, 1 / 3]], atol=1e-15)
    L0 = o.solve_mass(np.array([1.0, 0.0]))
    L1 = o.solve_mass(np.array([0.0, 1.0]))
    assert np.allclose(L0, [4, -2], atol=1e-13)
    assert np.allclose(L1, [-2, 4], atol=1e-13)


@pytest.mark.parametrize("p", range(1, 8))
def test_line_operator_differentiates_polynomials(p):
    """1-D upwind DG for f = a u on one line is exact for polynomial data (degree <= p).

    With consistent end fluxes a u(1), -a u(0), the right-hand side is
    int (a u)' phi_i, so M^{-1} b is the derivative a u' at the nodes.
    """
    o = LineOps(p)
    rng = np.random.default_rng(p)
    coef = rng.standard_normal(p + 1)
    u = np.polynomial.polynomial.polyval(o.s, coef)
    du = np.polynomial.polynomial.polyval(o.s, np.polynomial.polynomial.polyder(coef))
    a = 1.7
    ug = o.I @ u
    b = -(o.wg[:, None] * o.Dg).T @ (a * ug)
    b[-1] += a * u[-1]
    b[0] += -a * u[0]
    r = o.solve_mass(b)
    assert np.allclose(r, a * du, atol=1e-11 * max(1, np.abs(du).max()))
    # the nodal differentiation matrix is exact on the same data
    assert np.allclose(o.Dn @ u, du, atol=1e-11 * max(1, np.abs(du).max()))


def test_basis_is_cardinal():
    for p in range(1, 8):
        o = LineOps(p)
        from oracle.basis import lagrange
        assert np.allclose(lagrange(o.s, o.s), np.eye(p + 1), atol=1e-14)
        # partition of unity: derivatives sum to zero
        assert np.allclose(o.Dg.sum(1), 0, atol=1e-11)
