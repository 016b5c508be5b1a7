"""Pins of the oracle's 1D rules and barycentric interpolation (paper Sec. 4)."""
import numpy as np
import pytest

from oracle import quadrature as qd


@pytest.mark.parametrize("nq", range(1, 12))
def test_gauss_legendre_exactness_and_library(nq):
    x, w = qd.gauss_legendre(nq)
    assert abs(w.sum() - 2.0) < 1e-14
    for m in range(2 * nq):          # exact to degree 2 nq - 1 (Sec. 4)
        exact = 0.0 if m % 2 else 2.0 / (m + 1)
        assert abs(np.sum(w * x ** m) - exact) < 1e-14
    xl, wl = np.polynomial.legendre.leggauss(nq)   # textbook/library rule
    assert np.allclose(x, xl, atol=1e-15) and np.allclose(w, wl, atol=1e-14)


@pytest.mark.parametrize("p", range(1, 10))
def test_gauss_lobatto_exactness(p):
    x, w = qd.gauss_lobatto(p)
    assert x[0] == -1.0 and x[-1] == 1.0 and np.all(np.diff(x) > 0)
    assert abs(w.sum() - 2.0) < 1e-14
    for m in range(2 * p):           # exact to degree 2p - 1 (Sec. 4)
        exact = 0.0 if m % 2 else 2.0 / (m + 1)
        assert abs(np.sum(w * x ** m) - exact) < 1e-13
    # interior nodes are the roots of P_p'
    dP = np.polynomial.legendre.Legendre.basis(p).deriv()
    assert np.allclose(dP(x[1:-1]), 0.0, atol=1e-12)
    # degree 2p is NOT integrated exactly (the rule has exactly the stated order)
    assert abs(np.sum(w * x ** (2 * p)) - 2.0 / (2 * p + 1)) > 1e-6


@pytest.mark.parametrize("p", range(1, 9))
def test_barycentric_weights_closed_forms(p):
    """Generic product weights agree, up to one constant, with the closed forms
    (-1)^j sqrt(w_j) at GLL nodes and (-1)^j sqrt((1 - x_j^2) w_j) at GL nodes."""
    x, w = qd.gauss_lobatto(p)
    r = qd.barycentric_weights(x) / ((-1.0) ** np.arange(p + 1) * np.sqrt(w))
    assert np.ptp(r / r[0]) < 1e-12
    xg, wg = qd.gauss_legendre(p + 1)
    r = qd.barycentric_weights(xg) / ((-1.0) ** np.arange(p + 1) * np.sqrt((1 - xg ** 2) * wg))
    assert np.ptp(r / r[0]) < 1e-12


@pytest.mark.parametrize("p", range(0, 9))
def test_lagrange_cardinal_and_polynomial_exactness(p):
    nodes = qd.trace_nodes(p)
    L = qd.lagrange_matrix(nodes, nodes)
    assert np.array_equal(L, np.eye(p + 1))
    pts = np.linspace(-0.93, 0.97, 13)
    coef = np.random.default_rng(p).standard_normal(p + 1)
    poly = np.polynomial.Polynomial(coef)
    assert np.allclose(qd.lagrange_matrix(nodes, pts) @ poly(nodes), poly(pts), atol=1e-12)
    dpoly = poly.deriv()
    assert np.allclose(qd.lagrange_derivative_matrix(nodes, pts) @ poly(nodes), dpoly(pts), atol=1e-10)
