"""1D rules and barycentric Lagrange interpolation (paper Sec. 4).

Test infrastructure only (see oracle/__init__.py).

* Gauss-Legendre (GL) rule with nq points: exact for polynomials of degree
  2nq-1 (Sec. 4, discussion of GL vs GLL exactness).
* Gauss-Legendre-Lobatto (GLL) nodes of degree p: the endpoints -1, +1 and the
  p-1 roots of P_p'; weights 2 / (p (p+1) P_p(x_j)^2).  GLL with p+1 points is
  exact to degree 2p-1 (Sec. 4).  The GLL nodes are the interpolation nodes of
  the nodal tensor-product basis (Sec. 4).
* Barycentric weights by the generic product formula
  W_j = 1 / prod_{m != j} (x_j - x_m) and the second (true) barycentric
  formula for evaluating l_j anywhere (Sec. 4, Berrut & Trefethen).  The
  closed-form weights printed in Sec. 4 are garbled; the generic product is
  used and the closed forms (up to a constant) are checked in the tests.
* p = 0: the one-point "nodal" basis is the constant 1 and its node is taken
  at 0 (the paper leaves p = 0 undefined for GLL).
"""
import numpy as np


def legendre_and_derivative(n, x):
    """P_n(x) and P_n'(x) by the three-term recurrence (Bonnet)."""
    x = np.asarray(x, dtype=np.float64)
    p0 = np.ones_like(x)
    if n == 0:
        return p0, np.zeros_like(x)
    p1 = x.copy()
    for m in range(2, n + 1):
        p0, p1 = p1, ((2 * m - 1) * x * p1 - (m - 1) * p0) / m
    # derivative from P_n' = n (x P_n - P_{n-1}) / (x^2 - 1); at |x| = 1 use the
    # closed value n(n+1)/2 * (+-1)^(n+1)
    dp = np.empty_like(x)
    inner = np.abs(np.abs(x) - 1.0) > 1e-14
    dp[inner] = n * (x[inner] * p1[inner] - p0[inner]) / (x[inner] ** 2 - 1.0)
    dp[~inner] = 0.5 * n * (n + 1) * np.sign(x[~inner]) ** (n + 1)
    return p1, dp


def gauss_legendre(nq):
    """GL nodes (increasing) and weights on [-1, 1] by Newton on P_nq."""
    if nq < 1:
        raise ValueError("nq >= 1")
    k = np.arange(1, nq + 1)
    x = -np.cos(np.pi * (k - 0.25) / (nq + 0.5))  # classical starting guesses
    for _ in range(100):
        p, dp = legendre_and_derivative(nq, x)
        dx = p / dp
        x = x - dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    p, dp = legendre_and_derivative(nq, x)
    w = 2.0 / ((1.0 - x ** 2) * dp ** 2)
    return x, w


def gauss_lobatto(p):
    """GLL nodes (increasing) and weights for degree p >= 1 (p + 1 points)."""
    if p < 1:
        raise ValueError("GLL needs p >= 1")
    if p == 1:
        return np.array([-1.0, 1.0]), np.array([1.0, 1.0])
    # interior nodes: roots of P_p'.  Newton on P_p' with P_p'' from the
    # Legendre ODE (1 - x^2) P'' = 2 x P' - p (p+1) P.
    k = np.arange(1, p)
    x = -np.cos(np.pi * k / p)
    for _ in range(100):
        P, dP = legendre_and_derivative(p, x)
        d2P = (2.0 * x * dP - p * (p + 1) * P) / (1.0 - x ** 2)
        dx = dP / d2P
        x = x - dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    x = np.concatenate(([-1.0], x, [1.0]))
    P, _ = legendre_and_derivative(p, x)
    w = 2.0 / (p * (p + 1) * P ** 2)
    return x, w


def trace_nodes(p):
    """Interpolation nodes of the degree-p nodal basis: GLL for p >= 1, {0} for p = 0."""
    if p == 0:
        return np.array([0.0])
    return gauss_lobatto(p)[0]


def barycentric_weights(nodes):
    """Generic barycentric weights W_j = 1 / prod_{m != j}(x_j - x_m) (Sec. 4)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    n = len(nodes)
    W = np.ones(n)
    for j in range(n):
        for m in range(n):
            if m != j:
                W[j] /= (nodes[j] - nodes[m])
    return W


def lagrange_matrix(nodes, pts):
    """L[q, j] = l_j(pts[q]) by the second barycentric formula (Sec. 4).

    A point that coincides with a node returns the Kronecker delta row."""
    nodes = np.asarray(nodes, dtype=np.float64)
    pts = np.atleast_1d(np.asarray(pts, dtype=np.float64))
    n = len(nodes)
    if n == 1:
        return np.ones((len(pts), 1))
    W = barycentric_weights(nodes)
    L = np.zeros((len(pts), n))
    for q, x in enumerate(pts):
        diff = x - nodes
        hit = np.nonzero(diff == 0.0)[0]
        if len(hit):
            L[q, hit[0]] = 1.0
            continue
        t = W / diff
        L[q, :] = t / t.sum()
    return L


def diff_matrix(nodes):
    """D[a, b] = l_b'(x_a) at the nodes: D_ab = (W_b/W_a)/(x_a - x_b), D_aa = -sum_b D_ab."""
    nodes = np.asarray(nodes, dtype=np.float64)
    n = len(nodes)
    if n == 1:
        return np.zeros((1, 1))
    W = barycentric_weights(nodes)
    D = np.zeros((n, n))
    for a in range(n):
        for b in range(n):
            if a != b:
                D[a, b] = (W[b] / W[a]) / (nodes[a] - nodes[b])
        D[a, a] = -D[a, :].sum()
    return D


def lagrange_derivative_matrix(nodes, pts):
    """L'[q, j] = l_j'(pts[q]).

    l_j' is a polynomial of degree <= p, so it equals its interpolant at the
    nodes: l_j'(x) = sum_a l_a(x) D[a, j]."""
    return lagrange_matrix(nodes, pts) @ diff_matrix(nodes)
