"""Seeded synthetic inputs and analytic problem data shared by the tests, the
bench and the oracle.

This module holds no arithmetic of the HDG method or of the solver: only
random draws (numpy.random.default_rng with fixed seeds) and closed-form
functions of (x, y) that define PDE data -- the coefficient K, the source
f = -div(K grad u), the exact solution u and flux q = -K grad u, and the
Dirichlet datum g_D = u.  Each side (oracle, HIP library) evaluates these
functions at its own quadrature points.

Workloads (uniform n x n squares on [0,1]^2, tau = 1, zero Dirichlet data
unless stated):
  poisson_sin     n=16, k=1, K=1, u = sin(pi x) sin(pi y)         (small case)
  lognormal_k4    n=256, k=4, K_e = exp(z_e), z ~ N(0,1) seed 2, f = 1
  lognormal_k3    n=1024, k=3, K_e = exp(2 z_e), seed 3, f = 1
The variable-coefficient problem of the paper's convergence table (Sec. 5,
Table tab1) and polynomial exact-solution problems are also defined here.
"""
import numpy as np

PI = np.pi


# ---------------------------------------------------------------- coefficients
def kappa_lognormal(n, sigma, seed):
    """Per-element K_e = exp(sigma z_e), z ~ N(0, 1), e = i + n j."""
    rng = np.random.default_rng(seed)
    return np.exp(sigma * rng.standard_normal(n * n))


def kappa_const(n, value=1.0):
    return np.full(n * n, float(value))


def normal_vector(n_items, seed):
    """i.i.d. N(0, 1) draws (e.g. a random trace vector x for apply parity)."""
    return np.random.default_rng(seed).standard_normal(n_items)


def source_normal(n_elems, nq, seed):
    """Source values i.i.d. N(0, 1) per volume quadrature point, [n_elems, nq*nq]."""
    return np.random.default_rng(seed).standard_normal((n_elems, nq * nq))


# ------------------------------------------------------- manufactured problems
class SinSin:
    """-Laplace u = f, K = 1, u = sin(pi x) sin(pi y) (u = 0 on the boundary)."""
    kappa_value = 1.0

    @staticmethod
    def u(x, y):
        return np.sin(PI * x) * np.sin(PI * y)

    @staticmethod
    def q(x, y):
        return np.array([-PI * np.cos(PI * x) * np.sin(PI * y),
                         -PI * np.sin(PI * x) * np.cos(PI * y)])

    @staticmethod
    def f(x, y):
        return 2.0 * PI * PI * np.sin(PI * x) * np.sin(PI * y)

    gD = None


class TanhProblem:
    """Sec. 5 / Table tab1: K = tanh(x+y) + 1, u = x(x-1) y(y-1) exp(-x^2-y^2)."""

    @staticmethod
    def kappa(x, y):
        return np.tanh(x + y) + 1.0

    @staticmethod
    def _a(x):
        e = np.exp(-x * x)
        g = -2 * x ** 3 + 2 * x ** 2 + 2 * x - 1          # a'(x) = e^{-x^2} g(x)
        dg = -6 * x ** 2 + 4 * x + 2
        return x * (x - 1) * e, e * g, e * (dg - 2 * x * g)  # a, a', a''

    @classmethod
    def u(cls, x, y):
        return cls._a(x)[0] * cls._a(y)[0]

    @classmethod
    def grad_u(cls, x, y):
        ax, dax, _ = cls._a(x)
        ay, day, _ = cls._a(y)
        return np.array([dax * ay, ax * day])

    @classmethod
    def q(cls, x, y):
        return -cls.kappa(x, y) * cls.grad_u(x, y)

    @classmethod
    def f(cls, x, y):
        ax, dax, d2ax = cls._a(x)
        ay, day, d2ay = cls._a(y)
        lap = d2ax * ay + ax * d2ay
        dk = 1.0 - np.tanh(x + y) ** 2                      # dK/dx = dK/dy
        return -cls.kappa(x, y) * lap - dk * (dax * ay + ax * day)

    gD = None  # u vanishes on the boundary of the unit square


class PolyProblem:
    """K = c constant, u = x^k y^k + x y + 1 in Q_k (exact solution of the discrete problem)."""

    def __init__(self, k, c=1.0):
        self.k, self.c = k, float(c)

    def u(self, x, y):
        return x ** self.k * y ** self.k + x * y + 1.0

    def q(self, x, y):
        k, c = self.k, self.c
        ux = k * x ** (k - 1) * y ** k + y if k >= 1 else 0 * x
        uy = k * x ** k * y ** (k - 1) + x if k >= 1 else 0 * x
        return np.array([-c * ux, -c * uy])

    def f(self, x, y):
        k, c = self.k, self.c
        lap = 0.0 * x
        if k >= 2:
            lap = k * (k - 1) * (x ** (k - 2) * y ** k + x ** k * y ** (k - 2))
        return -c * lap

    def gD(self, x, y):
        return self.u(x, y)


class LinearProblem:
    """K = c, u = a0 + a1 x + a2 y (every degree p >= 1 reproduces it)."""

    def __init__(self, a0=0.3, a1=-1.2, a2=0.7, c=1.0):
        self.a = (a0, a1, a2)
        self.c = c

    def u(self, x, y):
        return self.a[0] + self.a[1] * x + self.a[2] * y

    def q(self, x, y):
        return np.array([-self.c * self.a[1] + 0 * x, -self.c * self.a[2] + 0 * y])

    def f(self, x, y):
        return 0.0 * x

    def gD(self, x, y):
        return self.u(x, y)


# ------------------------------------------------------------- named workloads
WORKLOADS = {
    "poisson_sin_n16_k1": dict(n=16, k=1, sigma=None, seed=None, source="sinsin"),
    "lognormal_n256_k4": dict(n=256, k=4, sigma=1.0, seed=2, source="one"),
    "lognormal_n1024_k3": dict(n=1024, k=3, sigma=2.0, seed=3, source="one"),
}


def workload_kappa(name):
    w = WORKLOADS[name]
    if w["sigma"] is None:
        return kappa_const(w["n"], 1.0)
    return kappa_lognormal(w["n"], w["sigma"], w["seed"])
