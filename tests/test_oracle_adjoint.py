"""Pins of the oracle's misfit gradient: central finite differences of L(theta)
computed through the direct solver, which involves no adjoint code."""
import numpy as np
import pytest

from oracle import adjoint, hdg
from workloads import normal_vector


def _case(n, k, seed, with_bd):
    rng = np.random.default_rng(seed)
    theta = rng.standard_normal(n * n)
    pr = hdg.Problem(n, k, np.exp(theta))
    f_qp = 1.0 + 0.5 * rng.standard_normal((n * n, pr.ref.nq ** 2))
    lam_bd = pr.boundary_trace(lambda x, y: x * x - 0.5 * y) if with_bd else None
    U_obs = 0.01 * rng.standard_normal((n * n, (k + 1) ** 2))
    return theta, adjoint.Misfit(n, k, f_qp, U_obs, lam_bd=lam_bd)


@pytest.mark.parametrize("n,k,with_bd", [(4, 1, False), (4, 2, True), (3, 3, False), (2, 0, True)])
def test_gradient_matches_central_differences(n, k, with_bd):
    theta, M = _case(n, k, 11 + n + k, with_bd)
    L0, g, _ = M.gradient(theta)
    h = 1e-5
    fd = np.zeros_like(theta)
    for e in range(theta.size):
        tp, tm = theta.copy(), theta.copy()
        tp[e] += h
        tm[e] -= h
        fd[e] = (M.value(tp) - M.value(tm)) / (2 * h)
    # central differences: truncation O(h^2 |L'''|) and rounding O(eps L / h)
    assert np.abs(g - fd).max() <= 1e-6 * max(np.abs(fd).max(), 1e-30), np.abs(g - fd).max()


def test_directional_derivative_second_order():
    """Taylor test: |L(theta + t v) - L(theta) - t g.v| = O(t^2)."""
    n, k = 6, 2
    theta, M = _case(n, k, 5, True)
    L0, g, _ = M.gradient(theta)
    v = normal_vector(theta.size, 3)
    errs = []
    for t in (1e-2, 5e-3, 2.5e-3):
        errs.append(abs(M.value(theta + t * v) - L0 - t * (g @ v)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.5 and 3.5 < r2 < 4.5, errs


def test_zero_misfit_has_zero_gradient():
    n, k = 4, 2
    theta, M = _case(n, k, 9, True)
    _, _, _, Us = M.forward(theta)
    M0 = adjoint.Misfit(n, k, M.f_qp, Us, lam_bd=M.lam_bd)
    L0, g, mu = M0.gradient(theta)
    assert L0 < 1e-25 and np.abs(g).max() < 1e-12 and np.abs(mu).max() < 1e-12
