"""Pins of the oracle's HDG discretization (paper Secs. 3 and 5)."""
import os

import numpy as np
import pytest

from oracle import hdg, mesh as ms, quadrature as qd
from workloads import PolyProblem, LinearProblem, TanhProblem, SinSin, kappa_lognormal

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 6])
@pytest.mark.parametrize("kappa,n", [(1.0, 4), (0.013, 16), (57.0, 64), (2.5, 1024)])
def test_block_symmetric_psd_constant_kernel(p, kappa, n):
    pr = hdg.Problem(n, p, np.full(n * n, kappa))
    K = pr.element_block(0)
    nrm = np.abs(K).max()
    assert np.abs(K - K.T).max() <= 1e-13 * nrm
    assert np.abs(K @ np.ones(len(K))).max() <= 1e-12 * nrm      # constant trace -> zero flux
    ev = np.linalg.eigvalsh(K)
    assert ev[0] >= -1e-12 * nrm
    assert ev[1] > 1e-9 * nrm                                     # kernel is exactly 1-dimensional


@pytest.mark.parametrize("kappa,tau,n", [(1.0, 1.0, 4), (3.7, 1.0, 16), (0.2, 2.5, 8)])
def test_p0_block_closed_form(kappa, tau, n):
    """p = 0: q_x = -K (l_r - l_l)/h, q_y = -K (l_t - l_b)/h, u = mean(l) + ...; the
    condensed block is K (L (+) L) + tau h (I - 11^T/4), L = [[1,-1],[-1,1]],
    local order (left, right, bottom, top)."""
    h = 1.0 / n
    pr = hdg.Problem(n, 0, np.full(n * n, kappa), tau)
    L = np.array([[1.0, -1.0], [-1.0, 1.0]])
    K0 = kappa * np.block([[L, np.zeros((2, 2))], [np.zeros((2, 2)), L]]) + tau * h * (np.eye(4) - 0.25)
    assert np.abs(pr.element_block(3) - K0).max() < 1e-14 * max(1.0, kappa)


@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_linear_patch(p):
    """Traces of a linear l with K constant: the local solver reproduces l and
    the condensed block returns the outward flux <K grad l . n, mu_m>_e."""
    n, kap = 8, 1.7
    pr = hdg.Problem(n, p, np.full(n * n, kap))
    g = np.array([0.4, -1.3])
    e = 2 + n * 5
    i, j = e % n, e // n
    h = 1.0 / n
    nodes = qd.trace_nodes(p)
    s = (nodes + 1) * h / 2
    x0, y0 = i * h, j * h
    ell = lambda x, y: 0.25 + g[0] * x + g[1] * y
    lam = np.concatenate([ell(x0 + 0 * s, y0 + s), ell(x0 + h + 0 * s, y0 + s),
                          ell(x0 + s, y0 + 0 * s), ell(x0 + s, y0 + h + 0 * s)])
    normals = [(-1, 0), (1, 0), (0, -1), (0, 1)]
    Me = pr.ref.Lq.T @ (pr.ref.Lq * (pr.ref.wq * h / 2)[:, None])
    flux = np.concatenate([kap * (g[0] * nx + g[1] * ny) * Me.sum(axis=1) for nx, ny in normals])
    assert np.abs(pr.element_block(e) @ lam - flux).max() < 1e-12 * kap


@pytest.mark.parametrize("n,p", [(5, 1), (6, 2), (4, 3)])
def test_global_matrix_spd_and_sparsity(n, p):
    kap = kappa_lognormal(n, 1.0, 11)
    S = hdg.Problem(n, p, kap).assemble()
    Sd = S.toarray()
    assert np.abs(Sd - Sd.T).max() < 1e-13 * np.abs(Sd).max()
    assert np.linalg.eigvalsh(Sd)[0] > 0
    assert np.diff(S.indptr).max() <= 7 * (p + 1)          # (4d - 1)(p + 1)^(d-1) in 2D


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_polynomial_solution_reproduced(k):
    """u in Q_k with K constant lies in the discrete spaces: Lambda, u_h and q_h are exact."""
    n, c = 4, 2.5
    prob = PolyProblem(k, c)
    pr = hdg.Problem(n, k, np.full(n * n, c))
    fq = pr.f_at_points(prob.f)
    lam_bd = pr.boundary_trace(prob.gD)
    lam = pr.solve_direct(pr.rhs(fq, lam_bd=lam_bd))
    uex = np.zeros(pr.N)
    for f in range(ms.n_faces(n)):
        mid, t = ms.face_midpoint_and_direction(n, f)
        pts = mid[None, :] + np.outer(qd.trace_nodes(k) * 0.5 / n, t)
        uex[f * (k + 1):(f + 1) * (k + 1)] = prob.u(pts[:, 0], pts[:, 1])
    assert np.linalg.norm(lam - uex) <= 1e-11 * np.linalg.norm(uex)
    Qs, Us = pr.reconstruct(lam, fq, lam_bd)
    eu, eq = pr.l2_errors(Qs, Us, prob.u, prob.q)
    assert eu < 1e-10 and eq < 1e-10


def test_linear_solution_any_degree_with_variable_kappa_elementwise_constant():
    """A linear u is not a solution for piecewise K (flux jumps); with K constant it is, for p = 1..3."""
    for p in (1, 2, 3):
        prob = LinearProblem(c=1.0)
        pr = hdg.Problem(3, p, np.ones(9))
        fq = pr.f_at_points(prob.f)
        lam_bd = pr.boundary_trace(prob.gD)
        lam = pr.solve_direct(pr.rhs(fq, lam_bd=lam_bd))
        Qs, Us = pr.reconstruct(lam, fq, lam_bd)
        assert max(pr.l2_errors(Qs, Us, prob.u, prob.q)) < 1e-12


def _tanh_errors(n, p):
    pr = hdg.Problem(n, p, TanhProblem.kappa, 1.0)
    fq = pr.f_at_points(TanhProblem.f)
    lam_bd = pr.boundary_trace(None)
    lam = pr.solve_direct(pr.rhs(fq, lam_bd=lam_bd))
    Qs, Us = pr.reconstruct(lam, fq, lam_bd)
    return np.array(pr.l2_errors(Qs, Us, TanhProblem.u, TanhProblem.q))


def test_table1_convergence_rates():
    """Rates of the paper's Table tab1 (p = 3..5, N up to 32) within 0.1."""
    rows = np.loadtxt(os.path.join(GOLDEN, "table1_rates.txt"))
    cache = {}
    for p, N, ru, rq in rows:
        p, N = int(p), int(N)
        for m in (N // 2, N):
            if (p, m) not in cache:
                cache[(p, m)] = _tanh_errors(m, p)
        rate = np.log2(cache[(p, N // 2)] / cache[(p, N)])
        assert abs(rate[0] - ru) < 0.1, (p, N, rate, ru)
        assert abs(rate[1] - rq) < 0.1, (p, N, rate, rq)


def test_sinsin_k1_rates():
    """Small case (K = 1, u = sin sin, k = 1): L2 rates of u_h and q_h -> k + 1 = 2."""
    errs = []
    for n in (4, 8, 16, 32):
        pr = hdg.Problem(n, 1, np.ones(n * n))
        fq = pr.f_at_points(SinSin.f)
        lam_bd = pr.boundary_trace(None)
        lam = pr.solve_direct(pr.rhs(fq, lam_bd=lam_bd))
        Qs, Us = pr.reconstruct(lam, fq, lam_bd)
        errs.append(pr.l2_errors(Qs, Us, SinSin.u, SinSin.q))
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])
    assert np.all(np.abs(rates[-1] - 2.0) < 0.15), rates


def test_manufactured_tanh_source_is_consistent():
    """f = -div(K grad u) of the tanh problem against a central finite difference."""
    x, y, d = 0.37, 0.61, 1e-4
    T = TanhProblem
    def flux(xx, yy):
        return T.kappa(xx, yy) * T.grad_u(xx, yy)
    div = ((flux(x + d, y)[0] - flux(x - d, y)[0]) + (flux(x, y + d)[1] - flux(x, y - d)[1])) / (2 * d)
    assert abs(-div - T.f(x, y)) < 1e-6
