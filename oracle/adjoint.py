"""Misfit and its gradient with respect to per-element log-coefficients.

Test infrastructure only (see oracle/__init__.py).

The paper solves forward problems only; this module adds the gradient of a
data misfit through the same discretisation, by the adjoint (Lagrangian)
method, using nothing but the paper's local solver and condensed system:

  theta_K = log K_K (one value per element), so the local matrix of eq.
  static_1 is A_K = exp(-theta_K) A0 and dA_K / dtheta_K = -A_K;
  [Q; U]_K = Abb_K^{-1} ([0; F_K] - [C; E] Lambda_K)           (eq. shur0)
  S(theta) Lambda = b(theta)                                    (eq. shur1)
  L(theta) = 1/2 sum_K |U_K - U_obs,K|^2   (U_K: the (p+1)^2 nodal values of
                                            the element's volume solution)

With rho(theta, Lambda) = b - S Lambda = sum_K R_K^T ([C^T, -E^T] [Q; U]_K
- tau M Lambda_K) and the Lagrangian L + mu^T rho:
  adjoint   S mu = (dU/dLambda)^T r,  r = U - U_obs,  where
            (dU/dLambda)^T r = -sum_K R_K^T [C^T, E^T] Abb_K^{-T} [0; r_K]
  gradient  dL/dtheta_K = w_K^T [A_K Q_K; 0],
            Abb_K^T w_K = [0; r_K] + [C; -E] mu_K,
because d[Q; U]_K / dtheta_K at fixed Lambda = Abb_K^{-1} [A_K Q_K; 0].
Every local solve below is a plain dense solve with Abb_K or its transpose.

Pinned by central finite differences of L through the direct solver
(tests/test_oracle_adjoint.py).
"""
import numpy as np

from .hdg import Problem, local_matrices, local_system, load_vector


class Misfit:
    """L(theta) for an n x n mesh at degree k with source values f_qp at the
    volume Gauss-Legendre points and boundary traces lam_bd (Problem.boundary_trace)."""

    def __init__(self, n, k, f_qp, U_obs, lam_bd=None, tau=1.0):
        self.n, self.k, self.tau = n, k, tau
        self.f_qp = np.asarray(f_qp, dtype=np.float64)
        self.U_obs = np.asarray(U_obs, dtype=np.float64).reshape(n * n, (k + 1) ** 2)
        self.lam_bd = lam_bd

    def problem(self, theta):
        return Problem(self.n, self.k, np.exp(np.asarray(theta, dtype=np.float64)), self.tau)

    def _lam_bd(self, pr):
        return np.zeros(4 * self.n * pr.P) if self.lam_bd is None else self.lam_bd

    def forward(self, theta):
        """Solve for Lambda directly, reconstruct U and Q; returns (L, Lambda, Q, U)."""
        pr = self.problem(theta)
        lam_bd = self._lam_bd(pr)
        lam = pr.solve_direct(pr.rhs(self.f_qp, lam_bd=lam_bd))
        Qs, Us = pr.reconstruct(lam, self.f_qp, lam_bd)
        return 0.5 * float(np.sum((Us - self.U_obs) ** 2)), lam, Qs, Us

    def value(self, theta):
        return self.forward(theta)[0]

    def adjoint_rhs(self, theta, Us):
        """(dU/dLambda)^T (U - U_obs) on interior trace DoFs."""
        pr = self.problem(theta)
        n2 = pr.P ** 2
        c = np.zeros(pr.N)
        for e in range(self.n * self.n):
            A, B, C, D, E, M = pr.element_mats(e)
            r = Us[e] - self.U_obs[e]
            a = np.linalg.solve(local_system(A, B, D).T, np.concatenate([np.zeros(2 * n2), r]))
            contrib = -(C.T @ a[:2 * n2] + E.T @ a[2 * n2:])
            d = pr.dofs[e]
            m = d >= 0
            np.add.at(c, d[m], contrib[m])
        return c

    def gradient(self, theta):
        """dL/dtheta by one forward and one adjoint solve (both direct); returns (L, grad, mu)."""
        Lval, lam, Qs, Us = self.forward(theta)
        pr = self.problem(theta)
        S = pr.assemble()
        mu = pr.solve_direct(self.adjoint_rhs(theta, Us), S)
        n2 = pr.P ** 2
        g = np.zeros(self.n * self.n)
        for e in range(self.n * self.n):
            A, B, C, D, E, M = pr.element_mats(e)
            d = pr.dofs[e]
            mu_e = np.where(d >= 0, mu[np.maximum(d, 0)], 0.0)   # boundary traces are data
            r = Us[e] - self.U_obs[e]
            rhs = np.concatenate([np.zeros(2 * n2), r]) + np.concatenate([C @ mu_e, -E @ mu_e])
            w = np.linalg.solve(local_system(A, B, D).T, rhs)
            g[e] = w[:2 * n2] @ (A @ Qs[e])
        return Lval, g, mu
