"""Misfit of the HDG volume solution as a differentiable function of the
per-element log-coefficients theta = log K (torch.autograd.Function).

Forward: a library handle for K = exp(theta) (the device set-up of every level;
a handle of the same mesh and options is reused through
hdg_update_coefficients), the right-hand side, one multigrid solve
S Lambda = b, reconstruction of U, and L = 1/2 |U - U_obs|^2.  Backward: the
adjoint right-hand side, one solve S mu = c with the same operator and
multigrid, and the element-local gradient kernel; every step runs in the
library's HIP kernels.
"""
import numpy as np
import torch

from . import Solver

# free handles per (n, k, solver options): a forward takes one (or makes one) and
# sets its coefficient; the handle goes back when its backward has run, or at
# once when no backward will run
_POOL = {}


def _key(n, k, opts):
    return (n, k, tuple(sorted((name, repr(v)) for name, v in opts.items())))


def _take(n, k, kappa, opts):
    free = _POOL.setdefault(_key(n, k, opts), [])
    if free:
        S = free.pop()
        S.update_coefficients(kappa)
        return S
    return Solver(n, k, kappa, **opts)


def _give(S, n, k, opts):
    _POOL.setdefault(_key(n, k, opts), []).append(S)


def release_handles():
    """Close every pooled handle (device memory of earlier misfit evaluations)."""
    for free in _POOL.values():
        for S in free:
            S.close()
    _POOL.clear()


class HDGMisfit(torch.autograd.Function):
    """L(theta) for an n x n mesh at degree k.

    theta: CPU or CUDA float64 tensor [n*n]; U_obs: CUDA float64 [n*n*(k+1)^2];
    f_qp: host array [n*n, nq*nq] of source values (nq = k + 2 Gauss-Legendre
    points per direction); gD_qp: host array [4n, nq] or None; solver_opts:
    keyword arguments of Solver (smoother, inner, precision, ...) plus rtol,
    mode and maxit of the two solves.
    """

    @staticmethod
    def forward(ctx, theta, U_obs, n, k, f_qp, gD_qp=None, solver_opts=None):
        opts = dict(solver_opts or {})
        rtol = opts.pop("rtol", 1e-12)
        mode = opts.pop("mode", "fcg" if opts.get("inner") else "pcg")
        maxit = opts.pop("maxit", 500)
        kappa = np.exp(theta.detach().double().cpu().numpy())
        S = _take(n, k, kappa, opts)
        try:
            b = S.assemble_rhs(f_qp, gD_qp)
            # a tolerance below the rounding floor of b - S Lambda ends at that floor
            lam, _, _, _ = S.solve(b, rtol=rtol, maxit=maxit, mode=mode, accept_floor=True)
            U = S.reconstruct(lam)
            c, L = S.adjoint_rhs(U, U_obs)
        except Exception:
            S.close()
            raise
        if ctx.needs_input_grad[0]:
            ctx.state = (S, lam, U, U_obs, c, rtol, maxit, mode, n, k, opts)
        else:
            _give(S, n, k, opts)
            ctx.state = None
        return torch.tensor(L, dtype=torch.float64, device=theta.device)

    @staticmethod
    def backward(ctx, gL):
        S, lam, U, U_obs, c, rtol, maxit, mode, n, k, opts = ctx.state
        ctx.state = None
        mu, _, _, _ = S.solve(c, rtol=rtol, maxit=maxit, mode=mode, accept_floor=True)
        g = S.misfit_gradient(lam, U, U_obs, mu)
        torch.cuda.current_stream().synchronize()
        _give(S, n, k, opts)
        grad_theta = (gL.to(g.device) * g)
        return grad_theta, None, None, None, None, None, None


def misfit(theta, U_obs, n, k, f_qp, gD_qp=None, **solver_opts):
    return HDGMisfit.apply(theta, U_obs, n, k, f_qp, gD_qp, solver_opts)
