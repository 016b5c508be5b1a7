"""Solve tolerances shared by the GPU parity tests.

A solve is checked on its true residual b - S x and against the oracle's
direct solve.  The requested tolerance is rtol = max(1e-12, 4 floor), where
floor = u || |S| |x_direct| ||_2 / ||b||_2 (u = 2^-53) is the size below which
no FP64 vector's computed residual can go (rounding of S x itself, measured on
the oracle's assembled matrix): the solve is asked for 1e-12 wherever FP64 can
show it, and for four times the floor where the floor is higher (smooth right-
hand sides with high coefficient contrast).  Solutions must then agree with the
direct solve to SOLUTION_RTOL.
"""
import numpy as np

SOLUTION_RTOL = 1e-10    # ||x - x_direct|| / ||x_direct||
RESID_RTOL = 1e-12       # requested ||b - S x|| / ||b|| where the floor allows


def residual_floor(S, b, x):
    """u || |S| |x| ||_2 / ||b||_2 for the oracle's assembled CSR matrix S."""
    return 2.0 ** -53 * np.linalg.norm(abs(S) @ np.abs(x)) / np.linalg.norm(b)


def solve_rtol(S, b, x):
    return max(RESID_RTOL, 4.0 * residual_floor(S, b, x))


def residual_agreement_bound(S, b, x):
    """Largest ||r1 - r2||_2 between two FP64 evaluations of b - S x that sum in
    different orders, with S's entries themselves rounded independently on the
    two sides: per row each evaluation is within gamma_m (|b| + |S| |x|) of the
    exact value, gamma_m = m u / (1 - m u), m = nonzeros of the row + 2 (the
    standard bound for a rounded inner product, e.g. Higham, Accuracy and
    Stability of Numerical Algorithms, Sec. 3.1)."""
    u = 2.0 ** -53
    m = int(np.diff(S.indptr).max()) + 2
    gamma = m * u / (1 - m * u)
    return 2.0 * gamma * np.linalg.norm(np.abs(b) + abs(S) @ np.abs(x))


def true_residual_ok(S, b, x, relres_gpu):
    """The oracle's b - S x of the GPU's x agrees with the residual the GPU
    reported for it, to the rounding of the two evaluations."""
    r = np.linalg.norm(b - S @ x)
    return r <= relres_gpu * np.linalg.norm(b) + residual_agreement_bound(S, b, x), r


def rel_err(x, xd):
    return np.linalg.norm(x - xd) / np.linalg.norm(xd)
