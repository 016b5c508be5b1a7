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


def rel_err(x, xd):
    return np.linalg.norm(x - xd) / np.linalg.norm(xd)
