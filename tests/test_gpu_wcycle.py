"""GPU: the W schedule of the multigrid cycle (Sec. 7 reports W- beside V-cycles),
and the hybrid WH (W on the Q1 levels, V on the p-levels).

Bars: three W- (and WH-) cycle iterates from zero match the oracle's to 1e-11
relative (same smoother, omega and Chebyshev bounds; edge meshes n = 2, k = 0);
W-cycle PCG and stationary W-cycles reach rtol = max(1e-12, 4 x rounding floor)
on the true residual and match the direct solve to 1e-10, in no more iterations
than the V-cycle; the multi-column solve with the W
or WH schedule matches the direct solve and the single-vector solve per column.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1705_09907_amd as H  # noqa: E402
from oracle import hdg, mg  # noqa: E402
from oracle import mesh as ms  # noqa: E402
from tolerances import SOLUTION_RTOL, solve_rtol, rel_err  # noqa: E402
from workloads import kappa_const, kappa_lognormal, normal_vector  # noqa: E402


def _kappa(n, sigma, seed=12):
    return kappa_const(n) if sigma is None else kappa_lognormal(n, sigma, seed)


def dev(a):
    return torch.tensor(np.asarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_inf(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("n,k,sigma", [(16, 1, None), (24, 3, 1.0), (32, 2, 2.0), (16, 0, 1.0), (2, 1, None),
                                       (10, 6, 1.0)])
@pytest.mark.parametrize("smoother,cycle", [("chain", "W"), ("face", "W"), ("chain", "WH")])
def test_wcycle_iterates(n, k, sigma, smoother, cycle):
    print(f"case wcycle {cycle} {smoother} n={n} k={k}", flush=True)
    kap = _kappa(n, sigma)
    Ho = mg.Hierarchy(n, k, kap, smoother=smoother, omega=0.8, cycle=cycle)
    lmax = [Ho.lmax[L.name] for L in Ho.levels if L.kind == 'q' and not L.coarsest]
    S = H.Solver(n, k, kap, smoother=smoother, omega=Ho.omega, cheb_lmax=lmax, cycle=cycle)
    try:
        N = ms.n_trace_dofs(n, k)
        b = normal_vector(N, 11)
        xo = np.zeros(N)
        xg = torch.zeros(N, dtype=torch.float64, device="cuda")
        bg = dev(b)
        for cyc in range(3):
            xo = Ho.vcycle(b, xo)
            S.vcycle(bg, xg)
            assert rel_inf(host(xg), xo) <= 1e-11, (cyc, rel_inf(host(xg), xo))
    finally:
        S.close()


@pytest.mark.parametrize("n,k,sigma", [(16, 1, None), (24, 3, 1.0), (32, 2, 2.0)])
@pytest.mark.parametrize("mode", ["pcg", "vcycle"])
def test_wcycle_solve_matches_direct(n, k, sigma, mode):
    print(f"case wcycle solve {mode} n={n} k={k}", flush=True)
    kap = _kappa(n, sigma)
    pr = hdg.Problem(n, k, kap)
    b = pr.rhs(np.ones((n * n, pr.ref.nq ** 2)))
    Sc = pr.assemble().tocsr()
    xd = pr.solve_direct(b, Sc)
    rtol = solve_rtol(Sc, b, xd)
    its = {}
    for cyc in ("V", "W"):
        S = H.Solver(n, k, kap, cycle=cyc)
        try:
            x, it, rr, hist = S.solve(dev(b), rtol=rtol, maxit=400, mode=mode)
        finally:
            S.close()
        assert rr <= rtol and hist[-1] <= rtol * np.linalg.norm(b), cyc
        assert rel_err(host(x), xd) <= SOLUTION_RTOL, cyc
        its[cyc] = it
    assert its["W"] <= its["V"], its


@pytest.mark.parametrize("n,k,sigma,R,prec,cycle", [(24, 3, 1.0, 5, "f64", "W"), (16, 2, 2.0, 9, "f32", "W"),
                                                    (2, 1, 1.0, 3, "f64", "W"), (32, 2, 2.0, 64, "f32", "WH"),
                                                    (24, 3, 1.0, 7, "f64", "WH")])
def test_wcycle_multi_solve(n, k, sigma, R, prec, cycle):
    print(f"case wcycle multi {cycle} n={n} k={k} R={R} {prec}", flush=True)
    kap = kappa_lognormal(n, sigma, 12)
    pr = hdg.Problem(n, k, kap)
    rng = np.random.default_rng(n + R)
    Bh = np.stack([pr.rhs(1.0 + rng.standard_normal((n * n, pr.ref.nq ** 2))) for _ in range(R)], axis=1)
    S = H.Solver(n, k, kap, precision=prec, cycle=cycle)
    try:
        A = pr.assemble().tocsr()
        XD = [pr.solve_direct(Bh[:, r], A) for r in range(R)]
        rtol = max(solve_rtol(A, Bh[:, r], XD[r]) for r in range(R))
        B = torch.tensor(Bh, device="cuda")
        X, its, rr = S.solve_multi(B, rtol=rtol, maxit=400)
        Xh = host(X)
        for r in range(R):
            assert rel_err(Xh[:, r], XD[r]) <= SOLUTION_RTOL, r
            assert rr[r] <= rtol, r
        for r in (0, R - 1):
            xs, _, _, _ = S.solve(B[:, r].contiguous(), rtol=rtol, maxit=400)
            assert rel_err(Xh[:, r], host(xs)) <= SOLUTION_RTOL
    finally:
        S.close()
