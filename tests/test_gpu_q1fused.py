"""GPU: fused Q1 level visits (one launch for the pre-smoothing Chebyshev steps,
residual and full-weighting restriction of a level, one for the bilinear
prolongation and the post-smoothing steps; Sec. 7's Chebyshev smoother on the
Q1 levels) against the one-operation launches and the oracle.

Bars: the fused and the separate schedules give bitwise-identical cycle
iterates (same per-vertex fused multiply-adds in the same order), in FP64 and
FP32, for V, W and WH cycles, full multigrid and nu1, nu2 from 1 to 6 (7: the
separate launches, by design); three fused V-cycle iterates match the oracle's
to 1e-11 relative; at the n = 1024, k = 3 workload (tiles of 32 x 32 vertices
on the finest Q1 level) one cycle is bitwise equal too, and the fused solve
reaches the same iterate count and solution.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1705_09907_amd as H  # noqa: E402
from oracle import mg  # noqa: E402
from oracle import mesh as ms  # noqa: E402
from workloads import kappa_lognormal, normal_vector  # noqa: E402


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _cycles(S, b, ncyc):
    x = torch.zeros_like(b)
    out = []
    for _ in range(ncyc):
        S.vcycle(b, x)
        out.append(host(x).copy())
    return out


@pytest.mark.parametrize("n,k,sigma,nu1,nu2,cycle,prec,cmax", [
    (16, 1, 1.0, 2, 2, "V", "f64", 8), (24, 3, 2.0, 2, 2, "V", "f64", 8), (32, 2, 1.0, 1, 3, "W", "f64", 8),
    (64, 1, 2.0, 6, 6, "V", "f64", 8), (64, 2, 1.0, 2, 2, "WH", "f32", 8), (48, 2, 1.0, 5, 4, "V", "f32", 8),
    (40, 1, 1.0, 7, 2, "V", "f64", 8), (128, 1, 1.0, 2, 2, "V", "f64", 2000), (2, 1, 1.0, 2, 2, "V", "f64", 8),
    (6, 0, 1.0, 3, 1, "W", "f64", 8), (256, 1, 2.0, 2, 2, "V", "f64", 2000), (512, 0, 1.0, 2, 2, "V", "f64", 2000),
    (512, 1, 1.0, 2, 2, "V", "f32", 2000)])
def test_fused_q1_visits_are_bitwise_identical(n, k, sigma, nu1, nu2, cycle, prec, cmax):
    """coarse_max = 8 puts every Q1 level down to 2 x 2 or 3 x 3 elements under
    the fused kernels; m = 512 takes the 16 x 16 tiles (the full-size case below
    the 32 x 32 ones), smaller levels 8 x 8."""
    print(f"case q1 fused vs separate n={n} k={k} nu=({nu1},{nu2}) {cycle} {prec} cmax={cmax}", flush=True)
    kap = kappa_lognormal(n, sigma, 5)
    N = ms.n_trace_dofs(n, k)
    b = torch.tensor(normal_vector(N, 3), dtype=torch.float64, device="cuda")
    res = {}
    for sched in ("fused", "separate"):
        S = H.Solver(n, k, kap, nu1=nu1, nu2=nu2, cycle=cycle, precision=prec, coarse_max=cmax,
                     q1_schedule=sched)
        try:
            res[sched] = _cycles(S, b, 3)
            xf = S.fmg(b, cycles=1)
            res[sched].append(host(xf).copy())
        finally:
            S.close()
    for c, (a, s) in enumerate(zip(res["fused"], res["separate"])):
        assert np.array_equal(a, s), c


@pytest.mark.parametrize("n,k,sigma,nu1,nu2", [(24, 3, 1.0, 2, 2), (32, 1, 2.0, 3, 3), (16, 2, 1.0, 1, 2)])
def test_fused_q1_cycle_matches_oracle(n, k, sigma, nu1, nu2):
    """coarse_max = 8: the fused visits on every Q1 level above 2 x 2 or 3 x 3."""
    print(f"case q1 fused vs oracle n={n} k={k}", flush=True)
    kap = kappa_lognormal(n, sigma, 12)
    Ho = mg.Hierarchy(n, k, kap, omega=0.8, nu1=nu1, nu2=nu2, coarse_max=8)
    lmax = [Ho.lmax[L.name] for L in Ho.levels if L.kind == 'q' and not L.coarsest]
    S = H.Solver(n, k, kap, omega=Ho.omega, cheb_lmax=lmax, nu1=nu1, nu2=nu2, coarse_max=8, q1_schedule="fused")
    assert S.num_hlevels() == len([L for L in Ho.levels if L.kind == 'q'])
    try:
        N = ms.n_trace_dofs(n, k)
        b = normal_vector(N, 11)
        xo = np.zeros(N)
        xg = torch.zeros(N, dtype=torch.float64, device="cuda")
        bg = torch.tensor(b, device="cuda")
        for c in range(3):
            xo = Ho.vcycle(b, xo)
            S.vcycle(bg, xg)
            err = np.abs(host(xg) - xo).max() / np.abs(xo).max()
            assert err <= 1e-11, (c, err)
    finally:
        S.close()


def test_fused_q1_full_size_workload():
    """n = 1024, k = 3, lognormal sigma = 2 coefficient (the benchmark's default
    workload): one cycle bitwise equal between the schedules; the fused solve
    converges in the same number of iterations to the same solution."""
    n, k = 1024, 3
    print(f"case q1 fused full size n={n} k={k}", flush=True)
    kap = kappa_lognormal(n, 2.0, 7)
    N = ms.n_trace_dofs(n, k)
    b = torch.tensor(normal_vector(N, 1), dtype=torch.float64, device="cuda")
    out = {}
    for sched in ("fused", "separate"):
        S = H.Solver(n, k, kap, q1_schedule=sched, inner={2: 3, 1: 3, 0: 8})
        try:
            x = torch.zeros_like(b)
            S.vcycle(b, x)
            xs, it, rr, _ = S.solve(b, rtol=1e-10, maxit=60, mode="fcg")
            out[sched] = (host(x).copy(), it, host(xs).copy())
        finally:
            S.close()
    assert np.array_equal(out["fused"][0], out["separate"][0])
    assert out["fused"][1] == out["separate"][1]
    assert np.array_equal(out["fused"][2], out["separate"][2])
