"""GPU: one full-multigrid pass (hdg_fmg, Sec. 7).

Bars: the FMG iterate matches the oracle's FMG to 1e-11 relative (same
smoother, omega and Chebyshev bounds; V and W schedules; 1 and 2 cycles per
level; n = 2 and k = 0 edges; 1e-10 with K-cycle levels, as for the K-cycle
itself); an exact solution in the range of the
prolongations from the coarsest level comes back to 1e-11; an FP32 cycle stays
within 1e-5 of the FP64 pass; cycles outside [1, 64] are rejected.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1705_09907_amd as H  # noqa: E402
from oracle import mg  # noqa: E402
from oracle import mesh as ms  # noqa: E402
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


def _pair(n, k, kap, smoother, cycle, precision="f64"):
    Ho = mg.Hierarchy(n, k, kap, smoother=smoother, omega=0.8, cycle=cycle)
    lmax = [Ho.lmax[L.name] for L in Ho.levels if L.kind == 'q' and not L.coarsest]
    S = H.Solver(n, k, kap, smoother=smoother, omega=Ho.omega, cheb_lmax=lmax, cycle=cycle, precision=precision)
    return Ho, S


@pytest.mark.parametrize("n,k,sigma,smoother,cycle", [
    (16, 1, None, "chain", "V"), (24, 3, 1.0, "chain", "V"), (32, 2, 2.0, "chain", "W"), (16, 0, 1.0, "chain", "V"),
    (2, 1, None, "chain", "V"), (10, 6, 1.0, "face", "V"), (24, 2, 1.0, "face", "W")])
@pytest.mark.parametrize("cycles", [1, 2])
def test_fmg_matches_oracle(n, k, sigma, smoother, cycle, cycles):
    print(f"case fmg {smoother} {cycle} n={n} k={k} cycles={cycles}", flush=True)
    kap = _kappa(n, sigma)
    Ho, S = _pair(n, k, kap, smoother, cycle)
    try:
        b = normal_vector(ms.n_trace_dofs(n, k), 5)
        xo = Ho.fmg(b, cycles=cycles)
        xg = S.fmg(dev(b), cycles=cycles)
        assert rel_inf(host(xg), xo) <= 1e-11, rel_inf(host(xg), xo)
    finally:
        S.close()


@pytest.mark.parametrize("n,k", [(16, 2), (24, 3)])
def test_fmg_reproduces_coarsest_range(n, k):
    print(f"case fmg range n={n} k={k}", flush=True)
    kap = kappa_lognormal(n, 1.0, 8)
    Ho, S = _pair(n, k, kap, "chain", "V")
    try:
        x = np.random.default_rng(n + k).standard_normal(Ho.levels[-1].A.shape[0])
        for lev in range(len(Ho.levels) - 2, -1, -1):
            x = Ho.levels[lev].Pmat @ x
        xg = host(S.fmg(dev(Ho.levels[0].A @ x)))
        assert np.linalg.norm(xg - x) <= 1e-11 * np.linalg.norm(x)
    finally:
        S.close()


def test_fmg_fp32_cycle_and_argument_checks():
    n, k = 24, 3
    print(f"case fmg f32 n={n} k={k}", flush=True)
    kap = kappa_lognormal(n, 1.0, 9)
    S64 = H.Solver(n, k, kap)
    S32 = H.Solver(n, k, kap, precision="f32")
    try:
        b = dev(normal_vector(ms.n_trace_dofs(n, k), 6))
        x64, x32 = host(S64.fmg(b)), host(S32.fmg(b))
        assert rel_inf(x32, x64) <= 1e-5
        for bad in (0, 65):
            with pytest.raises(H.HDGError):
                S64.fmg(b, cycles=bad)
    finally:
        S64.close()
        S32.close()


@pytest.mark.parametrize("n,k,inner,cycle", [(24, 3, {1: 2, 0: 2}, "V"), (16, 2, {0: 3}, "WH")])
def test_fmg_with_krylov_levels_matches_oracle(n, k, inner, cycle):
    """FMG on a hierarchy whose p = 1 / p = 0 corrections are K-cycle FCG steps."""
    print(f"case fmg kcycle {inner} {cycle} n={n} k={k}", flush=True)
    kap = kappa_lognormal(n, 1.0, 10)
    Ho = mg.Hierarchy(n, k, kap, omega=0.8, inner=inner, cycle=cycle)
    lmax = [Ho.lmax[L.name] for L in Ho.levels if L.kind == 'q' and not L.coarsest]
    S = H.Solver(n, k, kap, omega=Ho.omega, cheb_lmax=lmax, inner=inner, cycle=cycle)
    try:
        b = normal_vector(ms.n_trace_dofs(n, k), 7)
        xo = Ho.fmg(b)
        xg = host(S.fmg(dev(b)))
        assert rel_inf(xg, xo) <= 1e-10, rel_inf(xg, xo)
    finally:
        S.close()
