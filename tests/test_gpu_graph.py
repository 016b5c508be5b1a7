"""GPU: the preconditioner captured as a HIP graph and replayed.

The graph holds exactly the eager kernel sequence, so every replay must give
the eager result bit for bit.  The solve is repeated with eager work (applies,
synchronizations) between replays, and each repeat is compared.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1705_09907_amd as H  # noqa: E402
from oracle import hdg  # noqa: E402
from tolerances import SOLUTION_RTOL, solve_rtol, rel_err  # noqa: E402
from workloads import kappa_lognormal, normal_vector  # noqa: E402


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("n,k,sigma,opts,mode", [
    (24, 3, 1.0, dict(), "pcg"),
    (40, 3, 2.0, dict(inner={1: 2, 0: 2}), "fcg"),
    (32, 2, 2.0, dict(inner={0: 3}, precision="f32"), "fcg"),
    (16, 4, 1.0, dict(inner={2: 2, 0: 2}), "vcycle"),
    (24, 2, 1.0, dict(smoother="face", omega=0.7), "pcg"),
])
def test_graph_replays_equal_eager(n, k, sigma, opts, mode):
    print(f"case graph n={n} k={k} {opts} {mode}", flush=True)
    kap = kappa_lognormal(n, sigma, 12)
    pr = hdg.Problem(n, k, kap)
    b = torch.tensor(pr.rhs(np.ones((n * n, pr.ref.nq ** 2))), device="cuda")
    Se = H.Solver(n, k, kap, **opts)
    Sg = H.Solver(n, k, kap, graph=True, **opts)
    try:
        bh = host(b)
        Sc = pr.assemble().tocsr()
        xd = pr.solve_direct(bh, Sc)
        rtol = solve_rtol(Sc, bh, xd)
        xe, ite, rre, _ = Se.solve(b, rtol=rtol, maxit=400, mode=mode)
        xe = host(xe)
        z = torch.tensor(normal_vector(Sg.num_dofs(), 3), device="cuda")
        for rep in range(3):
            xg, itg, rrg, _ = Sg.solve(b, rtol=rtol, maxit=400, mode=mode)
            assert itg == ite and rrg == rre, (rep, itg, ite)
            assert np.array_equal(host(xg), xe), rep
            Sg.apply(k, z)                     # eager work between replays
            torch.cuda.synchronize()
        assert rel_err(xe, xd) <= SOLUTION_RTOL
    finally:
        Se.close()
        Sg.close()


@pytest.mark.parametrize("n,k,prec", [(64, 3, "f64"), (40, 4, "f32"), (2, 1, "f64")])
def test_autotuned_chain_shapes_give_identical_results(n, k, prec):
    """The autotuner only picks launch shapes: the solve is bit-identical to the
    default shapes, and every picked shape is a valid one."""
    print(f"case autotune n={n} k={k} {prec}", flush=True)
    kap = kappa_lognormal(n, 1.0, 5)
    pr = hdg.Problem(n, k, kap)
    b = torch.tensor(pr.rhs(np.ones((n * n, pr.ref.nq ** 2))), device="cuda")
    S0 = H.Solver(n, k, kap, precision=prec, inner={0: 2} if k >= 1 else None)
    S1 = H.Solver(n, k, kap, precision=prec, inner={0: 2} if k >= 1 else None, autotune=True)
    try:
        for p in range(k + 1):
            th, rm, ll = S1.chain_shape(p)
            assert th % 64 == 0 and 64 <= th <= 1024 and rm in (0, 1) and ll >= 0
            assert ((n - 1) // 2) * (p + 1) <= th * 8
        x0, it0, _, _ = S0.solve(b, rtol=1e-10, mode="fcg")
        x1, it1, _, _ = S1.solve(b, rtol=1e-10, mode="fcg")
        assert it0 == it1 and np.array_equal(host(x0), host(x1))
    finally:
        S0.close()
        S1.close()
