"""GPU: the device set-up (element blocks of every level, face slabs, smoother
factors, Q1 hierarchy) against the host set-up and the host element blocks.

Bars: the stored FP64 face blocks equal the blocks assembled from the host's
element blocks (hdg_element_block_host, Cholesky of the local U system) to
1e-13 relative (max norm over the face's 7 blocks, relative to the largest
entry), on every level, Galerkin and rediscretized coarse levels, coefficients
over e^{+-8}; reduced-precision levels to the rounding of their storage; a
device-built handle and a host-built handle give the same applies (1e-13) and
V-cycle iterates (1e-11); a coefficient update on an existing handle gives the
bitwise result of a fresh handle with that coefficient, and its solve matches
the oracle's direct solve.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1705_09907_amd as H  # noqa: E402
from oracle import hdg, mesh as ms  # noqa: E402
from tolerances import SOLUTION_RTOL, solve_rtol, rel_err  # noqa: E402
from workloads import kappa_lognormal, normal_vector  # noqa: E402


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _face_blocks_from_host(n, k, p, kap, f, coarse):
    """The 7 blocks of face f from hdg_element_block_host (host set-up)."""
    P = p + 1
    lo, hi, _ = ms.face_elements(n, f)
    llo, lhi = ms.face_local_index(n, f)
    Klo = H.element_block_host(n, k, p, kap[lo], coarse=coarse)
    Khi = H.element_block_host(n, k, p, kap[hi], coarse=coarse)
    out = np.zeros((7, P, P))
    out[0] = Klo[llo * P:(llo + 1) * P, llo * P:(llo + 1) * P] + Khi[lhi * P:(lhi + 1) * P, lhi * P:(lhi + 1) * P]
    for base, K, lf, e in ((1, Klo, llo, lo), (4, Khi, lhi, hi)):
        i, j = e % n, e // n
        faces = ms.element_faces(n, i, j)
        others = [g for g in range(4) if g != lf]
        for s, g in enumerate(others):
            if faces[g] >= 0:
                out[base + s] = K[lf * P:(lf + 1) * P, g * P:(g + 1) * P]
    return out


def _sample_faces(n):
    nv = n * (n - 1)
    nf = 2 * nv
    rng = np.random.default_rng(n)
    return sorted(set([0, n - 2, nv - 1, nv, nf - 1, nf // 2] + list(rng.integers(0, nf, 12))))


@pytest.mark.parametrize("n,k,sigma,coarse", [(12, 3, 4.0, "galerkin"), (9, 1, 1.0, "galerkin"),
                                               (10, 5, 2.0, "rediscretize"), (7, 8, 1.0, "galerkin"),
                                               (16, 0, 2.0, "galerkin")])
def test_device_face_blocks_match_host_blocks(n, k, sigma, coarse):
    print(f"case device blocks n={n} k={k} sigma={sigma} {coarse}", flush=True)
    kap = kappa_lognormal(n, sigma, 21)
    S = H.Solver(n, k, kap, coarse=coarse, smoother="face", omega=0.7)
    try:
        worst = 0.0
        for p in range(k, -1, -1):
            for f in _sample_faces(n):
                dev = S.face_blocks(p, f)
                ref = _face_blocks_from_host(n, k, p, kap, f, coarse)
                d = np.abs(dev - ref).max() / np.abs(ref).max()
                worst = max(worst, d)
                assert d <= 1e-13, (p, f, d)
        print(f"worst face-block difference {worst:.2e}", flush=True)
    finally:
        S.close()


@pytest.mark.parametrize("prec,um", [("f32", 2.0 ** -24), ("bf16", 2.0 ** -8)])
def test_reduced_precision_blocks_round_the_device_blocks(prec, um):
    n, k = 10, 3
    kap = kappa_lognormal(n, 2.0, 3)
    S = H.Solver(n, k, kap, precision=prec)
    try:
        for p in range(k, -1, -1):
            for f in _sample_faces(n):
                dev = S.face_blocks(p, f)
                ref = _face_blocks_from_host(n, k, p, kap, f, "galerkin")
                # the finest level keeps an FP64 copy; coarse levels are stored in the cycle precision
                tol = 1e-13 if p == k else 1.01 * um
                assert np.all(np.abs(dev - ref) <= tol * np.abs(ref) + 1e-13 * np.abs(ref).max()), (p, f)
    finally:
        S.close()


@pytest.mark.parametrize("n,k,sigma,smoother", [(24, 3, 2.0, "chain"), (16, 2, 1.0, "face"), (33, 4, 1.0, "chain"),
                                                (8, 1, 3.0, "chain"), (64, 2, 1.0, "chain"), (128, 1, 2.0, "face")])
def test_device_setup_matches_host_setup(n, k, sigma, smoother):
    print(f"case device vs host setup n={n} k={k} {smoother}", flush=True)
    kap = kappa_lognormal(n, sigma, 5)
    Sd = H.Solver(n, k, kap, smoother=smoother, omega=0.7 if smoother == "face" else None)
    Sh = H.Solver(n, k, kap, smoother=smoother, omega=0.7 if smoother == "face" else None, host_setup=True)
    try:
        om_d, lm_d = Sd.params()
        om_h, lm_h = Sh.params()
        # lambda_max of the Q1 levels: 30 Lanczos steps on the device against the host's
        assert len(lm_d) == len(lm_h) and np.allclose(lm_d, lm_h, rtol=1e-8), (lm_d, lm_h)
        for p in range(k, -1, -1):
            x = torch.tensor(normal_vector(Sd.num_dofs(p), 3 + p), device="cuda")
            yd, yh = host(Sd.apply(p, x)), host(Sh.apply(p, x))
            assert np.abs(yd - yh).max() <= 1e-13 * np.abs(yh).max(), p
        b = torch.tensor(normal_vector(Sd.num_dofs(), 9), device="cuda")
        xd = torch.zeros_like(b)
        xh = torch.zeros_like(b)
        for cyc in range(3):
            Sd.vcycle(b, xd)
            Sh.vcycle(b, xh)
            assert np.abs(host(xd) - host(xh)).max() <= 1e-11 * np.abs(host(xh)).max(), cyc
    finally:
        Sd.close()
        Sh.close()


@pytest.mark.parametrize("smoother,precision", [("chain", "f64"), ("face", "f64"), ("chain", "f32")])
def test_coefficient_update_equals_fresh_handle(smoother, precision):
    n, k = 20, 3
    kap1 = kappa_lognormal(n, 1.0, 1)
    kap2 = kappa_lognormal(n, 2.0, 2)
    print(f"case update {smoother} {precision}", flush=True)
    Su = H.Solver(n, k, kap1, smoother=smoother, precision=precision)
    Sf = H.Solver(n, k, kap2, smoother=smoother, precision=precision)
    try:
        Su.update_coefficients(kap2)
        om_u, lm_u = Su.params()
        om_f, lm_f = Sf.params()
        assert np.array_equal(om_u, om_f) and np.array_equal(lm_u, lm_f)
        for p in range(k, -1, -1):
            for f in _sample_faces(n):
                assert np.array_equal(Su.face_blocks(p, f), Sf.face_blocks(p, f)), (p, f)
        b = torch.tensor(normal_vector(Su.num_dofs(), 4), device="cuda")
        xu, xf = torch.zeros_like(b), torch.zeros_like(b)
        for _ in range(2):
            Su.vcycle(b, xu)
            Sf.vcycle(b, xf)
        assert torch.equal(xu, xf)
        # the right-hand side of the new coefficient, and a solve to the oracle's solution
        pr = hdg.Problem(n, k, kap2)
        bo = pr.rhs(np.ones((n * n, pr.ref.nq ** 2)))
        bg = Su.assemble_rhs(np.ones((n * n, pr.ref.nq ** 2)))
        assert np.abs(host(bg) - bo).max() <= 1e-12 * np.abs(bo).max()
        Sc = pr.assemble().tocsr()
        xd = pr.solve_direct(bo, Sc)
        rtol = solve_rtol(Sc, bo, xd)
        x, it, rr, _ = Su.solve(bg, rtol=rtol, maxit=400, mode="pcg")
        assert rr <= rtol and rel_err(host(x), xd) <= SOLUTION_RTOL
    finally:
        Su.close()
        Sf.close()


def test_update_rejects_bad_coefficients():
    n = 6
    S = H.Solver(n, 2, np.ones(n * n))
    try:
        bad = np.ones(n * n)
        bad[3] = -1.0
        with pytest.raises(H.HDGError) as ei:
            S.update_coefficients(bad)
        assert ei.value.status == -1
    finally:
        S.close()
    Sh = H.Solver(n, 2, np.ones(n * n), host_setup=True)
    try:
        with pytest.raises(H.HDGError) as ei:
            Sh.update_coefficients(np.ones(n * n))
        assert ei.value.status == -6
    finally:
        Sh.close()
