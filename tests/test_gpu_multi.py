"""GPU: trace apply for many right-hand sides at once (Y = S X, X [N, nrhs]).

Bars: FP64 against the oracle's assembled S times X, 1e-12 relative (max norm),
on every level, ragged tails, nrhs a multiple of 64 (whole wavefronts per face,
one or several 64-column chunks) or not; each column equals
the single-vector apply to 1e-14 (same summation order); FP32 and bfloat16
blocks obey the row-wise rounding bound of the reduced-precision apply, with
both the vector kernel and the matrix-core kernel; the full-size batch (n = 512,
k = 5, 64 right-hand sides) on sampled faces, both kernels.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1705_09907_amd as H  # noqa: E402
from oracle import hdg, mg, mesh as ms  # noqa: E402
from workloads import kappa_lognormal  # noqa: E402

U32 = 2.0 ** -24


def dev(a, dtype=torch.float64):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_inf(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("n,k,R", [(2, 1, 3), (16, 2, 64), (24, 3, 100), (19, 5, 1), (13, 8, 65), (16, 0, 7),
                                   (2, 1, 64), (13, 8, 128), (19, 5, 192), (17, 0, 64)])
def test_multi_apply_every_level_fp64(n, k, R):
    print(f"case multi apply n={n} k={k} R={R}", flush=True)
    kap = kappa_lognormal(n, 1.0, 3)
    Ho = mg.Hierarchy(n, k, kap, smoother="face", omega=0.7)
    S = H.Solver(n, k, kap)
    rng = np.random.default_rng(n + k + R)
    try:
        for L in Ho.levels:
            if L.kind != 'p':
                break
            p = L.p
            N = ms.n_trace_dofs(n, p)
            X = rng.standard_normal((N, R))
            Y = host(S.apply_multi(p, dev(X)))
            assert rel_inf(Y, L.A @ X) <= 1e-12, p
            for col in (0, R - 1):
                y1 = host(S.apply(p, dev(np.ascontiguousarray(X[:, col]))))
                assert np.abs(Y[:, col] - y1).max() <= 1e-14 * np.abs(y1).max()
    finally:
        S.close()


@pytest.mark.parametrize("kernel", ["vector", "matrix"])
@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("n,k,R", [(24, 3, 64), (24, 3, 128), (24, 3, 40), (19, 8, 64), (17, 0, 70), (9, 5, 3)])
def test_multi_apply_reduced_precision_bound(kernel, prec, n, k, R):
    print(f"case multi apply {kernel} {prec} n={n} k={k} R={R}", flush=True)
    kap = kappa_lognormal(n, 2.0, 5)
    Ho = mg.Hierarchy(n, k, kap, smoother="face", omega=0.7)
    S = H.Solver(n, k, kap, precision=prec, multi_kernel=kernel)
    rng = np.random.default_rng(9)
    try:
        for L in Ho.levels:
            if L.kind != 'p':
                break
            p = L.p
            N = ms.n_trace_dofs(n, p)
            X = rng.standard_normal((N, R)).astype(np.float32)
            Y = host(S.apply_multi(p, dev(X, torch.float32))).astype(np.float64)
            Xh = X.astype(np.float64)
            um = U32 if (prec == "f32" or p == k) else 2.0 ** -8
            lim = (um + (7 * (p + 1) + 2) * U32) * 1.01 * (abs(L.A) @ np.abs(Xh))
            assert np.all(np.abs(Y - L.A @ Xh) <= lim), p
    finally:
        S.close()


@pytest.mark.parametrize("kernel", ["vector", "matrix"])
def test_full_size_batch_sampled(kernel):
    """n = 512, k = 5, 64 right-hand sides, FP32 blocks: sampled faces against
    oracle rows under the rounding bound."""
    n, k, R = 512, 5, 64
    print(f"case full-size batch apply n=512 k=5 R=64 {kernel}", flush=True)
    kap = kappa_lognormal(n, 1.0, 4)
    S = H.Solver(n, k, kap, precision="f32", multi_kernel=kernel)
    P = k + 1
    try:
        N = S.num_dofs()
        gen = torch.Generator(device="cuda").manual_seed(4)
        X = torch.randn(N, R, device="cuda", dtype=torch.float32, generator=gen)
        Y = S.apply_multi(k, X)
        nf = ms.n_faces(n)
        nv = n * (n - 1)
        rng = np.random.default_rng(5)
        faces = sorted(set([0, 1, n - 2, nv - 1, nv, nf - 1, nf - 17, (nf // 16) * 16 - 1]
                           + list(rng.integers(0, nf, 40))))
        Xh = host(X).astype(np.float64)
        Yh = host(Y).astype(np.float64)
        cache = {}
        for f in faces:
            lo, hi, o = ms.face_elements(n, f)
            llo, lhi = ms.face_local_index(n, f)
            blocks = {}
            for e, lf in ((lo, llo), (hi, lhi)):
                if e not in cache:
                    cache[e] = hdg.condensed_block(*hdg.local_matrices(
                        hdg.RefOps(k), 1.0 / n, 1.0, np.full((k + 2) ** 2, 1.0 / kap[e])), 1.0)
                i, j = e % n, e // n
                for g, gf in enumerate(ms.element_faces(n, i, j)):
                    if gf >= 0:
                        blk = cache[e][lf * P:(lf + 1) * P, g * P:(g + 1) * P]
                        blocks[gf] = blocks.get(gf, 0) + blk
            exact = np.zeros((P, R))
            scale = np.zeros((P, R))
            for gf, blk in blocks.items():
                xg = Xh[gf * P:(gf + 1) * P]
                exact += blk @ xg
                scale += np.abs(blk) @ np.abs(xg)
            lim = (U32 + (7 * P + 2) * U32) * 1.01 * scale
            assert np.all(np.abs(Yh[f * P:(f + 1) * P] - exact) <= lim), f
    finally:
        S.close()


@pytest.mark.parametrize("meshes", [
    [(16, 2), (24, 3), (7, 1), (40, 4), (2, 2), (33, 0)],          # P <= 5 instance
    [(12, 6), (9, 2), (20, 8), (5, 4)],                             # P <= 9 instance
])
def test_batch_of_meshes_one_launch_bitwise(meshes):
    """Many meshes of different sizes and degrees in one launch: every mesh's
    result is bit-identical to its own apply, and matches the oracle."""
    print(f"case batch {meshes}", flush=True)
    solvers, xs, refs = [], [], []
    try:
        for i, (n, k) in enumerate(meshes):
            kap = kappa_lognormal(n, 1.0, 40 + i)
            S = H.Solver(n, k, kap)
            x = dev(np.random.default_rng(i).standard_normal(S.num_dofs()))
            solvers.append(S)
            xs.append(x)
            refs.append(host(S.apply(k, x)))
        ys = H.apply_batch(solvers, xs)
        for (n, k), y, r, x, i in zip(meshes, ys, refs, xs, range(len(meshes))):
            assert np.array_equal(host(y), r), (n, k)
        # coarse levels too
        lv = [max(0, s.k - 1) for s in solvers]
        ys = H.apply_batch(solvers, [torch.ones(s.num_dofs(l), dtype=torch.float64, device="cuda")
                                     for s, l in zip(solvers, lv)], levels=lv)
        for s, l, y in zip(solvers, lv, ys):
            one = torch.ones(s.num_dofs(l), dtype=torch.float64, device="cuda")
            assert np.array_equal(host(y), host(s.apply(l, one)))
        n, k = meshes[0]
        Ho = mg.Hierarchy(n, k, kappa_lognormal(n, 1.0, 40), smoother="face", omega=0.7)
        assert rel_inf(host(H.apply_batch(solvers[:1], xs[:1])[0]), Ho.levels[0].A @ host(xs[0])) <= 1e-12
    finally:
        for s in solvers:
            s.close()


@pytest.mark.parametrize("meshes", [[(16, 1, "f32"), (24, 3, "bf16"), (40, 4, "f32"), (7, 8, "bf16"), (2, 1, "f32")],
                                    [(64, 2, "f32"), (96, 5, "f32"), (33, 3, "bf16")]])
def test_batch_of_meshes_reduced_precision_bitwise(meshes):
    """The many-mesh launch in the handles' reduced cycle precision (FP32 or
    bfloat16 blocks, FP32 vectors; handles of both kinds in one launch): every
    mesh's result is bit-identical to its own hdg_apply_trace_operator_lp, on the
    finest and a coarser level."""
    print(f"case batch lp {meshes}", flush=True)
    solvers, xs = [], []
    try:
        for i, (n, k, prec) in enumerate(meshes):
            S = H.Solver(n, k, kappa_lognormal(n, 1.0, 50 + i), precision=prec)
            solvers.append(S)
            xs.append(torch.tensor(np.random.default_rng(i).standard_normal(S.num_dofs()), dtype=torch.float32,
                                   device="cuda"))
        ys = H.apply_batch(solvers, xs, lp=True)
        for S, x, y, m in zip(solvers, xs, ys, meshes):
            assert np.array_equal(host(y), host(S.apply_lp(S.k, x))), m
        lv = [max(0, s.k - 1) for s in solvers]
        xc = [torch.tensor(np.random.default_rng(10 + i).standard_normal(s.num_dofs(l)), dtype=torch.float32,
                           device="cuda") for i, (s, l) in enumerate(zip(solvers, lv))]
        ys = H.apply_batch(solvers, xc, levels=lv, lp=True)
        for S, l, x, y, m in zip(solvers, lv, xc, ys, meshes):
            assert np.array_equal(host(y), host(S.apply_lp(l, x))), (m, l)
    finally:
        for s in solvers:
            s.close()
