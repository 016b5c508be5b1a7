"""GPU: the allocation-free many-mesh apply (hdg_apply_trace_operator_batch_noalloc)
against the allocating one (hdg_apply_trace_operator_batch), through the C ABI.

Bar: bit-identical outputs (same kernel, same order of operations) on two calls
in a row, the second with fewer and smaller meshes than the first, so stale
descriptors of the first call in the shared device table would show; a count
above HDG_BATCH_NOALLOC_MAX is rejected before any launch.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1705_09907_amd as H  # noqa: E402
from workloads import kappa_lognormal, normal_vector  # noqa: E402

NOALLOC_MAX = 256


def _call(fn, solvers, xs, ys):
    cnt = len(solvers)
    hs = (ctypes.c_void_p * cnt)(*[s._h.value for s in solvers])
    ps = (ctypes.c_int32 * cnt)(*[s.k for s in solvers])
    xv = (ctypes.c_void_p * cnt)(*[x.data_ptr() for x in xs])
    yv = (ctypes.c_void_p * cnt)(*[y.data_ptr() for y in ys])
    return fn(cnt, hs, ps, xv, yv)


def _batch(spec, seed0):
    solvers = [H.Solver(n, k, kappa_lognormal(n, 1.0, seed0 + i)) for i, (n, k) in enumerate(spec)]
    xs = [torch.tensor(normal_vector(s.num_dofs(), seed0 + 50 + i), device="cuda") for i, s in enumerate(solvers)]
    return solvers, xs


@pytest.mark.parametrize("first,second", [([(24, 3), (16, 2), (9, 4), (40, 1), (7, 8)], [(5, 1), (3, 0)]),
                                          ([(64, 2), (33, 5)], [(17, 3)])])
def test_noalloc_batch_matches_allocating_batch(first, second):
    print(f"case noalloc batch {first} then {second}", flush=True)
    for spec, seed0 in ((first, 100), (second, 200)):
        solvers, xs = _batch(spec, seed0)
        try:
            y_ref = [torch.full_like(x, np.nan) for x in xs]
            y_new = [torch.full_like(x, np.nan) for x in xs]
            assert _call(H.lib.hdg_apply_trace_operator_batch, solvers, xs, y_ref) == 0
            assert _call(H.lib.hdg_apply_trace_operator_batch_noalloc, solvers, xs, y_new) == 0
            torch.cuda.synchronize()
            for i, (a, b) in enumerate(zip(y_ref, y_new)):
                assert torch.equal(a, b), (spec[i], float((a - b).abs().max()))
                assert bool(torch.isfinite(b).all())
        finally:
            for s in solvers:
                s.close()


def test_noalloc_batch_rejects_too_many_meshes():
    S = H.Solver(4, 1, np.ones(16))
    try:
        x = torch.zeros(S.num_dofs(), dtype=torch.float64, device="cuda")
        y = torch.zeros_like(x)
        cnt = NOALLOC_MAX + 1
        st = _call(H.lib.hdg_apply_trace_operator_batch_noalloc, [S] * cnt, [x] * cnt, [y] * cnt)
        assert st == -1
        assert b"HDG_BATCH_NOALLOC_MAX" in H.lib.hdg_last_error(S._h)
        assert _call(H.lib.hdg_apply_trace_operator_batch_noalloc, [S], [x], [y]) == 0
    finally:
        S.close()
