"""MI355X-native HDG trace operator and nested p/h multigrid (arXiv:1705.09907).

Thin ctypes binding over the C ABI of ``libhdggmg.so`` (include/hdggmg.h):
argument marshalling only -- every step runs in the library's HIP kernels.
PyTorch supplies device memory (float64 CUDA tensors) and the stream.  There is
no CPU fallback: importing this package without the built library raises.
"""
import ctypes
import os

import numpy as np
# torch first: it loads its own HIP runtime, and the library's HIP dependency
# then resolves to that same runtime.  Loaded the other way round, the process
# holds two HIP runtimes, and torch's streams and allocations mean nothing to
# the library's (device calls then fail).
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhdggmg.so")

HDG_MAX_DEGREE = 8
HDG_MAX_HLEVELS = 24
SMOOTHERS = {"chain": 0, "face": 1, "patch": 2}
COARSE = {"galerkin": 0, "rediscretize": 1}
MODES = {"pcg": 0, "vcycle": 1, "fcg": 2}
CYCLES = {"V": 0, "W": 1, "WH": 2}
MULTI_KERNELS = {"auto": 0, "vector": 1, "matrix": 2}
CHAIN_SHAPES = {"auto": 0, "lean": 1, "wide": 2, "flat": 3, "tri": 4}
Q1_SCHEDULES = {"fused": 0, "separate": 1}
PRECISIONS = {"f64": 0, "f32": 1, "bf16": 2}
STATUS = {0: "ok", -1: "invalid argument", -2: "out of memory", -3: "HIP error",
          -4: "not converged", -5: "non-finite value", -6: "invalid state",
          -7: "stopped at the rounding floor of the residual"}


class Config(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("k", ctypes.c_int32), ("tau", ctypes.c_double),
                ("nu1", ctypes.c_int32), ("nu2", ctypes.c_int32),
                ("smoother", ctypes.c_int32), ("coarse", ctypes.c_int32),
                ("omega", ctypes.c_double * (HDG_MAX_DEGREE + 1)),
                ("cheb_lo", ctypes.c_double), ("cheb_hi", ctypes.c_double),
                ("cheb_lmax", ctypes.c_double * HDG_MAX_HLEVELS),
                ("coarse_max", ctypes.c_int32), ("nq", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("inner_steps", ctypes.c_int32 * (HDG_MAX_DEGREE + 1)),
                ("graph", ctypes.c_int32), ("autotune", ctypes.c_int32), ("cycle", ctypes.c_int32),
                ("multi_kernel", ctypes.c_int32), ("setup_on_host", ctypes.c_int32),
                ("chain_shape", ctypes.c_int32), ("q1_schedule", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 1)]


_P = ctypes.c_void_p
_I32, _I64, _D = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_PD = ctypes.POINTER(ctypes.c_double)
_PI32, _PI64 = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)

# name -> argtypes; every function returns hdg_status_t (int) unless listed in _RESTYPES
SIGNATURES = {
    "hdg_config_default": [_I32, _I32, ctypes.POINTER(Config)],
    "hdg_create": [ctypes.POINTER(Config), _PD, _P, ctypes.POINTER(_P)],
    "hdg_destroy": [_P],
    "hdg_update_coefficients": [_P, _PD],
    "hdg_get_face_blocks": [_P, _I32, _I64, _PD],
    "hdg_num_dofs": [_P, _I32, _PI64],
    "hdg_num_hlevels": [_P, _PI32],
    "hdg_hlevel_mesh": [_P, _I32, _PI32],
    "hdg_get_params": [_P, _PD, _PD],
    "hdg_get_chain_shape": [_P, _I32, _PI32, _PI32, _PI32],
    "hdg_get_element_block": [_P, _I32, _I64, _PD],
    "hdg_element_block_host": [_I32, _I32, _I32, _D, _D, _I32, _PD],
    "hdg_quadrature_nodes": [_I32, _PD],
    "hdg_assemble_rhs": [_P, _PD, _PD, _P],
    "hdg_apply_trace_operator": [_P, _I32, _P, _P],
    "hdg_apply_abs": [_P, _I32, _P, _P],
    "hdg_apply_trace_operator_lp": [_P, _I32, _P, _P],
    "hdg_apply_trace_operator_timed": [_P, _I32, _I32, _P, _P, _PD],
    "hdg_apply_trace_operator_multi": [_P, _I32, _I32, _I32, _P, _P],
    "hdg_apply_trace_operator_batch": [_I32, _P, _P, _P, _P],
    "hdg_apply_trace_operator_batch_noalloc": [_I32, _P, _P, _P, _P],
    "hdg_apply_trace_operator_batch_lp": [_I32, _P, _P, _P, _P],
    "hdg_residual": [_P, _I32, _P, _P, _P, _PD],
    "hdg_smooth": [_P, _I32, _P, _P, _I32],
    "hdg_restrict": [_P, _I32, _P, _P],
    "hdg_prolong": [_P, _I32, _P, _P],
    "hdg_vcycle": [_P, _P, _P],
    "hdg_fmg": [_P, _P, _P, _I32],
    "hdg_solve": [_P, _P, _P, _D, _I32, _I32, _PI32, _PD, _PD],
    "hdg_solve_multi": [_P, _I32, _P, _P, _D, _I32, _PI32, _PD],
    "hdg_reconstruct": [_P, _P, _P, _P],
    "hdg_misfit_adjoint_rhs": [_P, _P, _P, _P, _PD],
    "hdg_misfit_gradient": [_P, _P, _P, _P, _P, _P],
    "hdg_last_error": [_P],
    "hdg_status_string": [_I32],
}
_RESTYPES = {"hdg_last_error": ctypes.c_char_p, "hdg_status_string": ctypes.c_char_p}


def load_library(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python paper_1705_09907_amd/build.py` "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, args in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = _RESTYPES.get(name, ctypes.c_int)
    return lib


lib = load_library()


class HDGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _dptr(t, name, numel=None, dtype="float64"):
    import torch
    if (not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != getattr(torch, dtype)
            or not t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous {dtype} CUDA tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} entries, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


def _host(a, name, size=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if size is not None and a.size != size:
        raise ValueError(f"{name} has {a.size} entries, expected {size}")
    return a, a.ctypes.data_as(_PD)


def element_block_host(n, k, p, kappa_e, tau=1.0, coarse="galerkin"):
    """Condensed block of one element computed by the library's host setup (no device)."""
    out = np.zeros((4 * (p + 1), 4 * (p + 1)))
    st = lib.hdg_element_block_host(n, k, p, tau, kappa_e, COARSE[coarse], out.ctypes.data_as(_PD))
    if st != 0:
        raise HDGError(st, "hdg_element_block_host: bad arguments")
    return out


def quadrature_nodes(nq):
    x = np.zeros(nq)
    st = lib.hdg_quadrature_nodes(nq, x.ctypes.data_as(_PD))
    if st != 0:
        raise HDGError(st, "bad nq")
    return x


def apply_batch(solvers, xs, ys=None, levels=None, noalloc=False, lp=False):
    """y_i = S_i x_i for many meshes in one kernel launch (FP64; synchronizes).
    noalloc=True calls hdg_apply_trace_operator_batch_noalloc (same products, no
    allocation, at most HDG_BATCH_NOALLOC_MAX meshes); lp=True calls
    hdg_apply_trace_operator_batch_lp (the handles' reduced cycle precision,
    float32 vectors)."""
    import torch
    cnt = len(solvers)
    levels = [s.k for s in solvers] if levels is None else list(levels)
    ys = [torch.empty_like(x) for x in xs] if ys is None else ys
    H = (ctypes.c_void_p * cnt)(*[s._h.value for s in solvers])
    Pv = (ctypes.c_int32 * cnt)(*levels)
    dt = "float32" if lp else "float64"
    Xv = (ctypes.c_void_p * cnt)(*[_dptr(x, "x", s.num_dofs(l), dt).value for s, x, l in zip(solvers, xs, levels)])
    Yv = (ctypes.c_void_p * cnt)(*[_dptr(y, "y", s.num_dofs(l), dt).value for s, y, l in zip(solvers, ys, levels)])
    if lp and noalloc:
        raise ValueError("the allocation-free batch apply is FP64 only")
    fn = (lib.hdg_apply_trace_operator_batch_lp if lp else
          lib.hdg_apply_trace_operator_batch_noalloc if noalloc else lib.hdg_apply_trace_operator_batch)
    st = fn(cnt, H, Pv, Xv, Yv)
    if st != 0:
        raise HDGError(st, lib.hdg_last_error(solvers[0]._h).decode())
    return ys


class Solver:
    """Handle over hdg_create: one n x n mesh, degree k, per-element kappa."""

    def __init__(self, n, k, kappa, tau=1.0, nu1=2, nu2=2, smoother="chain", coarse="galerkin",
                 omega=None, cheb_lmax=None, cheb=(0.1, 1.1), coarse_max=2000, nq=None, stream=None,
                 precision="f64", inner=None, graph=False, autotune=False, cycle="V", multi_kernel="auto",
                 host_setup=False, chain_shape="auto", q1_schedule="fused"):
        import torch
        cfg = Config()
        lib.hdg_config_default(n, k, ctypes.byref(cfg))
        cfg.tau, cfg.nu1, cfg.nu2 = tau, nu1, nu2
        cfg.smoother, cfg.coarse = SMOOTHERS[smoother], COARSE[coarse]
        if omega is not None:
            om = omega if isinstance(omega, dict) else {p: omega for p in range(k + 1)}
            for p, v in om.items():
                cfg.omega[p] = v
        if cheb_lmax is not None:
            for l, v in enumerate(cheb_lmax):
                cfg.cheb_lmax[l] = v
        cfg.cheb_lo, cfg.cheb_hi = cheb
        cfg.coarse_max = coarse_max
        if nq is not None:
            cfg.nq = nq
        cfg.precision = PRECISIONS[precision]
        for p, m in (inner or {}).items():
            cfg.inner_steps[p] = m
        cfg.graph = 1 if graph else 0
        cfg.autotune = 1 if autotune else 0
        cfg.cycle = CYCLES[cycle]
        cfg.multi_kernel = MULTI_KERNELS[multi_kernel]
        cfg.setup_on_host = 1 if host_setup else 0
        cfg.chain_shape = CHAIN_SHAPES[chain_shape]
        cfg.q1_schedule = Q1_SCHEDULES[q1_schedule]
        self.n, self.k, self.nq, self.precision = n, k, cfg.nq, precision
        kap, kp = _host(kappa, "kappa", n * n)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        st = lib.hdg_create(ctypes.byref(cfg), kp, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
        if st != 0:
            raise HDGError(st, "hdg_create failed (see arguments)")
        self._h = h

    # ---------------------------------------------------------------- helpers
    def _check(self, st):
        if st != 0:
            raise HDGError(st, lib.hdg_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib.hdg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def num_dofs(self, p=None):
        p = self.k if p is None else p
        v = ctypes.c_int64()
        self._check(lib.hdg_num_dofs(self._h, p, ctypes.byref(v)))
        return v.value

    def num_hlevels(self):
        v = ctypes.c_int32()
        self._check(lib.hdg_num_hlevels(self._h, ctypes.byref(v)))
        return v.value

    def hlevel_mesh(self, level):
        v = ctypes.c_int32()
        self._check(lib.hdg_hlevel_mesh(self._h, level, ctypes.byref(v)))
        return v.value

    def params(self):
        om = np.zeros(self.k + 1)
        lm = np.zeros(self.num_hlevels())
        self._check(lib.hdg_get_params(self._h, om.ctypes.data_as(_PD), lm.ctypes.data_as(_PD)))
        return om, lm

    def chain_shape(self, p):
        """(workgroup size, XCD-aware order, LDS staging level) of the chain solve at level p."""
        t, r, l = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(lib.hdg_get_chain_shape(self._h, p, ctypes.byref(t), ctypes.byref(r), ctypes.byref(l)))
        return t.value, r.value, l.value

    def element_block(self, p, e):
        out = np.zeros((4 * (p + 1), 4 * (p + 1)))
        self._check(lib.hdg_get_element_block(self._h, p, e, out.ctypes.data_as(_PD)))
        return out

    def face_blocks(self, p, f):
        """The 7 blocks [7, p+1, p+1] of face f at level p as stored on the device."""
        out = np.zeros((7, p + 1, p + 1))
        self._check(lib.hdg_get_face_blocks(self._h, p, f, out.ctypes.data_as(_PD)))
        return out

    def update_coefficients(self, kappa):
        """New per-element coefficient on this handle (device set-up, no reallocation)."""
        kap, kp = _host(kappa, "kappa", self.n * self.n)
        self._check(lib.hdg_update_coefficients(self._h, kp))

    def _empty(self, p):
        import torch
        return torch.empty(self.num_dofs(p), dtype=torch.float64, device="cuda")

    # ------------------------------------------------------------- operations
    def assemble_rhs(self, f_qp, gD_qp=None, out=None):
        f, fp = _host(f_qp, "f_qp", self.n * self.n * self.nq * self.nq)
        gp = None
        if gD_qp is not None:
            g, gp = _host(gD_qp, "gD_qp", 4 * self.n * self.nq)
        out = self._empty(self.k) if out is None else out
        self._check(lib.hdg_assemble_rhs(self._h, fp, gp, _dptr(out, "b", self.num_dofs())))
        return out

    def apply(self, p, x, y=None):
        N = self.num_dofs(p)
        y = self._empty(p) if y is None else y
        self._check(lib.hdg_apply_trace_operator(self._h, p, _dptr(x, "x", N), _dptr(y, "y", N)))
        return y

    def apply_abs(self, p, x, y=None):
        """y = |S_p| |x| entrywise (the rounding scale of S_p x)."""
        N = self.num_dofs(p)
        y = self._empty(p) if y is None else y
        self._check(lib.hdg_apply_abs(self._h, p, _dptr(x, "x", N), _dptr(y, "y", N)))
        return y

    def apply_lp(self, p, x, y=None):
        """y = S_p x in the cycle precision (float32 tensors) of an f32 / bf16 handle."""
        import torch
        N = self.num_dofs(p)
        y = torch.empty(N, dtype=torch.float32, device="cuda") if y is None else y
        self._check(lib.hdg_apply_trace_operator_lp(self._h, p, _dptr(x, "x", N, "float32"),
                                                    _dptr(y, "y", N, "float32")))
        return y

    def apply_timed(self, p, x, y):
        """y = S_p x (float64 tensors: FP64 operator; float32: the cycle precision),
        returning the kernel's own duration in microseconds (synchronizes)."""
        import torch
        N = self.num_dofs(p)
        lp = x.dtype == torch.float32
        dt = "float32" if lp else "float64"
        us = ctypes.c_double()
        self._check(lib.hdg_apply_trace_operator_timed(
            self._h, p, PRECISIONS[self.precision] if lp else 0, _dptr(x, "x", N, dt), _dptr(y, "y", N, dt),
            ctypes.byref(us)))
        return us.value

    def apply_multi(self, p, X, Y=None):
        """Y = S_p X for X [N(p), nrhs] (float64: FP64 operator; float32: the cycle precision)."""
        import torch
        N = self.num_dofs(p)
        if X.dim() != 2 or X.shape[0] != N:
            raise ValueError(f"X must be [{N}, nrhs]")
        lp = X.dtype == torch.float32
        dt = "float32" if lp else "float64"
        Y = torch.empty_like(X) if Y is None else Y
        R = X.shape[1]
        self._check(lib.hdg_apply_trace_operator_multi(
            self._h, p, PRECISIONS[self.precision] if lp else 0, R, _dptr(X, "X", N * R, dt),
            _dptr(Y, "Y", N * R, dt)))
        return Y

    def residual(self, p, b, x, r=None, norm=False):
        N = self.num_dofs(p)
        r = self._empty(p) if r is None else r
        nv = ctypes.c_double()
        self._check(lib.hdg_residual(self._h, p, _dptr(b, "b", N), _dptr(x, "x", N), _dptr(r, "r", N),
                                     ctypes.byref(nv) if norm else None))
        return (r, nv.value) if norm else r

    def smooth(self, p, b, x, sweeps=1):
        N = self.num_dofs(p)
        self._check(lib.hdg_smooth(self._h, p, _dptr(b, "b", N), _dptr(x, "x", N), sweeps))
        return x

    def restrict(self, p_fine, r_fine, out=None):
        out = self._empty(p_fine - 1) if out is None else out
        self._check(lib.hdg_restrict(self._h, p_fine, _dptr(r_fine, "r_fine", self.num_dofs(p_fine)),
                                     _dptr(out, "r_coarse", self.num_dofs(p_fine - 1))))
        return out

    def prolong(self, p_fine, e_coarse, x_fine):
        self._check(lib.hdg_prolong(self._h, p_fine, _dptr(e_coarse, "e_coarse", self.num_dofs(p_fine - 1)),
                                    _dptr(x_fine, "x_fine", self.num_dofs(p_fine))))
        return x_fine

    def vcycle(self, b, x):
        N = self.num_dofs()
        self._check(lib.hdg_vcycle(self._h, _dptr(b, "b", N), _dptr(x, "x", N)))
        return x

    def fmg(self, b, x=None, cycles=1):
        """One full-multigrid pass for S_k x = b (x is overwritten); returns x."""
        N = self.num_dofs()
        if x is None:
            x = torch.empty_like(b)
        self._check(lib.hdg_fmg(self._h, _dptr(b, "b", N), _dptr(x, "x", N), int(cycles)))
        return x

    # ------------------------------------------------ misfit gradient (adjoint)
    def _evec(self, t, name, per):
        return _dptr(t, name, self.n * self.n * per)

    def reconstruct(self, lam, U=None, Q=None, with_q=False):
        """U (and Q) of every element from the traces lam and the last assembled source."""
        import torch
        P2 = (self.k + 1) ** 2
        U = torch.empty(self.n * self.n * P2, dtype=torch.float64, device="cuda") if U is None else U
        if with_q and Q is None:
            Q = torch.empty(self.n * self.n * 2 * P2, dtype=torch.float64, device="cuda")
        self._check(lib.hdg_reconstruct(self._h, _dptr(lam, "lam", self.num_dofs()), self._evec(U, "U", P2),
                                        self._evec(Q, "Q", 2 * P2) if Q is not None else None))
        return (U, Q) if with_q else U

    def adjoint_rhs(self, U, U_obs, c=None):
        """c = (dU/dLambda)^T (U - U_obs) and L = 1/2 |U - U_obs|^2."""
        P2 = (self.k + 1) ** 2
        c = self._empty(self.k) if c is None else c
        L = ctypes.c_double()
        self._check(lib.hdg_misfit_adjoint_rhs(self._h, self._evec(U, "U", P2), self._evec(U_obs, "U_obs", P2),
                                               _dptr(c, "c", self.num_dofs()), ctypes.byref(L)))
        return c, L.value

    def misfit_gradient(self, lam, U, U_obs, mu, grad=None):
        """dL/dtheta per element from the forward and adjoint traces."""
        import torch
        P2 = (self.k + 1) ** 2
        N = self.num_dofs()
        grad = torch.empty(self.n * self.n, dtype=torch.float64, device="cuda") if grad is None else grad
        self._check(lib.hdg_misfit_gradient(self._h, _dptr(lam, "lam", N), self._evec(U, "U", P2),
                                            self._evec(U_obs, "U_obs", P2), _dptr(mu, "mu", N),
                                            self._evec(grad, "grad", 1)))
        return grad

    def solve_multi(self, B, X=None, rtol=1e-10, maxit=200, raise_on_fail=True):
        """Solve S X = B for B [N, nrhs] (float64); returns X, iterations and relative residuals per column."""
        import torch
        N = self.num_dofs()
        if B.dim() != 2 or B.shape[0] != N:
            raise ValueError(f"B must be [{N}, nrhs]")
        R = B.shape[1]
        X = torch.zeros_like(B) if X is None else X
        its = np.zeros(R, dtype=np.int32)
        rr = np.zeros(R)
        st = lib.hdg_solve_multi(self._h, R, _dptr(B, "B", N * R), _dptr(X, "X", N * R), rtol, maxit,
                                 its.ctypes.data_as(_PI32), rr.ctypes.data_as(_PD))
        self.last_status = st
        if st != 0 and (raise_on_fail or st not in (-4, -7)):
            self._check(st)
        return X, its, rr

    def solve(self, b, x=None, rtol=1e-10, maxit=200, mode="pcg", raise_on_fail=True, accept_floor=False):
        """Solve S x = b; returns x, iterations, the true relative residual and the
        residual history.  raise_on_fail=False returns instead of raising when the
        solve ends NOT_CONVERGED or AT_FLOOR; accept_floor=True returns on AT_FLOOR
        (the true residual reached the rounding floor of b - S x above rtol).  The
        status of the last call is kept in last_status."""
        import torch
        N = self.num_dofs()
        if x is None:
            x = torch.zeros(N, dtype=torch.float64, device="cuda")
        it = ctypes.c_int32()
        rr = ctypes.c_double()
        hist = np.zeros(maxit + 1)
        st = lib.hdg_solve(self._h, _dptr(b, "b", N), _dptr(x, "x", N), rtol, maxit, MODES[mode],
                           ctypes.byref(it), ctypes.byref(rr), hist.ctypes.data_as(_PD))
        self.last_status = st
        tolerated = (-4, -7) if not raise_on_fail else ((-7,) if accept_floor else ())
        if st != 0 and st not in tolerated:
            self._check(st)
        return x, it.value, rr.value, hist[:it.value + 1]
