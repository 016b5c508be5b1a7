"""Nested p -> h geometric multigrid for the HDG trace system (paper Secs. 6-7).

Test infrastructure only (see oracle/__init__.py).

Hierarchy (Sec. 6, diagram fig_mg_description):
  * p-levels p = k, k-1, ..., 0 on the fixed mesh (full arithmetic
    coarsening).  Coarse operator either re-discretized (the paper's choice,
    subspace non-inheritance: the degree-p HDG blocks) or Galerkin (subspace
    inheritance) computed element by element, Kc^{(p-1)} = P4^T Kc^{(p)} P4,
    with P4 the p-prolongation on the element's four faces; the two give the
    same assembled result as P^T S P.
  * p-transfer (eqs. eq_mg_pro / eq_mg_res): prolongation is the natural
    embedding of degree-(p-1) traces into degree-p traces, face by face; in
    the nodal basis P_p[a, b] = l_b^{(p-1)}(xi_a^{(p)}).  Restriction is its
    adjoint, R = P^T, on residual (dual) vectors.
  * h-levels (eqs. eq_h_mg_pro / eq_h_mg_res, Gopalakrishnan-Tan): from the
    p = 0 trace space M_J, the next space M_{J-1} is continuous Q1 on the
    same mesh (zero on the boundary); P_J maps a Q1 function to the L2
    projection of its skeleton restriction onto face-wise constants (the
    face mean, i.e. the average of the two end-vertex values).  Coarser
    levels are Q1 on meshes n/2, n/4, ... with bilinear interpolation.
    Restriction is P^T and every h-level operator is the Galerkin product
    A_{k-1} = P^T A_k P (Sec. 6, coarse grid operator).
  * coarsest: direct solve (dense Cholesky) once the Q1 level has at most
    coarse_max unknowns or its mesh size is odd (the paper's coarsest
    system has dimension about 2000).
Smoothers (Sec. 6, relaxation).  On the p-levels the additive Schwarz
smoother x <- x + w sum_s R_s^T A_s^{-1} R_s (b - A x) with zero overlap and
either
  'face'  one subdomain per facet (A_s = the (p+1) x (p+1) diagonal block), or
  'chain' one subdomain per chain of facets: the vertical faces of one
          element row, or the horizontal faces of one element column
          (A_s = the block-tridiagonal restriction of A to the chain).
The weighting W of the paper's weighted Schwarz is the scalar w.  On every Q1
level: Chebyshev iteration preconditioned by the diagonal, degree nu, on the
interval [lo, hi] * lambda_max(diag^{-1} A) (Sec. 6: Chebyshev for the
h-levels).
Cycle: the V-cycle of Algs. algo_2 (p-levels) and algo_1 (h-levels) read as
the standard recursive cycle: pre-smooth nu1, restrict the residual, recurse
with zero initial guess, prolong-add, post-smooth nu2; the coarsest level is
solved exactly.  The cycle is symmetric (R = P^T, symmetric smoothers,
nu1 = nu2), so it also serves as a preconditioner for conjugate gradients
(Sec. 6, p-transfer paragraph).  Convergence monitor: the residual ratio of
Sec. 7; stop at ||b - S x||_2 <= rtol ||b||_2.

W schedule (Sec. 7 reports W-cycles beside V-cycles): every coarse-grid
correction is two cycles of the coarser level, the second started from the
first's result; the coarsest exact solve is not repeated.  The hybrid 'WH'
(not in the paper) repeats only corrections onto Q1 levels (the p = 0 -> Q1
step and the h-levels), where each level costs a quarter of the one above, and
keeps the V schedule on the p-levels.

Krylov-accelerated coarse levels (not in the paper; an extension of its
cycle): the K-cycle of Notay and Vassilevski (Numer. Linear Algebra Appl. 15,
2008).  On the p-levels named in `inner`, the coarse-grid correction is not
one recursive cycle but m steps of flexible conjugate gradients on that
level's system, each step preconditioned by one cycle started at that level
(itself possibly Krylov-accelerated further down).  Flexible CG is Notay's
FCG(1) (SIAM J. Sci. Comput. 22, 2000): the new direction is A-orthogonalised
against the previous one only, d = z - (z . q_prev / d_prev . q_prev) d_prev,
and the step is alpha = d . r / d . q.  A cycle containing such levels is a
nonlinear map, so the outer solver is FCG as well (mode 'fcg'); with a fixed
symmetric cycle FCG reproduces preconditioned CG.

Parity unpinned: the multigrid convergence factor itself.  The paper's
figure (rho < 0.22) is for an FSAI smoother, so no printed value exists for
these smoothers; tests check V-cycle and PCG solutions against the direct
solve, the symmetry of the cycle, and report the factor.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import scipy.linalg as sla

from . import quadrature as qd
from . import mesh as ms
from .hdg import Problem


# ------------------------------------------------------------------ transfers
def p_prolongation_1d(p):
    """P_p [(p+1) x p]: degree-(p-1) nodal traces evaluated at the degree-p nodes (eq. eq_mg_pro)."""
    return qd.lagrange_matrix(qd.trace_nodes(p - 1), qd.trace_nodes(p))


def p_prolongation(n, p):
    """Global p-prolongation M^{p-1} -> M^p, block diagonal over the interior faces."""
    return sp.kron(sp.identity(ms.n_faces(n), format='csr'), sp.csr_matrix(p_prolongation_1d(p)),
                   format='csr')


def q1_index(m, i, j):
    """Interior vertex (i, j), 1 <= i, j <= m-1, of the m x m mesh -> (i-1) + (m-1)(j-1); -1 on the boundary."""
    if i <= 0 or j <= 0 or i >= m or j >= m:
        return -1
    return (i - 1) + (m - 1) * (j - 1)


def trace_from_q1(n):
    """P_J: Q1 (interior vertices, mesh n) -> p = 0 traces: face value = mean of its end vertices (eq. eq_h_mg_pro)."""
    nf = ms.n_faces(n)
    rows, cols, vals = [], [], []
    for f in range(nf):
        lo, hi, o = ms.face_elements(n, f)
        i, j = hi % n, hi // n
        ends = [(i, j), (i, j + 1)] if o == 'v' else [(i, j), (i + 1, j)]
        for (a, b) in ends:
            v = q1_index(n, a, b)
            if v >= 0:
                rows.append(f)
                cols.append(v)
                vals.append(0.5)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf, (n - 1) ** 2))


def q1_bilinear(m):
    """Bilinear interpolation from Q1 on mesh m/2 to Q1 on mesh m (interior vertices)."""
    mc = m // 2
    rows, cols, vals = [], [], []
    for J in range(1, m):
        for I in range(1, m):
            r = q1_index(m, I, J)
            xs = [(I // 2, 1.0)] if I % 2 == 0 else [(I // 2, 0.5), (I // 2 + 1, 0.5)]
            ys = [(J // 2, 1.0)] if J % 2 == 0 else [(J // 2, 0.5), (J // 2 + 1, 0.5)]
            for (ci, wx) in xs:
                for (cj, wy) in ys:
                    c = q1_index(mc, ci, cj)
                    if c >= 0:
                        rows.append(r)
                        cols.append(c)
                        vals.append(wx * wy)
    return sp.csr_matrix((vals, (rows, cols)), shape=((m - 1) ** 2, (mc - 1) ** 2))


def element_prolongation(p):
    """P4 = blockdiag(P_p, P_p, P_p, P_p): the p-prolongation on one element's four faces."""
    return np.kron(np.eye(4), p_prolongation_1d(p))


# ------------------------------------------------------------------ smoothers
def face_blocks(S, P):
    """The (P x P) diagonal blocks of S, one per face, [nf, P, P]."""
    nf = S.shape[0] // P
    Sd = S.tocsr()
    out = np.zeros((nf, P, P))
    for f in range(nf):
        out[f] = Sd[f * P:(f + 1) * P, f * P:(f + 1) * P].toarray()
    return out


def block_apply(blocks, r):
    P = blocks.shape[1]
    return np.einsum('fab,fb->fa', blocks, r.reshape(-1, P)).reshape(-1)


def chains(n):
    """Faces of each chain: vertical faces of element row j (j = 0..n-1), then
    horizontal faces of element column i (i = 0..n-1), each in increasing x / y."""
    nv = n * (n - 1)
    out = [[(i - 1) + (n - 1) * j for i in range(1, n)] for j in range(n)]
    out += [[nv + i + n * (j - 1) for j in range(1, n)] for i in range(n)]
    return out


class ChainSolver:
    """Exact solves with the restriction of A to every chain of faces (zero-overlap Schwarz)."""

    def __init__(self, A, n, P):
        A = A.tocsr()
        self.parts = []
        for faces in chains(n):
            idx = (np.asarray(faces)[:, None] * P + np.arange(P)[None, :]).reshape(-1)
            self.parts.append((idx, spla.splu(A[idx][:, idx].tocsc())))

    def __call__(self, r):
        z = np.zeros_like(r)
        for idx, lu in self.parts:
            z[idx] = lu.solve(r[idx])
        return z


def patch_schwarz(A, n, P):
    """Sec. 6, additive Schwarz relaxation with overlap: one subdomain per element,
    the trace unknowns of its interior faces (neighbouring subdomains share the
    face between them), and the weighting W of the inverse counting matrix:
    every interior face lies in exactly two subdomains, so W = 1/2 and
        W M = 1/2 sum_K R_K^T (R_K A R_K^T)^{-1} R_K.
    Returns W M as a sparse matrix."""
    A = A.tocsr()
    rows, cols, vals = [], [], []
    for j in range(n):
        for i in range(n):
            faces = [f for f in ms.element_faces(n, i, j) if f >= 0]
            idx = (np.asarray(faces)[:, None] * P + np.arange(P)[None, :]).reshape(-1)
            MK = np.linalg.inv(A[idx][:, idx].toarray())
            rows.append(np.repeat(idx, idx.size))
            cols.append(np.tile(idx, idx.size))
            vals.append(MK.reshape(-1))
    M = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=A.shape).tocsr()
    return 0.5 * M


def chebyshev(A, dinv, lmax, lo, hi, b, x, steps):
    """Chebyshev iteration on the interval [lo, hi] lmax for diag^{-1} A (Saad, Alg. 12.1).

    theta, delta: center and half width; rho_k recurrence; update
    d_k = rho_k rho_{k-1} d_{k-1} + (2 rho_k / delta) z_k, z_k = diag^{-1}(b - A x)."""
    a, c = lo * lmax, hi * lmax
    theta, delta = 0.5 * (c + a), 0.5 * (c - a)
    sigma = theta / delta
    rho = 1.0 / sigma
    z = dinv * (b - A @ x)
    d = z / theta
    x = x + d
    for _ in range(1, steps):
        rho_new = 1.0 / (2.0 * sigma - rho)
        z = dinv * (b - A @ x)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * z
        x = x + d
        rho = rho_new
    return x


def lanczos_lmax(apply_op, apply_prec, n, steps=30, seed_vec=None):
    """Largest eigenvalue of M^{-1} A by Lanczos in the M inner product.

    Deterministic start vector v_i = 1 + 0.5 sin(i) unless given."""
    v = seed_vec if seed_vec is not None else 1.0 + 0.5 * np.sin(np.arange(n, dtype=np.float64))
    z = apply_prec(v)
    beta = np.sqrt(v @ z)
    v, z = v / beta, z / beta
    v_old = np.zeros(n)
    alphas, betas = [], []
    b_prev = 0.0
    for _ in range(min(steps, n)):
        w = apply_op(z)
        alpha = w @ z
        w = w - alpha * v - b_prev * v_old
        zw = apply_prec(w)
        b_new = np.sqrt(max(w @ zw, 0.0))
        alphas.append(alpha)
        if b_new < 1e-14 * abs(alpha):
            break
        betas.append(b_new)
        v_old, v, z = v, w / b_new, zw / b_new
        b_prev = b_new
    m = len(alphas)
    T = np.diag(alphas) + np.diag(betas[:m - 1], 1) + np.diag(betas[:m - 1], -1)
    return float(np.linalg.eigvalsh(T)[-1])


def assemble_blocks(n, p, blocks):
    """S = sum_K R_K^T Kc_K R_K over interior DoFs from per-element blocks [n*n, 4P, 4P]."""
    P = p + 1
    dofs = ms.element_dof_map(n, p)
    rows, cols, vals = [], [], []
    for e in range(n * n):
        d = dofs[e]
        m = d >= 0
        dd = d[m]
        rows.append(np.repeat(dd, len(dd)))
        cols.append(np.tile(dd, len(dd)))
        vals.append(blocks[e][np.ix_(m, m)].reshape(-1))
    N = ms.n_trace_dofs(n, p)
    S = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N)).tocsr()
    S.sum_duplicates()
    return S


# ------------------------------------------------------------------ hierarchy
class Level:
    pass


class Hierarchy:
    """Nested p/h multigrid for per-element kappa on the n x n mesh at degree k.

    coarse:   'galerkin' (element-wise P4^T Kc P4) or 'rediscretize' (paper)
    smoother: 'chain', 'face' or 'patch' additive Schwarz on the p-levels
    omega:    damping per p (dict) or scalar; default 0.8 for 'chain' and
              4 / (3 lambda_max(D^{-1} S_p)) for 'face'
    lmax:     dict name -> lambda_max(diag^{-1} A) on the Q1 levels (names
              'q<m>'); default: 30 Lanczos steps
    """

    def __init__(self, n, k, kappa, tau=1.0, nu1=2, nu2=2, coarse='galerkin', smoother='chain',
                 omega=None, lmax=None, cheb_lo=0.1, cheb_hi=1.1, coarse_max=2000, blocks_k=None,
                 inner=None, cycle='V'):
        if cycle not in ('V', 'W', 'WH'):
            raise ValueError("cycle must be 'V', 'W' or 'WH'")
        self.cycle = cycle
        self.n, self.k, self.nu1, self.nu2 = n, k, nu1, nu2
        self.inner = dict(inner or {})   # p-level -> flexible-CG steps of its coarse correction
        self.cheb_lo, self.cheb_hi = cheb_lo, cheb_hi
        self.smoother = smoother
        if omega is None or np.isscalar(omega):
            om = {} if omega is None else {p: float(omega) for p in range(k + 1)}
        else:
            om = dict(omega)
        lmax = dict(lmax or {})
        self.levels = []
        blocks = None
        for p in range(k, -1, -1):
            L = Level()
            L.kind, L.p, L.P, L.name = 'p', p, p + 1, 'p%d' % p
            if p == k or coarse == 'rediscretize':
                if p == k and blocks_k is not None:
                    blocks = blocks_k
                else:
                    prob = Problem(n, p, kappa, tau)
                    blocks = np.array([prob.element_block(e) for e in range(n * n)])
            else:
                P4 = element_prolongation(p + 1)
                blocks = np.einsum('ai,eab,bj->eij', P4, blocks, P4)
            L.blocks = blocks
            L.A = assemble_blocks(n, p, blocks)
            if smoother == 'chain':
                L.M = ChainSolver(L.A, n, L.P)
                om.setdefault(p, 0.8)
            elif smoother == 'patch':
                L.M = (lambda r, W=patch_schwarz(L.A, n, L.P): W @ r)
                om.setdefault(p, 1.0)
            else:
                L.Dinv = np.linalg.inv(face_blocks(L.A, L.P))
                L.M = (lambda r, Di=L.Dinv: block_apply(Di, r))
                if p not in om:
                    lam = lanczos_lmax(lambda v, A=L.A: A @ v, L.M, L.A.shape[0])
                    om[p] = 4.0 / (3.0 * lam)
            L.omega = om[p]
            L.Pmat = p_prolongation(n, p) if p >= 1 else trace_from_q1(n)
            self.levels.append(L)
        A = (L.Pmat.T @ L.A @ L.Pmat).tocsr()
        m = n
        while True:
            L = Level()
            L.kind, L.m, L.name = 'q', m, 'q%d' % m
            L.A = A
            self.levels.append(L)
            if A.shape[0] <= coarse_max or m % 2 == 1 or m < 4:
                L.coarsest = True
                L.chol = sla.cho_factor(A.toarray(), lower=True)
                break
            L.coarsest = False
            L.dinv = 1.0 / A.diagonal()
            if L.name not in lmax:
                lmax[L.name] = lanczos_lmax(lambda v, A=A: A @ v, lambda v, d=L.dinv: d * v, A.shape[0])
            L.lmax = lmax[L.name]
            L.Pmat = q1_bilinear(m)
            A = (L.Pmat.T @ A @ L.Pmat).tocsr()
            m //= 2
        self.omega, self.lmax = om, lmax

    def smooth(self, L, b, x, nu):
        if L.kind == 'p':
            for _ in range(nu):
                x = x + L.omega * L.M(b - L.A @ x)
            return x
        return chebyshev(L.A, L.dinv, L.lmax, self.cheb_lo, self.cheb_hi, b, x, nu)

    def _repeat(self, C):
        """Whether the coarse correction onto level C is taken twice: every level
        under 'W', the Q1 levels only under 'WH'; never the coarsest."""
        if getattr(C, 'coarsest', False):
            return False
        return self.cycle == 'W' or (self.cycle == 'WH' and C.kind == 'q')

    def vcycle(self, b, x, lev=0):
        """One (nu1, nu2) cycle at level index lev (Algs. algo_2 then algo_1), with
        the V or W schedule of self.cycle."""
        L = self.levels[lev]
        if getattr(L, 'coarsest', False):
            return sla.cho_solve(L.chol, b)
        x = self.smooth(L, b, x, self.nu1)
        r = b - L.A @ x
        rc = L.Pmat.T @ r
        C = self.levels[lev + 1]
        m = self.inner.get(C.p, 0) if C.kind == 'p' else 0
        if m > 0:
            ec = self.krylov_correction(lev + 1, rc, m)
        else:
            ec = self.vcycle(rc, np.zeros(rc.shape[0]), lev + 1)
            if self._repeat(C):
                ec = self.vcycle(rc, ec, lev + 1)
        x = x + L.Pmat @ ec
        x = self.smooth(L, b, x, self.nu2)
        return x

    def krylov_correction(self, lev, b, m):
        """m steps of FCG(1) for A_lev e = b from e = 0, each preconditioned by one
        cycle started at level lev (the K-cycle's coarse correction)."""
        A = self.levels[lev].A
        e = np.zeros_like(b)
        r = b.copy()
        d = q = dq = None
        for step in range(m):
            z = self.vcycle(r, np.zeros_like(r), lev)
            d = z if d is None else z - ((z @ q) / dq) * d
            q = A @ d
            dq = d @ q
            if not dq > 0.0:        # r == 0: nothing left to correct
                break
            alpha = (d @ r) / dq
            e = e + alpha * d
            r = r - alpha * q
        return e

    def fmg(self, b, cycles=1):
        """One full-multigrid pass (Sec. 7) for S x = b from nothing: b is
        restricted to every level (b_{l+1} = P_l^T b_l, the right-hand sides of
        the Galerkin coarse systems), the coarsest system is solved exactly, and
        on each finer level the prolonged coarser result starts `cycles` cycles
        of that level (V or W by self.cycle).  Returns the finest iterate."""
        bs = [b]
        for L in self.levels[:-1]:
            bs.append(L.Pmat.T @ bs[-1])
        x = sla.cho_solve(self.levels[-1].chol, bs[-1])
        for lev in range(len(self.levels) - 2, -1, -1):
            x = self.levels[lev].Pmat @ x
            for _ in range(cycles):
                x = self.vcycle(bs[lev], x, lev)
        return x

    def solve(self, b, x0=None, rtol=1e-10, maxit=200, mode='pcg'):
        """Solve S x = b to ||r||_2 <= rtol ||b||_2.

        mode 'vcycle': repeated V-cycles (the paper's stationary solver);
        mode 'pcg': conjugate gradients preconditioned by one V-cycle with zero
        initial guess; mode 'fcg': flexible CG, FCG(1), with the same
        preconditioner (needed when the cycle has Krylov-accelerated levels).
        Returns x and the residual-norm history (entry 0 is the initial
        residual; for 'pcg' / 'fcg' the recursively updated residual)."""
        S = self.levels[0].A
        x = np.zeros(S.shape[0]) if x0 is None else np.array(x0, dtype=np.float64)
        nb = np.linalg.norm(b)
        r = b - S @ x
        hist = [np.linalg.norm(r)]
        if mode == 'vcycle':
            while hist[-1] > rtol * nb and len(hist) <= maxit:
                x = self.vcycle(b, x)
                hist.append(np.linalg.norm(b - S @ x))
            return x, np.array(hist)
        if mode == 'fcg':
            d = q = dq = None
            while hist[-1] > rtol * nb and len(hist) <= maxit:
                z = self.vcycle(r, np.zeros_like(r))
                d = z if d is None else z - ((z @ q) / dq) * d
                q = S @ d
                dq = d @ q
                alpha = (d @ r) / dq
                x = x + alpha * d
                r = r - alpha * q
                hist.append(np.linalg.norm(r))
            return x, np.array(hist)
        z = self.vcycle(r, np.zeros_like(r))
        d = z.copy()
        rz = r @ z
        while hist[-1] > rtol * nb and len(hist) <= maxit:
            q = S @ d
            alpha = rz / (d @ q)
            x = x + alpha * d
            r = r - alpha * q
            hist.append(np.linalg.norm(r))
            if hist[-1] <= rtol * nb:
                break
            z = self.vcycle(r, np.zeros_like(r))
            rz_new = r @ z
            d = z + (rz_new / rz) * d
            rz = rz_new
        return x, np.array(hist)


def convergence_factor(hist):
    """Mean factor (||r_m|| / ||r_0||)^(1/m) and the last ratio rho_m (Sec. 7)."""
    m = len(hist) - 1
    if m <= 0:
        return 0.0, 0.0
    return float((hist[-1] / hist[0]) ** (1.0 / m)), float(hist[-1] / hist[-2])
