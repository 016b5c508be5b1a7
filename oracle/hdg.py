"""HDG (LDG-H) local solvers, static condensation and the assembled trace system.

Test infrastructure only (see oracle/__init__.py).

Follows paper Sec. 3:
  * weak form eqs. eq_h1-eq_h3 with the flux variable q = -K grad u from the
    mixed form eq2.  Reading: the volume term of eq_h1 is (K^{-1} q_h, v)
    (the printed eq_h1 drops K^{-1}; the mixed form eq2 has it).
  * local element systems eqs. static_1 / static_2:
        A Q - B^T U + C Lambda = R,   B Q + D U + E Lambda = F
    with A = (K^{-1} phi_j, phi_i) (x2 components), B[i, j] = (div v_j, w_i),
    C[j, m] = <mu_m, v_j . n>, D = tau sum_edges <w_j, w_i>,
    E[i, m] = -tau <mu_m, w_i>.
  * static condensation eq. shur0: [Q; U] = Abb^{-1} ( -[C; E] Lambda + [R; F] ),
    Abb = [[A, -B^T], [B, D]].
  * transmission condition eq. shur1: per interior edge the two elements'
    G Q + tau H U - tau M Lambda sum to zero.  With G = C^T|_e and
    tau H = -E^T|_e, substituting eq. shur0 gives the per-element condensed
    block
        Kc = [C^T, -E^T] Abb^{-1} [C; E] + tau M_dK
    and source flux g = [C^T, -E^T] Abb^{-1} [0; F].
  * procedure steps (i)-(iv) of Sec. 3 (local problems, assembly, solve,
    reconstruction).  Readings: trace unknowns and test functions live on the
    interior skeleton only; boundary traces equal the L2 projection P_h g_D;
    tau is one constant on every edge (Sec. 5 sets tau = 1).
Basis and quadrature follow Sec. 4: nodal tensor-product GLL basis
phi_I = l_i(xi) l_j(eta), I = i + j (p+1), integrals by Gauss-Legendre with nq
points per direction (nq defaults to p + 2, exact for the polynomial
integrands when K is constant per element), affine map with Jacobian h^2/4 on
elements and h/2 on edges.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import quadrature as qd
from . import mesh as ms


class RefOps:
    """Reference-element tables for degree p and nq GL points per direction."""

    def __init__(self, p, nq=None):
        self.p = p
        self.P = p + 1
        self.nq = nq if nq is not None else p + 2
        self.nodes = qd.trace_nodes(p)
        self.xq, self.wq = qd.gauss_legendre(self.nq)
        self.Lq = qd.lagrange_matrix(self.nodes, self.xq)            # [nq, P]
        self.Dq = qd.lagrange_derivative_matrix(self.nodes, self.xq)  # [nq, P]
        self.Lm1 = qd.lagrange_matrix(self.nodes, [-1.0])[0]         # l_i(-1)
        self.Lp1 = qd.lagrange_matrix(self.nodes, [1.0])[0]          # l_i(+1)
        P, nq = self.P, self.nq
        # volume point qq = a + nq b (a along x), basis I = i + P j
        self.Phi = np.einsum('ai,bj->baji', self.Lq, self.Lq).reshape(nq * nq, P * P)
        self.dPhi_xi = np.einsum('ai,bj->baji', self.Dq, self.Lq).reshape(nq * nq, P * P)
        self.dPhi_eta = np.einsum('ai,bj->baji', self.Lq, self.Dq).reshape(nq * nq, P * P)
        self.wv = np.outer(self.wq, self.wq).reshape(nq * nq)  # w_b w_a at qq = a + nq b
        # trace of the volume basis on each local edge at the edge GL points:
        # Tr[lf][q, I]
        Tr = []
        for lf in range(4):
            T = np.zeros((nq, P * P))
            for jj in range(P):
                for ii in range(P):
                    I = ii + P * jj
                    if lf == ms.LEFT:
                        T[:, I] = self.Lm1[ii] * self.Lq[:, jj]
                    elif lf == ms.RIGHT:
                        T[:, I] = self.Lp1[ii] * self.Lq[:, jj]
                    elif lf == ms.BOTTOM:
                        T[:, I] = self.Lq[:, ii] * self.Lm1[jj]
                    else:
                        T[:, I] = self.Lq[:, ii] * self.Lp1[jj]
            Tr.append(T)
        self.Tr = Tr
        self.normals = [(-1.0, 0.0), (1.0, 0.0), (0.0, -1.0), (0.0, 1.0)]

    def volume_points(self, i, j, h):
        """Physical coordinates of the nq*nq GL points of element (i, j), qq = a + nq b."""
        xs = (i + 0.5 * (1.0 + self.xq)) * h
        ys = (j + 0.5 * (1.0 + self.xq)) * h
        X = np.tile(xs, self.nq)
        Y = np.repeat(ys, self.nq)
        return X, Y


def local_matrices(ref, h, tau, inv_kappa_q):
    """A, B, C, D, E, M_dK of eqs. static_1/static_2 for one element.

    inv_kappa_q: 1/K at the nq*nq volume GL points (constant K: a constant array)."""
    P = ref.P
    n2 = P * P
    wv = ref.wv * (h * h / 4.0)
    Mk = ref.Phi.T @ (ref.Phi * (wv * inv_kappa_q)[:, None])
    A = np.zeros((2 * n2, 2 * n2))
    A[:n2, :n2] = Mk
    A[n2:, n2:] = Mk
    # B[I, J] = (div v_J, w_I); d/dx = (2/h) d/dxi
    B = np.zeros((n2, 2 * n2))
    B[:, :n2] = ref.Phi.T @ (ref.dPhi_xi * (wv * 2.0 / h)[:, None])
    B[:, n2:] = ref.Phi.T @ (ref.dPhi_eta * (wv * 2.0 / h)[:, None])
    we = ref.wq * (h / 2.0)
    C = np.zeros((2 * n2, 4 * P))
    E = np.zeros((n2, 4 * P))
    D = np.zeros((n2, n2))
    M = np.zeros((4 * P, 4 * P))
    Me = ref.Lq.T @ (ref.Lq * we[:, None])
    for lf in range(4):
        T = ref.Tr[lf]
        nx, ny = ref.normals[lf]
        cols = slice(lf * P, (lf + 1) * P)
        TM = T.T @ (ref.Lq * we[:, None])   # <phi_I, mu_m>_e  [n2, P]
        C[:n2, cols] = nx * TM
        C[n2:, cols] = ny * TM
        E[:, cols] = -tau * TM
        D += tau * (T.T @ (T * we[:, None]))
        M[cols, cols] = Me
    return A, B, C, D, E, M


def local_system(A, B, D):
    """Abb = [[A, -B^T], [B, D]] of eq. shur0."""
    n2 = D.shape[0]
    Abb = np.zeros((3 * n2, 3 * n2))
    Abb[:2 * n2, :2 * n2] = A
    Abb[:2 * n2, 2 * n2:] = -B.T
    Abb[2 * n2:, :2 * n2] = B
    Abb[2 * n2:, 2 * n2:] = D
    return Abb


def condensed_block(A, B, C, D, E, M, tau):
    """Kc = [C^T, -E^T] Abb^{-1} [C; E] + tau M_dK (eqs. shur0 into shur1)."""
    Abb = local_system(A, B, D)
    CE = np.vstack([C, E])
    X = np.linalg.solve(Abb, CE)
    return np.hstack([C.T, -E.T]) @ X + tau * M


def source_flux(A, B, C, D, E, F):
    """g = [C^T, -E^T] Abb^{-1} [0; F]  (eq. shur0 with R = 0, into shur1)."""
    Abb = local_system(A, B, D)
    n2 = D.shape[0]
    rhs = np.concatenate([np.zeros(2 * n2), F])
    return np.hstack([C.T, -E.T]) @ np.linalg.solve(Abb, rhs)


def load_vector(ref, h, f_q):
    """F[I] = (f, w_I)_K with f given at the nq*nq GL points of the element."""
    return ref.Phi.T @ (f_q * ref.wv * (h * h / 4.0))


class Problem:
    """Discrete HDG problem on the n x n mesh at degree p.

    kappa: per-element array [n*n] (e = i + n j), or a callable K(x, y)
           evaluated at the volume GL points (Sec. 5's variable coefficient).
    """

    def __init__(self, n, p, kappa, tau=1.0, nq=None):
        self.n, self.p, self.P, self.tau = n, p, p + 1, float(tau)
        self.h = 1.0 / n
        self.ref = RefOps(p, nq)
        self.kappa = kappa
        self.dofs = ms.element_dof_map(n, p)
        self.bdofs = ms.element_bdry_map(n, p)
        self.N = ms.n_trace_dofs(n, p)
        self._const = not callable(kappa)
        if self._const:
            self.kappa = np.asarray(kappa, dtype=np.float64).reshape(n * n)

    def inv_kappa_q(self, e):
        i, j = e % self.n, e // self.n
        if self._const:
            return np.full(self.ref.nq ** 2, 1.0 / self.kappa[e])
        X, Y = self.ref.volume_points(i, j, self.h)
        return 1.0 / self.kappa(X, Y)

    def element_mats(self, e):
        return local_matrices(self.ref, self.h, self.tau, self.inv_kappa_q(e))

    def element_block(self, e):
        """Condensed block Kc of element e (4P x 4P, local faces l, r, b, t)."""
        return condensed_block(*self.element_mats(e), self.tau)

    def all_blocks(self, elems=None):
        elems = range(self.n * self.n) if elems is None else elems
        return {e: self.element_block(e) for e in elems}

    def assemble(self, blocks=None):
        """Global trace matrix S = sum_K R_K^T Kc_K R_K over interior DoFs (CSR)."""
        rows, cols, vals = [], [], []
        for e in range(self.n * self.n):
            K = blocks[e] if blocks is not None else self.element_block(e)
            d = self.dofs[e]
            m = d >= 0
            dd = d[m]
            Ki = K[np.ix_(m, m)]
            rows.append(np.repeat(dd, len(dd)))
            cols.append(np.tile(dd, len(dd)))
            vals.append(Ki.reshape(-1))
        S = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(self.N, self.N)).tocsr()
        S.sum_duplicates()
        return S

    def boundary_trace(self, gD, nq_proj=None):
        """Lambda on boundary faces = P_h g_D, the edge-wise L2 projection (Sec. 3)."""
        n, P, h = self.n, self.P, self.h
        nqp = nq_proj if nq_proj is not None else max(self.ref.nq, self.p + 4)
        xq, wq = qd.gauss_legendre(nqp)
        L = qd.lagrange_matrix(self.ref.nodes, xq)
        Me = L.T @ (L * (wq * h / 2)[:, None])
        out = np.zeros(4 * n * P)
        if gD is None:
            return out
        for nb in range(4 * n):
            x0, t = ms.boundary_face_geometry(n, nb)
            pts = x0[None, :] + np.outer(0.5 * (1 + xq) * h, t)
            rhs = L.T @ (gD(pts[:, 0], pts[:, 1]) * wq * h / 2)
            out[nb * P:(nb + 1) * P] = np.linalg.solve(Me, rhs)
        return out

    def rhs(self, f_qp, gD=None, lam_bd=None):
        """b = sum_K R_K^T (g_K - Kc_K[:, bdry] Lambda_bdry) on interior DoFs.

        f_qp: [n*n, nq*nq] source values at the volume GL points."""
        if lam_bd is None:
            lam_bd = self.boundary_trace(gD)
        b = np.zeros(self.N)
        for e in range(self.n * self.n):
            A, B, C, D, E, M = self.element_mats(e)
            F = load_vector(self.ref, self.h, f_qp[e])
            g = source_flux(A, B, C, D, E, F)
            bd = self.bdofs[e]
            if np.any(bd >= 0):
                K = condensed_block(A, B, C, D, E, M, self.tau)
                lb = np.where(bd >= 0, lam_bd[np.maximum(bd, 0)], 0.0)
                g = g - K @ lb
            d = self.dofs[e]
            m = d >= 0
            np.add.at(b, d[m], g[m])
        return b

    def f_at_points(self, f):
        """Source values at the volume GL points of every element, [n*n, nq*nq]."""
        out = np.zeros((self.n * self.n, self.ref.nq ** 2))
        for e in range(self.n * self.n):
            X, Y = self.ref.volume_points(e % self.n, e // self.n, self.h)
            out[e] = f(X, Y)
        return out

    def solve_direct(self, b, S=None):
        """Step (iii): sparse direct solve of S Lambda = b (SuperLU)."""
        S = self.assemble() if S is None else S
        return spla.spsolve(S.tocsc(), b)

    def reconstruct(self, lam, f_qp, lam_bd):
        """Step (iv), eq. shur0: [Q; U]_K = Abb^{-1} ([0; F] - [C; E] Lambda_K)."""
        n2 = self.P * self.P
        Qs = np.zeros((self.n * self.n, 2 * n2))
        Us = np.zeros((self.n * self.n, n2))
        for e in range(self.n * self.n):
            A, B, C, D, E, M = self.element_mats(e)
            d, bd = self.dofs[e], self.bdofs[e]
            lk = np.where(d >= 0, lam[np.maximum(d, 0)], 0.0)
            lk = np.where(bd >= 0, lam_bd[np.maximum(bd, 0)], lk)
            F = load_vector(self.ref, self.h, f_qp[e])
            rhs = np.concatenate([np.zeros(2 * n2), F]) - np.vstack([C, E]) @ lk
            sol = np.linalg.solve(local_system(A, B, D), rhs)
            Qs[e], Us[e] = sol[:2 * n2], sol[2 * n2:]
        return Qs, Us

    def l2_errors(self, Qs, Us, u, q, nq_err=None):
        """||u - u_h||_L2 and ||q - q_h||_L2 by GL quadrature with nq_err >= p + 4 points (Sec. 5)."""
        nqe = nq_err if nq_err is not None else self.p + 5
        xq, wq = qd.gauss_legendre(nqe)
        L = qd.lagrange_matrix(self.ref.nodes, xq)
        Phi = np.einsum('ai,bj->baji', L, L).reshape(nqe * nqe, self.P ** 2)
        wv = np.outer(wq, wq).reshape(-1) * self.h ** 2 / 4
        n2 = self.P ** 2
        eu = eq = 0.0
        for e in range(self.n * self.n):
            i, j = e % self.n, e // self.n
            X = np.tile((i + 0.5 * (1 + xq)) * self.h, nqe)
            Y = np.repeat((j + 0.5 * (1 + xq)) * self.h, nqe)
            uh = Phi @ Us[e]
            qx, qy = Phi @ Qs[e, :n2], Phi @ Qs[e, n2:]
            qex = q(X, Y)
            eu += np.sum(wv * (u(X, Y) - uh) ** 2)
            eq += np.sum(wv * ((qex[0] - qx) ** 2 + (qex[1] - qy) ** 2))
        return np.sqrt(eu), np.sqrt(eq)
