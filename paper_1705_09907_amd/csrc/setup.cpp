// Host-side setup: 1D rules, reference matrices, condensed element blocks,
// Galerkin p-coarsening, mesh maps, sparse helpers for the Q1 levels.
#include "setup.hpp"

#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <thread>

namespace hdg {

// ----------------------------------------------------------------- 1D rules
// Legendre P_n and P_n' by the three-term recurrence.
static void legendre(int n, double x, double& P, double& dP) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { P = 1.0; dP = 0.0; return; }
  for (int m = 2; m <= n; ++m) {
    double p2 = ((2.0 * m - 1.0) * x * p1 - (m - 1.0) * p0) / m;
    p0 = p1; p1 = p2;
  }
  P = p1;
  if (std::fabs(std::fabs(x) - 1.0) < 1e-15)
    dP = 0.5 * n * (n + 1) * ((n % 2 == 1 || x > 0) ? 1.0 : -1.0);
  else
    dP = n * (x * p1 - p0) / (x * x - 1.0);
}

void gauss_legendre(int nq, Vec& x, Vec& w) {
  x.assign(nq, 0.0); w.assign(nq, 0.0);
  for (int k = 0; k < nq; ++k) {
    // root k of P_nq, increasing order, Newton from the Chebyshev-like guess
    double t = -std::cos(M_PI * (k + 0.75) / (nq + 0.5));
    for (int it = 0; it < 100; ++it) {
      double P, dP; legendre(nq, t, P, dP);
      double dt = P / dP; t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    double P, dP; legendre(nq, t, P, dP);
    x[k] = t; w[k] = 2.0 / ((1.0 - t * t) * dP * dP);
  }
}

Vec trace_nodes(int p) {
  if (p == 0) return Vec{0.0};
  Vec x(p + 1);
  x[0] = -1.0; x[p] = 1.0;
  for (int k = 1; k < p; ++k) {
    // interior GLL node = root of P_p'; Newton with P_p'' from the Legendre ODE
    double t = -std::cos(M_PI * k / p);
    for (int it = 0; it < 100; ++it) {
      double P, dP; legendre(p, t, P, dP);
      double d2P = (2.0 * t * dP - p * (p + 1.0) * P) / (1.0 - t * t);
      double dt = dP / d2P; t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    x[k] = t;
  }
  return x;
}

void lagrange_eval(const Vec& nodes, double x, double* l) {
  const int P = (int)nodes.size();
  for (int j = 0; j < P; ++j) {
    double v = 1.0;
    for (int m = 0; m < P; ++m)
      if (m != j) v *= (x - nodes[m]) / (nodes[j] - nodes[m]);
    l[j] = v;
  }
}

void lagrange_deriv(const Vec& nodes, double x, double* dl) {
  const int P = (int)nodes.size();
  for (int j = 0; j < P; ++j) {
    double s = 0.0;
    for (int i = 0; i < P; ++i) {
      if (i == j) continue;
      double v = 1.0 / (nodes[j] - nodes[i]);
      for (int m = 0; m < P; ++m)
        if (m != j && m != i) v *= (x - nodes[m]) / (nodes[j] - nodes[m]);
      s += v;
    }
    dl[j] = s;
  }
}

// -------------------------------------------------------------- dense helpers
// C[m x n] = A[m x k] B[k x n]
static void matmul(int m, int k, int n, const double* A, const double* B, double* C) {
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int l = 0; l < k; ++l) s += A[i * k + l] * B[l * n + j];
      C[i * n + j] = s;
    }
}

// In-place lower Cholesky of SPD A (N x N row major).  Returns false if not SPD.
static bool cholesky(int N, double* A) {
  for (int j = 0; j < N; ++j) {
    double d = A[j * N + j];
    for (int k = 0; k < j; ++k) d -= A[j * N + k] * A[j * N + k];
    if (!(d > 0.0)) return false;
    d = std::sqrt(d);
    A[j * N + j] = d;
    for (int i = j + 1; i < N; ++i) {
      double s = A[i * N + j];
      for (int k = 0; k < j; ++k) s -= A[i * N + k] * A[j * N + k];
      A[i * N + j] = s / d;
    }
  }
  return true;
}

// X <- L^{-1} X for X [N x m] (L lower from cholesky)
static void forward_sub(int N, const double* L, int m, double* X) {
  for (int i = 0; i < N; ++i) {
    const double inv = 1.0 / L[i * N + i];
    for (int c = 0; c < m; ++c) {
      double s = X[i * m + c];
      for (int k = 0; k < i; ++k) s -= L[i * N + k] * X[k * m + c];
      X[i * m + c] = s * inv;
    }
  }
}

// X <- L^{-T} X
static void backward_sub(int N, const double* L, int m, double* X) {
  for (int i = N - 1; i >= 0; --i) {
    const double inv = 1.0 / L[i * N + i];
    for (int c = 0; c < m; ++c) {
      double s = X[i * m + c];
      for (int k = i + 1; k < N; ++k) s -= L[k * N + i] * X[k * m + c];
      X[i * m + c] = s * inv;
    }
  }
}

// Column c of A^{-1} from the factor: L y = e_c, then L^T x = y.  Each column's
// operations are those (and in the order) of forward_sub / backward_sub on the
// identity, so the result is the same to the bit; but the columns run in
// parallel with contiguous inner loops (L^T is transposed once), where the
// all-columns sweep walks X down its columns: at N = 1900 that took 38 s,
// against under a second.
static void inverse_by_columns(int N, const double* L, double* X) {
  Vec Lt((size_t)N * N, 0.0);
  for (int i = 0; i < N; ++i)
    for (int k = i; k < N; ++k) Lt[(size_t)i * N + k] = L[(size_t)k * N + i];
  parallel_for(N, [&](int64_t c0, int64_t c1) {
    Vec y(N);
    for (int64_t c = c0; c < c1; ++c) {
      for (int i = 0; i < N; ++i) {
        const double inv = 1.0 / L[(size_t)i * N + i];
        double s = i == c ? 1.0 : 0.0;
        const double* Li = L + (size_t)i * N;
        for (int k = 0; k < i; ++k) s -= Li[k] * y[k];
        y[i] = s * inv;
      }
      for (int i = N - 1; i >= 0; --i) {
        const double inv = 1.0 / L[(size_t)i * N + i];
        double s = y[i];
        const double* Ti = Lt.data() + (size_t)i * N;
        for (int k = i + 1; k < N; ++k) s -= Ti[k] * y[k];
        y[i] = s * inv;
      }
      for (int i = 0; i < N; ++i) X[(size_t)i * N + c] = y[i];
    }
  });
}

// Cholesky factor of an SPD matrix with lower bandwidth bw (A[i][j] = 0 for
// |i - j| > bw): the factor keeps the band, so the loops of cholesky() run over
// the band only.  The terms skipped are exact zeros, so the factor is the one
// cholesky() computes, to the bit, in O(N bw^2) instead of O(N^3).
static bool cholesky_band(int N, int bw, double* A) {
  for (int j = 0; j < N; ++j) {
    const int k0 = std::max(0, j - bw);
    double d = A[(size_t)j * N + j];
    for (int k = k0; k < j; ++k) d -= A[(size_t)j * N + k] * A[(size_t)j * N + k];
    if (!(d > 0.0)) return false;
    d = std::sqrt(d);
    A[(size_t)j * N + j] = d;
    const int i1 = std::min(N - 1, j + bw);
    for (int i = j + 1; i <= i1; ++i) {
      double s = A[(size_t)i * N + j];
      for (int k = std::max(0, i - bw); k < j; ++k) s -= A[(size_t)i * N + k] * A[(size_t)j * N + k];
      A[(size_t)i * N + j] = s / d;
    }
    for (int i = i1 + 1; i < N; ++i) A[(size_t)i * N + j] = 0.0;
  }
  return true;
}

// Columns of A^{-1} from a banded factor (inverse_by_columns restricted to the
// band of L; the same operations on the nonzero terms, so the same result).
static void inverse_by_columns_band(int N, int bw, const double* L, double* X) {
  parallel_for(N, [&](int64_t c0, int64_t c1) {
    Vec y(N);
    for (int64_t c = c0; c < c1; ++c) {
      for (int i = 0; i < N; ++i) {
        const double inv = 1.0 / L[(size_t)i * N + i];
        double s = i == c ? 1.0 : 0.0;
        const double* Li = L + (size_t)i * N;
        for (int k = std::max(0, i - bw); k < i; ++k) s -= Li[k] * y[k];
        y[i] = s * inv;
      }
      for (int i = N - 1; i >= 0; --i) {
        const double inv = 1.0 / L[(size_t)i * N + i];
        double s = y[i];
        const int k1 = std::min(N - 1, i + bw);
        for (int k = i + 1; k <= k1; ++k) s -= L[(size_t)k * N + i] * y[k];
        y[i] = s * inv;
      }
      for (int i = 0; i < N; ++i) X[(size_t)i * N + c] = y[i];
    }
  });
}

bool cholesky_inverse(int N, Vec& A) {
  int bw = 0;  // lower bandwidth
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < i - bw; ++j)
      if (A[(size_t)i * N + j] != 0.0) {
        bw = i - j;
        break;
      }
  if (N > 64 && 4 * bw < N) {
    if (!cholesky_band(N, bw, A.data())) return false;
    Vec I((size_t)N * N, 0.0);
    inverse_by_columns_band(N, bw, A.data(), I.data());
    A.swap(I);
    return true;
  }
  if (!cholesky(N, A.data())) return false;
  Vec L(A);
  Vec I((size_t)N * N, 0.0);
  if (N > 64) {
    inverse_by_columns(N, L.data(), I.data());
  } else {
    for (int i = 0; i < N; ++i) I[(size_t)i * N + i] = 1.0;
    forward_sub(N, L.data(), N, I.data());
    backward_sub(N, L.data(), N, I.data());
  }
  A.swap(I);
  return true;
}

// ------------------------------------------------------- reference matrices
void RefDegree::build(int p_, double h_, double tau_) {
  p = p_; P = p + 1; h = h_; tau = tau_;
  const int P2 = P * P, F4 = 4 * P;
  const Vec nodes = trace_nodes(p);
  Vec xq, wq;
  const int nq = p + 2;  // exact for the degree-(2p+1) integrands of M1, K1
  gauss_legendre(nq, xq, wq);
  Vec l(P), dl(P);
  M1.assign(P * P, 0.0);
  Vec K1(P * P, 0.0);
  for (int q = 0; q < nq; ++q) {
    lagrange_eval(nodes, xq[q], l.data());
    lagrange_deriv(nodes, xq[q], dl.data());
    for (int i = 0; i < P; ++i)
      for (int j = 0; j < P; ++j) {
        M1[i * P + j] += wq[q] * l[i] * l[j];
        K1[i * P + j] += wq[q] * l[i] * dl[j];
      }
  }
  Vec Lm(P), Lp(P);
  lagrange_eval(nodes, -1.0, Lm.data());
  lagrange_eval(nodes, 1.0, Lp.data());
  Vec M1inv(M1);
  if (!cholesky_inverse(P, M1inv)) throw std::runtime_error("1D mass not SPD");

  const int PP = P;
  auto I2 = [PP](int a, int b) { return a + PP * b; };
  // B [P2][2 P2]; A0^{-1} = diag(Mv^{-1}, Mv^{-1}), Mv^{-1} = (4/h^2) M1^{-1} (x) M1^{-1}
  Vec B((size_t)P2 * 2 * P2), A0inv_blk((size_t)P2 * P2);
  for (int i2 = 0; i2 < P; ++i2) for (int i1 = 0; i1 < P; ++i1)
    for (int j2 = 0; j2 < P; ++j2) for (int j1 = 0; j1 < P; ++j1) {
      const int I = I2(i1, i2), J = I2(j1, j2);
      B[(size_t)I * 2 * P2 + J] = 0.5 * h * K1[i1 * P + j1] * M1[i2 * P + j2];
      B[(size_t)I * 2 * P2 + P2 + J] = 0.5 * h * M1[i1 * P + j1] * K1[i2 * P + j2];
      A0inv_blk[(size_t)I * P2 + J] = 4.0 / (h * h) * M1inv[i1 * P + j1] * M1inv[i2 * P + j2];
    }
  // edge moments T_lf[I][m] = <phi_I, mu_m>_lf
  const double nx[4] = {-1, 1, 0, 0}, ny[4] = {0, 0, -1, 1};
  Vec T((size_t)4 * P2 * P, 0.0);
  for (int i2 = 0; i2 < P; ++i2) for (int i1 = 0; i1 < P; ++i1)
    for (int m = 0; m < P; ++m) {
      const int I = I2(i1, i2);
      T[((size_t)0 * P2 + I) * P + m] = 0.5 * h * Lm[i1] * M1[i2 * P + m];
      T[((size_t)1 * P2 + I) * P + m] = 0.5 * h * Lp[i1] * M1[i2 * P + m];
      T[((size_t)2 * P2 + I) * P + m] = 0.5 * h * M1[i1 * P + m] * Lm[i2];
      T[((size_t)3 * P2 + I) * P + m] = 0.5 * h * M1[i1 * P + m] * Lp[i2];
    }
  C.assign((size_t)2 * P2 * F4, 0.0);
  E.assign((size_t)P2 * F4, 0.0);
  for (int lf = 0; lf < 4; ++lf)
    for (int I = 0; I < P2; ++I)
      for (int m = 0; m < P; ++m) {
        const double t = T[((size_t)lf * P2 + I) * P + m];
        C[(size_t)I * F4 + lf * P + m] = nx[lf] * t;
        C[(size_t)(P2 + I) * F4 + lf * P + m] = ny[lf] * t;
        E[(size_t)I * F4 + lf * P + m] = -tau * t;
      }
  Dm.assign((size_t)P2 * P2, 0.0);
  for (int i2 = 0; i2 < P; ++i2) for (int i1 = 0; i1 < P; ++i1)
    for (int j2 = 0; j2 < P; ++j2) for (int j1 = 0; j1 < P; ++j1) {
      const double v = Lm[i1] * Lm[j1] * M1[i2 * P + j2] + Lp[i1] * Lp[j1] * M1[i2 * P + j2] +
                       M1[i1 * P + j1] * Lm[i2] * Lm[j2] + M1[i1 * P + j1] * Lp[i2] * Lp[j2];
      Dm[(size_t)I2(i1, i2) * P2 + I2(j1, j2)] = tau * 0.5 * h * v;
    }
  Mb.assign((size_t)F4 * F4, 0.0);
  for (int lf = 0; lf < 4; ++lf)
    for (int a = 0; a < P; ++a)
      for (int c = 0; c < P; ++c) Mb[(size_t)(lf * P + a) * F4 + lf * P + c] = 0.5 * h * M1[a * P + c];
  // BA = B A0^{-1}  [P2][2 P2]
  Vec BA((size_t)P2 * 2 * P2, 0.0);
  for (int I = 0; I < P2; ++I)
    for (int half = 0; half < 2; ++half)
      for (int J = 0; J < P2; ++J) {
        double s = 0.0;
        for (int L = 0; L < P2; ++L)
          s += B[(size_t)I * 2 * P2 + half * P2 + L] * A0inv_blk[(size_t)L * P2 + J];
        BA[(size_t)I * 2 * P2 + half * P2 + J] = s;
      }
  Bt.assign((size_t)2 * P2 * P2, 0.0);
  for (int I = 0; I < P2; ++I)
    for (int J = 0; J < 2 * P2; ++J) Bt[(size_t)J * P2 + I] = B[(size_t)I * 2 * P2 + J];
  Mvinv = A0inv_blk;
  G.assign((size_t)P2 * P2, 0.0);
  matmul(P2, 2 * P2, P2, BA.data(), Bt.data(), G.data());
  H.assign((size_t)P2 * F4, 0.0);
  matmul(P2, 2 * P2, F4, BA.data(), C.data(), H.data());
  // P1 = C^T A0^{-1} C
  Vec AC((size_t)2 * P2 * F4, 0.0);
  for (int half = 0; half < 2; ++half)
    matmul(P2, P2, F4, A0inv_blk.data(), C.data() + (size_t)half * P2 * F4,
           AC.data() + (size_t)half * P2 * F4);
  Vec Ct((size_t)F4 * 2 * P2);
  for (int r = 0; r < 2 * P2; ++r)
    for (int c = 0; c < F4; ++c) Ct[(size_t)c * 2 * P2 + r] = C[(size_t)r * F4 + c];
  P1.assign((size_t)F4 * F4, 0.0);
  matmul(F4, 2 * P2, F4, Ct.data(), AC.data(), P1.data());
}

void element_block(const RefDegree& r, double kappa, double* K, double* work) {
  const int P2 = r.P * r.P, F4 = 4 * r.P;
  double* Z = work;               // P2 x P2
  double* W = work + P2 * P2;     // P2 x F4
  for (int i = 0; i < P2 * P2; ++i) Z[i] = r.Dm[i] + kappa * r.G[i];
  for (int i = 0; i < P2 * F4; ++i) W[i] = kappa * r.H[i] - r.E[i];
  if (!cholesky(P2, Z)) throw std::runtime_error("local U system not SPD");
  forward_sub(P2, Z, F4, W);
  for (int a = 0; a < F4; ++a)
    for (int b = 0; b < F4; ++b) {
      double s = 0.0;
      for (int l = 0; l < P2; ++l) s += W[l * F4 + a] * W[l * F4 + b];
      K[a * F4 + b] = r.tau * r.Mb[a * F4 + b] + kappa * r.P1[a * F4 + b] - s;
    }
}

void element_source(const RefDegree& r, double kappa, const double* F, double* g, double* work) {
  const int P2 = r.P * r.P, F4 = 4 * r.P;
  double* Z = work;
  double* u = work + P2 * P2;
  for (int i = 0; i < P2 * P2; ++i) Z[i] = r.Dm[i] + kappa * r.G[i];
  for (int i = 0; i < P2; ++i) u[i] = F[i];
  if (!cholesky(P2, Z)) throw std::runtime_error("local U system not SPD");
  forward_sub(P2, Z, 1, u);
  backward_sub(P2, Z, 1, u);
  for (int a = 0; a < F4; ++a) {
    double s = 0.0;
    for (int l = 0; l < P2; ++l) s += (kappa * r.H[l * F4 + a] - r.E[l * F4 + a]) * u[l];
    g[a] = s;
  }
}

// Cyclic Jacobi eigenvalue iteration for a symmetric N x N matrix (row major):
// on return A is diagonal (the eigenvalues) and W holds the eigenvectors as
// columns (Golub & Van Loan, Matrix Computations, Sec. 8.5).
static void jacobi_eigen(int N, Vec& A, Vec& W) {
  W.assign((size_t)N * N, 0.0);
  for (int i = 0; i < N; ++i) W[(size_t)i * N + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) (i == j ? diag : off) += A[(size_t)i * N + j] * A[(size_t)i * N + j];
    if (off <= 1e-30 * diag) return;
    for (int p = 0; p < N - 1; ++p)
      for (int q = p + 1; q < N; ++q) {
        const double apq = A[(size_t)p * N + q];
        if (apq == 0.0) continue;
        const double app = A[(size_t)p * N + p], aqq = A[(size_t)q * N + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < N; ++k) {  // A <- J^T A J
          const double akp = A[(size_t)k * N + p], akq = A[(size_t)k * N + q];
          A[(size_t)k * N + p] = c * akp - s * akq;
          A[(size_t)k * N + q] = s * akp + c * akq;
        }
        for (int k = 0; k < N; ++k) {
          const double apk = A[(size_t)p * N + k], aqk = A[(size_t)q * N + k];
          A[(size_t)p * N + k] = c * apk - s * aqk;
          A[(size_t)q * N + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < N; ++k) {
          const double wkp = W[(size_t)k * N + p], wkq = W[(size_t)k * N + q];
          W[(size_t)k * N + p] = c * wkp - s * wkq;
          W[(size_t)k * N + q] = s * wkp + c * wkq;
        }
      }
  }
  throw std::runtime_error("Jacobi eigenvalue iteration did not converge");
}

PencilRef pencil_reference(const RefDegree& r) {
  const int N = r.P * r.P;
  PencilRef out;
  out.P2 = N;
  Vec L((size_t)N * N);
  for (int i = 0; i < N * N; ++i) L[i] = r.Dm[i] + r.G[i];
  if (!cholesky(N, L.data())) throw std::runtime_error("D + G not SPD");
  // Gh = L^{-1} G L^{-T}
  Vec X(r.G);
  forward_sub(N, L.data(), N, X.data());  // L^{-1} G
  Vec Gh((size_t)N * N);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) Gh[(size_t)i * N + j] = X[(size_t)j * N + i];
  forward_sub(N, L.data(), N, Gh.data());  // L^{-1} (L^{-1} G)^T
  for (int i = 0; i < N; ++i)
    for (int j = i + 1; j < N; ++j) {  // symmetrise the rounding
      const double s = 0.5 * (Gh[(size_t)i * N + j] + Gh[(size_t)j * N + i]);
      Gh[(size_t)i * N + j] = Gh[(size_t)j * N + i] = s;
    }
  Vec W;
  jacobi_eigen(N, Gh, W);
  out.V = W;
  backward_sub(N, L.data(), N, out.V.data());  // V = L^{-T} W
  out.delta.assign(N, 0.0);
  out.mu.assign(N, 0.0);
  for (int i = 0; i < N; ++i) {  // delta_i = v_i^T D v_i, mu_i = v_i^T G v_i, computed directly
    double d = 0.0, g = 0.0;
    for (int a = 0; a < N; ++a)
      for (int b = 0; b < N; ++b) {
        const double w = out.V[(size_t)a * N + i] * out.V[(size_t)b * N + i];
        d += w * r.Dm[(size_t)a * N + b];
        g += w * r.G[(size_t)a * N + b];
      }
    out.delta[i] = std::max(d, 0.0);
    out.mu[i] = std::max(g, 0.0);
  }
  return out;
}

Vec p_prolongation(int p) {
  const Vec fine = trace_nodes(p), coarse = trace_nodes(p - 1);
  Vec out((size_t)(p + 1) * p);
  for (int a = 0; a <= p; ++a) lagrange_eval(coarse, fine[a], out.data() + (size_t)a * p);
  return out;
}

void galerkin_block(const Vec& Pp, int p, const double* Kf, double* Kc) {
  // Kf: 4(p+1) square, Kc: 4p square; P4 = blockdiag(Pp) [4(p+1) x 4p]
  const int Pf = p + 1, Pc = p, Ff = 4 * Pf, Fc = 4 * Pc;
  std::vector<double> T((size_t)Ff * Fc, 0.0);   // Kf P4
  for (int r = 0; r < Ff; ++r)
    for (int lf = 0; lf < 4; ++lf)
      for (int b = 0; b < Pc; ++b) {
        double s = 0.0;
        for (int a = 0; a < Pf; ++a) s += Kf[(size_t)r * Ff + lf * Pf + a] * Pp[(size_t)a * Pc + b];
        T[(size_t)r * Fc + lf * Pc + b] = s;
      }
  for (int lf = 0; lf < 4; ++lf)
    for (int b = 0; b < Pc; ++b)
      for (int c = 0; c < Fc; ++c) {
        double s = 0.0;
        for (int a = 0; a < Pf; ++a) s += Pp[(size_t)a * Pc + b] * T[(size_t)(lf * Pf + a) * Fc + c];
        Kc[(size_t)(lf * Pc + b) * Fc + c] = s;
      }
}

// --------------------------------------------------------------- mesh helpers
int64_t element_face(int n, int i, int j, int lf) {
  const int64_t nv = (int64_t)n * (n - 1);
  switch (lf) {
    case 0: return i >= 1 ? (int64_t)(i - 1) + (int64_t)(n - 1) * j : -1;
    case 1: return i <= n - 2 ? (int64_t)i + (int64_t)(n - 1) * j : -1;
    case 2: return j >= 1 ? nv + i + (int64_t)n * (j - 1) : -1;
    default: return j <= n - 2 ? nv + i + (int64_t)n * j : -1;
  }
}

void face_elements(int n, int64_t f, int64_t& lo, int64_t& hi, int& lf_lo, int& lf_hi) {
  const int64_t nv = (int64_t)n * (n - 1);
  if (f < nv) {
    const int64_t j = f / (n - 1), i = f % (n - 1) + 1;
    lo = (i - 1) + (int64_t)n * j; hi = i + (int64_t)n * j; lf_lo = 1; lf_hi = 0;
  } else {
    const int64_t g = f - nv, j = g / n + 1, i = g % n;
    lo = i + (int64_t)n * (j - 1); hi = i + (int64_t)n * j; lf_lo = 3; lf_hi = 2;
  }
}

void other_faces(int lf, int out[3]) {
  int c = 0;
  for (int g = 0; g < 4; ++g)
    if (g != lf) out[c++] = g;
}

int slab_pairs(int P) { return (7 * P * P + 1) / 2; }

int64_t slab_doubles(int n, int P) {
  const int64_t tiles = (n_faces(n) + 63) / 64;
  return tiles * slab_pairs(P) * 128;
}

void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& body) {
  int nt = (int)std::min<unsigned>(std::max(1u, std::thread::hardware_concurrency()), 32u);
  if (n < 64 || nt == 1) { body(0, n); return; }
  std::vector<std::thread> th;
  const int64_t chunk = (n + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) {
    const int64_t a = t * chunk, b = std::min<int64_t>(n, a + chunk);
    if (a >= b) break;
    th.emplace_back([&body, a, b] { body(a, b); });
  }
  for (auto& t : th) t.join();
}

// ---------------------------------------------------------------- sparse Q1
Csr csr_transpose(const Csr& A) {
  Csr T;
  T.nrows = A.ncols; T.ncols = A.nrows;
  T.ptr.assign(T.nrows + 1, 0);
  for (int64_t k = 0; k < (int64_t)A.col.size(); ++k) T.ptr[A.col[k] + 1]++;
  for (int64_t r = 0; r < T.nrows; ++r) T.ptr[r + 1] += T.ptr[r];
  T.col.resize(A.col.size()); T.val.resize(A.val.size());
  std::vector<int64_t> pos(T.ptr.begin(), T.ptr.end() - 1);
  for (int64_t r = 0; r < A.nrows; ++r)
    for (int64_t k = A.ptr[r]; k < A.ptr[r + 1]; ++k) {
      const int64_t d = pos[A.col[k]]++;
      T.col[d] = r; T.val[d] = A.val[k];
    }
  return T;
}

Csr csr_multiply(const Csr& A, const Csr& B) {
  Csr C;
  C.nrows = A.nrows; C.ncols = B.ncols;
  C.ptr.assign(C.nrows + 1, 0);
  std::vector<int64_t> mark(B.ncols, -1);
  std::vector<double> acc(B.ncols, 0.0);
  std::vector<int64_t> cols;
  for (int64_t r = 0; r < A.nrows; ++r) {
    cols.clear();
    for (int64_t k = A.ptr[r]; k < A.ptr[r + 1]; ++k) {
      const int64_t a = A.col[k];
      for (int64_t l = B.ptr[a]; l < B.ptr[a + 1]; ++l) {
        const int64_t c = B.col[l];
        if (mark[c] != r) { mark[c] = r; acc[c] = 0.0; cols.push_back(c); }
        acc[c] += A.val[k] * B.val[l];
      }
    }
    std::sort(cols.begin(), cols.end());
    for (int64_t c : cols) { C.col.push_back(c); C.val.push_back(acc[c]); }
    C.ptr[r + 1] = (int64_t)C.col.size();
  }
  return C;
}

void csr_matvec(const Csr& A, const double* x, double* y) {
  for (int64_t r = 0; r < A.nrows; ++r) {
    double s = 0.0;
    for (int64_t k = A.ptr[r]; k < A.ptr[r + 1]; ++k) s += A.val[k] * x[A.col[k]];
    y[r] = s;
  }
}

static inline int64_t q1_index(int m, int i, int j) {
  if (i <= 0 || j <= 0 || i >= m || j >= m) return -1;
  return (int64_t)(i - 1) + (int64_t)(m - 1) * (j - 1);
}

Csr q1_bilinear(int m) {
  const int mc = m / 2;
  Csr A;
  A.nrows = (int64_t)(m - 1) * (m - 1); A.ncols = (int64_t)(mc - 1) * (mc - 1);
  A.ptr.assign(A.nrows + 1, 0);
  for (int J = 1; J < m; ++J)
    for (int I = 1; I < m; ++I) {
      int xi[2], yi[2]; double wx[2], wy[2]; int nx = 0, ny = 0;
      if (I % 2 == 0) { xi[0] = I / 2; wx[0] = 1.0; nx = 1; }
      else { xi[0] = I / 2; xi[1] = I / 2 + 1; wx[0] = wx[1] = 0.5; nx = 2; }
      if (J % 2 == 0) { yi[0] = J / 2; wy[0] = 1.0; ny = 1; }
      else { yi[0] = J / 2; yi[1] = J / 2 + 1; wy[0] = wy[1] = 0.5; ny = 2; }
      std::vector<std::pair<int64_t, double>> e;
      for (int b = 0; b < ny; ++b)
        for (int a = 0; a < nx; ++a) {
          const int64_t c = q1_index(mc, xi[a], yi[b]);
          if (c >= 0) e.emplace_back(c, wx[a] * wy[b]);
        }
      std::sort(e.begin(), e.end());
      for (auto& pr : e) { A.col.push_back(pr.first); A.val.push_back(pr.second); }
      A.ptr[q1_index(m, I, J) + 1] = (int64_t)A.col.size();
    }
  return A;
}

Csr stencil_to_csr(int m, const Vec& st) {
  const int64_t Nv = (int64_t)(m - 1) * (m - 1);
  Csr A;
  A.nrows = A.ncols = Nv;
  A.ptr.assign(Nv + 1, 0);
  for (int j = 1; j < m; ++j)
    for (int i = 1; i < m; ++i) {
      const int64_t v = q1_index(m, i, j);
      for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di) {
          const int64_t c = q1_index(m, i + di, j + dj);
          const double a = st[(size_t)((di + 1) + 3 * (dj + 1)) * Nv + v];
          if (c >= 0 && a != 0.0) { A.col.push_back(c); A.val.push_back(a); }
        }
      A.ptr[v + 1] = (int64_t)A.col.size();
    }
  return A;
}

Vec csr_to_stencil(int m, const Csr& A) {
  const int64_t Nv = (int64_t)(m - 1) * (m - 1);
  Vec st((size_t)9 * Nv, 0.0);
  for (int64_t v = 0; v < Nv; ++v) {
    const int i = (int)(v % (m - 1)) + 1, j = (int)(v / (m - 1)) + 1;
    for (int64_t k = A.ptr[v]; k < A.ptr[v + 1]; ++k) {
      const int64_t c = A.col[k];
      const int ci = (int)(c % (m - 1)) + 1, cj = (int)(c / (m - 1)) + 1;
      const int di = ci - i, dj = cj - j;
      if (std::abs(di) > 1 || std::abs(dj) > 1) throw std::runtime_error("Q1 operator not 9-point");
      st[(size_t)((di + 1) + 3 * (dj + 1)) * Nv + v] += A.val[k];
    }
  }
  return st;
}

double lanczos_lmax(const Csr& A, const Vec& dinv, int steps) {
  const int64_t N = A.nrows;
  Vec v(N), z(N), w(N), vold(N, 0.0);
  for (int64_t i = 0; i < N; ++i) v[i] = 1.0 + 0.25 * std::cos(0.7 * (double)i);
  double beta = 0.0;
  for (int64_t i = 0; i < N; ++i) { z[i] = dinv[i] * v[i]; beta += v[i] * z[i]; }
  beta = std::sqrt(beta);
  for (int64_t i = 0; i < N; ++i) { v[i] /= beta; z[i] /= beta; }
  std::vector<double> al, be;
  double bprev = 0.0;
  for (int s = 0; s < steps && s < N; ++s) {
    csr_matvec(A, z.data(), w.data());
    double a = 0.0;
    for (int64_t i = 0; i < N; ++i) a += w[i] * z[i];
    double bn = 0.0;
    for (int64_t i = 0; i < N; ++i) {
      w[i] -= a * v[i] + bprev * vold[i];
      bn += w[i] * dinv[i] * w[i];
    }
    bn = std::sqrt(std::max(bn, 0.0));
    al.push_back(a);
    if (bn < 1e-14 * std::fabs(a)) break;
    be.push_back(bn);
    for (int64_t i = 0; i < N; ++i) { vold[i] = v[i]; v[i] = w[i] / bn; z[i] = dinv[i] * v[i]; }
    bprev = bn;
  }
  // largest eigenvalue of the tridiagonal matrix by bisection (Sturm count)
  const int m = (int)al.size();
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? std::fabs(be[i - 1]) : 0.0) + (i < m - 1 ? std::fabs(be[i]) : 0.0);
    lo = std::min(lo, al[i] - r); hi = std::max(hi, al[i] + r);
  }
  auto count_below = [&](double x) {
    int c = 0; double d = 1.0;
    for (int i = 0; i < m; ++i) {
      const double b2 = i > 0 ? be[i - 1] * be[i - 1] : 0.0;
      d = al[i] - x - (i > 0 ? b2 / d : 0.0);
      if (d == 0.0) d = 1e-300;
      if (d < 0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (count_below(mid) >= m) hi = mid; else lo = mid;
  }
  return hi;
}

}  // namespace hdg
