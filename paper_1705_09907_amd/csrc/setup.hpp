// Host-side setup of the HDG trace operator and its multigrid hierarchy.
//
// Sec. 3 (eqs. static_1/static_2, shur0, shur1) gives, per element, the
// condensed block K_e = [C^T, -E^T] Abb^{-1} [C; E] + tau M.  Because the flux
// mass matrix is A = K_e^{-1} A0 with A0 independent of the element (uniform
// mesh, K constant per element), Q is eliminated in closed form and only the
// SPD system for U remains:
//     Z(K) = D + K G,  G = B A0^{-1} B^T,  R(K) = K H - E,  H = B A0^{-1} C,
//     K_e = tau M + K C^T A0^{-1} C - R^T Z^{-1} R,
//     g_e = R^T Z^{-1} F   (source flux of eq. shur0 with R = 0).
// G, H and C^T A0^{-1} C are built once per degree; each element costs one
// (p+1)^2 Cholesky factorization.
#pragma once
#include <cstdint>
#include <functional>
#include <string>
#include <vector>

namespace hdg {

using Vec = std::vector<double>;

// ---------------------------------------------------------------- 1D rules
void gauss_legendre(int nq, Vec& x, Vec& w);
Vec trace_nodes(int p);                       // GLL for p >= 1, {0} for p = 0
void lagrange_eval(const Vec& nodes, double x, double* l);   // l_j(x), product form
void lagrange_deriv(const Vec& nodes, double x, double* dl); // l_j'(x), product rule

// ------------------------------------------------------- reference matrices
struct RefDegree {
  int p = 0, P = 1;
  double h = 1.0, tau = 1.0;
  Vec M1;          // [P][P]  int l_i l_j on [-1, 1]
  Vec G;           // [P2][P2]
  Vec H;           // [P2][4P]
  Vec P1;          // [4P][4P]
  Vec Dm;          // [P2][P2]  tau-weighted edge mass of the volume basis
  Vec E;           // [P2][4P]
  Vec Mb;          // [4P][4P]  block diagonal edge mass of the trace basis (no tau)
  Vec C;           // [2 P2][4P] trace coupling of the flux equation (x half, then y half)
  Vec Bt;          // [2 P2][P2] B^T, B = divergence coupling of the U equation
  Vec Mvinv;       // [P2][P2]  inverse volume mass; A0^{-1} = diag(Mvinv, Mvinv)
  void build(int p, double h, double tau);
};

// Simultaneous diagonalisation of the pencil (G, D + G) (both symmetric, D + G
// SPD): V^T (D + G) V = I, V^T G V = diag(mu), V^T D V = diag(delta), so that
// for every coefficient K > 0   (D + K G)^{-1} = V diag(1 / (delta + K mu)) V^T.
// Element-local solves with the U system then need no per-element factorisation.
struct PencilRef {
  int P2 = 0;
  Vec V;           // [P2][P2], column i = eigenvector i
  Vec delta, mu;   // [P2]
};
PencilRef pencil_reference(const RefDegree& r);

// Condensed block of one element (4P x 4P row major) for coefficient kappa.
// work must hold at least P2*P2 + P2*4P doubles.
void element_block(const RefDegree& r, double kappa, double* K, double* work);
// Source flux g (4P) for load vector F (P2); same factorization as the block.
void element_source(const RefDegree& r, double kappa, const double* F, double* g, double* work);
// P_p [(p+1) x p]: degree-(p-1) nodal basis at the degree-p nodes.
Vec p_prolongation(int p);
// Kc = P4^T Kf P4 for one element (Kf: 4(p+1) square, Kc: 4p square).
void galerkin_block(const Vec& Pp, int p, const double* Kf, double* Kc);

// ------------------------------------------------------------ mesh helpers
inline int64_t n_faces(int n) { return 2LL * n * (n - 1); }
// interior face of local face lf of element (i, j), or -1
int64_t element_face(int n, int i, int j, int lf);
// the two elements of face f, and the local index of f in each
void face_elements(int n, int64_t f, int64_t& lo, int64_t& hi, int& lf_lo, int& lf_hi);

// Face-major block layout used by the device: per face 7 blocks of P x P,
// slot 0 = K_lo[f,f] + K_hi[f,f], slots 1-3 = K_lo[f, g] for the other local
// faces g of the lo element in increasing local order, slots 4-6 = K_hi[f, g]
// likewise; zero blocks where g is a boundary face.  Entries of a face are
// e = slot P^2 + a P + c; faces are grouped in tiles of 64, and entry pairs
// (2q, 2q+1) of the 64 faces of a tile are stored lane-interleaved:
// index = ((tile * E2/2 + q) * 64 + lane) * 2 + (e & 1), E2 = 7 P^2 rounded up
// to even.
int slab_pairs(int P);                       // E2 / 2
int64_t slab_doubles(int n, int P);
void other_faces(int lf, int out[3]);        // the 3 local faces != lf in increasing order

// parallel for over [0, n) with the hardware threads of the host
void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& body);

// ------------------------------------------------------------- Q1 hierarchy
struct Csr {
  int64_t nrows = 0, ncols = 0;
  std::vector<int64_t> ptr;
  std::vector<int64_t> col;
  Vec val;
};
Csr csr_transpose(const Csr& A);
Csr csr_multiply(const Csr& A, const Csr& B);
void csr_matvec(const Csr& A, const double* x, double* y);
Csr q1_bilinear(int m);                           // Q1 on mesh m/2 -> mesh m
Csr stencil_to_csr(int m, const Vec& st);         // st: [9][(m-1)^2]
Vec csr_to_stencil(int m, const Csr& A);          // inverse of the above
double lanczos_lmax(const Csr& A, const Vec& dinv, int steps);
bool cholesky_inverse(int N, Vec& A);             // SPD A (N x N) -> A^{-1} in place

}  // namespace hdg
