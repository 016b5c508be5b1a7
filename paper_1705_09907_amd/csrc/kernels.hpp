// Launchers of the gfx950 kernels (defined in kernels.hip).  All pointers are
// device pointers; every launch is asynchronous on `stream`.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace hdg {

// Operation fused into the face-owned gather y_f = sum of the two elements'
// block rows of face f times x (Sec. 8, Alg. algo_mv).
enum TraceMode : int {
  TM_APPLY = 0,          // y = S x
  TM_RESID = 1,          // y = b - S x
  TM_FACE_SWEEP = 2,     // y = x + omega Dinv (b - S x)        (facet Schwarz sweep)
  TM_RESID_RESTRICT = 3, // y = P_p^T (b - S x)  (coarse vector, p - 1)
  TM_APPLY_DOT = 4       // y = S x and per-workgroup partial sums of x . y
};

struct TraceArgs {
  const double* slab;    // face-major blocks (layout of setup.hpp)
  const double* x;
  const double* b;       // RESID / SWEEP / RESID_RESTRICT
  const double* dinv;    // SWEEP: face-block inverses, tile-pair layout
  double* y;
  double* partial;       // optional: per-wavefront sum of squares of (b - S x), or of x . y
  const double* pmat;    // RESID_RESTRICT: P_p [(p+1) x p], row major (device)
  double omega;
  int n;
  int64_t nf;            // interior faces
  int64_t ntiles;        // ceil(nf / 64)
};

int trace_grid(int64_t ntiles);      // workgroups of a trace launch
int trace_partials(int64_t ntiles);  // partial sums written when TraceArgs::partial is set (one per wavefront)
hipError_t launch_trace(int P, int mode, const TraceArgs& a, hipStream_t s);

// x = omega Dinv b (first facet sweep from a zero guess)
hipError_t launch_dinv_apply(int P, const double* dinv, const double* b, double omega, double* x,
                             int64_t nf, hipStream_t s);
// face-local p-transfers, P = p_fine + 1
hipError_t launch_p_restrict(int P, const double* pmat, const double* rf, double* rc, int64_t nf,
                             hipStream_t s);
hipError_t launch_p_prolong_add(int P, const double* pmat, const double* ec, double* xf, int64_t nf,
                                hipStream_t s);

// chain Schwarz: out = x + omega M^{-1} r (x == nullptr: out = omega M^{-1} r);
// M = block-tridiagonal matrix of each chain of faces, solved by block cyclic
// reduction with the factors of chain_factor_layout (api.cpp).  out may alias x.
struct ChainArgs {
  const double* factors;  // per chain: cstride doubles
  int64_t cstride;
  const double* r;
  const double* x;
  double* out;
  double omega;
  int n;
};
hipError_t launch_chain_solve(int P, const ChainArgs& a, hipStream_t s);

// Q1 levels: 9-point stencil st[9][Nv] on the interior vertices of an m x m mesh.
hipError_t launch_q1_resid(const double* st, const double* b, const double* x, double* r, int m,
                           hipStream_t s);
// Chebyshev step: z = dinv (b - A x); d = c1 d + c2 z; xo = x + d  (x == nullptr: x = 0)
hipError_t launch_q1_cheb(const double* st, const double* dinv, const double* b, const double* x,
                          double* d, double* xo, double c1, double c2, int m, hipStream_t s);
hipError_t launch_q1_restrict(const double* rf, double* rc, int m_fine, hipStream_t s);
hipError_t launch_q1_prolong_add(const double* ec, double* xf, int m_fine, hipStream_t s);
// p = 0 faces <-> Q1 vertices of the same mesh
hipError_t launch_pj_restrict(const double* rface, double* rv, int n, hipStream_t s);
hipError_t launch_pj_prolong_add(const double* ev, double* xface, int n, hipStream_t s);
// y = Ainv b, dense m x m row major
hipError_t launch_dense_gemv(const double* Ainv, const double* b, double* y, int m, hipStream_t s);

// deterministic reductions
int reduce_grid(int64_t n);
hipError_t launch_dot_partials(const double* a, const double* b, int64_t n, double* partial,
                               hipStream_t s);
hipError_t launch_sum_partials(const double* partial, int np, double* out, hipStream_t s);
// vector updates
hipError_t launch_axpy(double alpha, const double* x, double* y, int64_t n, hipStream_t s);   // y += a x
hipError_t launch_xpby(const double* x, double beta, double* y, int64_t n, hipStream_t s);    // y = x + b y
// r -= alpha q and per-workgroup sum of squares of the new r
hipError_t launch_axpy_norm(double alpha, const double* q, double* r, int64_t n, double* partial,
                            hipStream_t s);
hipError_t launch_copy(const double* x, double* y, int64_t n, hipStream_t s);
hipError_t launch_fill(double v, double* y, int64_t n, hipStream_t s);

}  // namespace hdg
