// Launchers of the gfx950 kernels (defined in kernels.hip).  All pointers are
// device pointers; every launch is asynchronous on `stream`.
//
// Precision: vectors are FP64 (Prec::F64) or FP32 (Prec::F32, Prec::BF16);
// block matrices are stored in FP64, FP32 or BF16 respectively and accumulated
// in the vector type.  Pointers to vectors and matrices are untyped here and
// interpreted by the precision passed to each launcher.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace hdg {

enum class Prec : int { F64 = 0, F32 = 1, BF16 = 2 };
inline size_t vec_bytes(Prec p) { return p == Prec::F64 ? 8 : 4; }      // vector element
inline size_t mat_bytes(Prec p) { return p == Prec::F64 ? 8 : (p == Prec::F32 ? 4 : 2); }
inline int mat_lanes16(Prec p) { return (int)(16 / mat_bytes(p)); }      // entries per 16-byte load

// Operation fused into the face-owned gather y_f = sum of the two elements'
// block rows of face f times x (Sec. 8, Alg. algo_mv).
enum TraceMode : int {
  TM_APPLY = 0,          // y = S x
  TM_RESID = 1,          // y = b - S x
  TM_FACE_SWEEP = 2,     // y = x + omega Dinv (b - S x)        (facet Schwarz sweep)
  TM_RESID_RESTRICT = 3, // y = P_p^T (b - S x)  (coarse vector, p - 1)
  TM_APPLY_DOT = 4,      // y = S x and per-wavefront partial sums of x . y
  TM_ABS = 5,            // y = |S| |x| entrywise (FP64 only): the rounding scale of S x
  TM_UPDATE = 6          // y = b + omega S x (b nullable: 0); y may alias b (element-patch Schwarz)
};

struct TraceArgs {
  const void* slab;      // face-major blocks (layout of setup.hpp), matrix precision
  const void* x;
  const void* b;         // RESID / SWEEP / RESID_RESTRICT
  const void* dinv;      // SWEEP: face-block inverses, same interleaved layout
  void* y;
  double* partial;       // optional: per-wavefront sum of squares of (b - S x), or of x . y (FP64)
  const void* pmat;      // RESID_RESTRICT: P_p [(p+1) x p], row major, vector precision
  double omega;
  int n;
  int64_t nf;            // interior faces
  int64_t ntiles;        // ceil(nf / 64)
  void* ev_start;        // TM_APPLY: optional hipEvent_t pair recorded at the kernel's start / end
  void* ev_stop;
};

int trace_grid(int64_t ntiles);      // workgroups of a trace launch
int trace_partials(int64_t ntiles);  // partial sums written when TraceArgs::partial is set
hipError_t launch_trace(Prec pr, int P, int mode, const TraceArgs& a, hipStream_t s);

// Y = S X for nrhs right-hand sides at once; X, Y [nf P][nrhs] (right-hand
// sides contiguous), vector precision.  The blocks of a group of faces are read
// once into LDS and applied to every right-hand side.
struct MultiArgs {
  const void* slab;
  const void* X;
  void* Y;               // APPLY / RESID: [nf P][nrhs]; RESID_RESTRICT: [nf (P-1)][nrhs]
  const void* B;         // RESID, RESID_RESTRICT
  const void* pmat;      // RESID_RESTRICT: P_p, vector precision
  int nrhs;
  int n;
  int64_t nf, ntiles;
  int remap;   // XCD-contiguous group order
  int kernel;  // FP32 / bfloat16 blocks: 0 vector kernel, 1 matrix-core kernel (FP64 always vector)
};
// mode: TM_APPLY (Y = S X), TM_RESID (Y = B - S X) or TM_RESID_RESTRICT
// (Y = P_p^T (B - S X) on the coarse level)
hipError_t launch_trace_multi(Prec pr, int P, const MultiArgs& a, hipStream_t s, int mode = TM_APPLY);

// y_m = S_m x_m for many meshes in one launch: a fixed grid walks the
// (mesh, tile) items; tile0 = first item of the mesh (prefix sum of ntiles).
// mp: the block storage (Prec) of slab; FP64 blocks go with FP64 vectors, FP32
// and bfloat16 blocks with FP32 vectors.
struct BatchMesh {
  const void* slab;
  const void* x;
  void* y;
  int64_t nf, ntiles, tile0;
  int n, P;
  int mp;
};
// Allocation-free variant: the descriptor table lives in a file-scope device
// array of kBatchNoallocMax entries (one per GPU); batch_scratch_address returns
// its device address on the current device (looked up once per device).
constexpr int kBatchNoallocMax = 256;
constexpr int kMaxDevices = 64;
hipError_t batch_scratch_address(void** out);
// pmax: the largest P in the batch (selects the register budget); lp: every
// mesh has FP32 or bfloat16 blocks and FP32 vectors (else FP64 throughout)
hipError_t launch_trace_batch(const BatchMesh* meshes_dev, int nmesh, int64_t total_tiles, int grid, int pmax,
                              hipStream_t s, bool lp = false);

// x = omega Dinv b (first facet sweep from a zero guess)
hipError_t launch_dinv_apply(Prec pr, int P, const void* dinv, const void* b, double omega, void* x,
                             int64_t nf, hipStream_t s);
// face-local p-transfers, P = p_fine + 1, P_p in vector precision
hipError_t launch_p_restrict(Prec pr, int P, const void* pmat, const void* rf, void* rc, int64_t nf,
                             hipStream_t s);
hipError_t launch_p_prolong_add(Prec pr, int P, const void* pmat, const void* ec, void* xf, int64_t nf,
                                hipStream_t s);

// chain Schwarz: out = x + omega M^{-1} r (x == nullptr: out = omega M^{-1} r);
// M = block-tridiagonal matrix of each chain of faces, solved by block cyclic
// reduction with the factors built in api.cpp (vector precision).  out may alias x.
struct ChainArgs {
  const void* factors;  // per chain: cstride entries
  int64_t cstride;
  const void* r;
  const void* x;
  void* out;
  double omega;
  int n;
  int threads;          // workgroup size; 0 = chain_threads(P, n)
  int lds_level;        // factors of levels >= lds_level are staged in LDS (chain_lds_level)
  int remap;            // 1: XCD-aware chain order (consecutive chains on one XCD)
  int64_t lds_cap;      // LDS bytes a workgroup may use on this device (0: 64 KiB)
  int shape;            // 0 by the mesh, 1 lean, 2 wide, 3 flat, 4 partitioned (chain_shape_kind)
  const void* tri;      // shape 4: the partitioned solve's factors
  // shape 4 with r == null and these set: the right-hand side is the residual
  // b - S x, computed in the launch from the level's face slab (P = 1, stored in
  // the vector precision: FP64 or FP32 cycles, not bfloat16 slabs) and x
  const void* b;
  const void* slab;
};
int chain_threads(int P, int n);
int chain_flat_threads(int P, int n);            // workgroup size of the flat schedule (0: none at P)
int chain_shape_kind(int P, int n, int shape);   // the kind ChainArgs::shape selects (0: not available)
int chain_max_threads(int P, bool wide);         // launch bound of the chain kernel at P
int chain_remap(int P);
// first level whose factors (and all later ones) fit in `budget` bytes of LDS
// LDS of one workgroup on gfx950 (the chain solves keep a whole chain there)
constexpr int64_t kMaxLdsBytes = 160 * 1024;
int chain_lds_level(int P, int n, size_t elem_bytes, int64_t budget);
// dynamic LDS of a chain launch: right-hand side plus the staged factors
size_t chain_lds_bytes(int P, int n, size_t elem_bytes, int lds_level);
hipError_t launch_chain_solve(Prec pr, int P, const ChainArgs& a, hipStream_t s);
// Partitioned tridiagonal solve of the P = 1 chains (ChainArgs::shape 4): one
// wavefront per chain, one segment of >= 2 positions per lane; its factors
// (ChainArgs::tri, chain_tri_stride(n) entries per chain) come from
// launch_chain_tri_factor.  chain_tri_lmax: register bound of a segment's
// length (4, 8, 16 or 32), 0 where the schedule is not available (n < 5 or
// n > 2049).
constexpr int kTriScalars = 20;
int chain_tri_lmax(int n);
int64_t chain_tri_stride(int n);
size_t chain_tri_lds_bytes(int n, int chains_per_wg, size_t elem_bytes);
hipError_t launch_chain_tri_factor(Prec vp, const double* EB, int n, void* tri, int* fail, hipStream_t s);

// Q1 levels (vector precision): 9-point stencil st[9][Nv] on the interior
// vertices of an m x m mesh.
hipError_t launch_q1_resid(Prec pr, const void* st, const void* b, const void* x, void* r, int m,
                           hipStream_t s);
// Chebyshev step: z = dinv (b - A x); d = c1 d + c2 z; xo = x + d  (x == nullptr: x = 0)
hipError_t launch_q1_cheb(Prec pr, const void* st, const void* dinv, const void* b, const void* x,
                          void* d, void* xo, double c1, double c2, int m, hipStream_t s);
hipError_t launch_q1_restrict(Prec pr, const void* rf, void* rc, int m_fine, hipStream_t s);
hipError_t launch_q1_prolong_add(Prec pr, const void* ec, void* xf, int m_fine, hipStream_t s);
// the cycle kernels above read the symmetric 5-entry stencil st[5][Nv]
// (directions 4 ... 8, launch_q1_finish); this one the set-up's FP64 st[9][Nv]
hipError_t launch_q1_resid9(const double* st, const double* b, const double* x, double* r, int m, hipStream_t s);

// Fused Q1 level visits: launch_q1_pre does nu Chebyshev steps from x_in (null:
// zero), writes the iterate to x_out and the restricted residual to bc;
// launch_q1_post adds the prolonged coarse correction ec to x_in, does nu steps
// and writes x_out.  x_out must not alias x_in.  m even, 1 <= nu <= kQ1MaxNu,
// tile from q1_fused_tile(m).  Same arithmetic as the one-operation kernels.
constexpr int kQ1MaxNu = 6;
constexpr int kQ1Threads = 256;
struct Q1FusedArgs {
  const void* st = nullptr;
  const void* dinv = nullptr;
  const void* b = nullptr;
  const void* x_in = nullptr;
  void* x_out = nullptr;
  const void* ec = nullptr;
  void* bc = nullptr;
  int m = 0;
  int nu = 0;
  int tile = 0;
  double c1[kQ1MaxNu] = {};
  double c2[kQ1MaxNu] = {};
};
int q1_fused_tile(int m);
hipError_t launch_q1_pre(Prec pr, const Q1FusedArgs& a, hipStream_t s);
hipError_t launch_q1_post(Prec pr, const Q1FusedArgs& a, hipStream_t s);
// p = 0 faces <-> Q1 vertices of the same mesh
hipError_t launch_pj_restrict(Prec pr, const void* rface, void* rv, int n, hipStream_t s);
hipError_t launch_pj_prolong_add(Prec pr, const void* ev, void* xface, int n, hipStream_t s);
// y = Ainv b with an FP64 dense m x m inverse; b, y in vector precision
hipError_t launch_dense_gemv(Prec pr, const double* Ainv, const void* b, void* y, int m, hipStream_t s);

// Element-local kernels of the misfit gradient (FP64), one wavefront per element.
// ref packs the degree-k reference data: V [P2][P2] (column i = eigenvector i of
// the pencil (G, D + G)), delta [P2], mu [P2], E [P2][4P], H [P2][4P],
// C [2 P2][4P], Bt [2 P2][P2], Mvinv [P2][P2]; so that for element coefficient K
// (D + K G)^{-1} = V diag(1 / (delta + K mu)) V^T.
struct ElemArgs {
  const double* ref;
  const double* kappa;    // [n n]
  const double* lam;      // trace vector, interior faces
  const double* lam_bd;   // [4 n][P] boundary traces (bottom, right, top, left)
  const double* F;        // [n n][P2] load vectors
  const double* U;        // [n n][P2]
  const double* Uobs;     // [n n][P2]
  const double* mu;       // adjoint trace vector, interior faces
  double* Uout;           // reconstruct: U
  double* Qout;           // reconstruct: Q [n n][2 P2] (nullable)
  double* tout;           // adjoint: element trace contributions [n n][4P]
  double* misfit;         // adjoint: 1/2 |U - Uobs|^2 per element [n n]
  double* grad;           // gradient: dL/dtheta per element [n n]
  int n;
};
// U = (D + K G)^{-1} (F - (E - K H) Lambda_K), Q = K A0^{-1} (B^T U - C Lambda_K)
hipError_t launch_elem_reconstruct(int P, const ElemArgs& a, hipStream_t s);
// t_K = -(E - K H)^T (D + K G)^{-1} (U_K - Uobs_K), misfit_K = 1/2 |U_K - Uobs_K|^2
hipError_t launch_elem_adjoint(int P, const ElemArgs& a, hipStream_t s);
// c_f = t_lo[f] + t_hi[f] on interior faces (face-owned gather of element rows)
hipError_t launch_face_gather(int P, const double* t, double* c, int n, hipStream_t s);
// grad_K = K (C mu_K - B^T w)^T A0^{-1} (B^T U_K - C Lambda_K),
//          w = (D + K G)^{-1} (U_K - Uobs_K - (E - K H) mu_K)
hipError_t launch_elem_gradient(int P, const ElemArgs& a, hipStream_t s);

// ---- many right-hand sides (multi.hip): vectors [rows][R], vector precision
hipError_t launch_p_restrict_m(Prec pr, int P, const void* pm, const void* rf, void* rc, int64_t nf, int R,
                               hipStream_t s);
hipError_t launch_p_prolong_add_m(Prec pr, int P, const void* pm, const void* ec, void* xf, int64_t nf, int R,
                                  hipStream_t s);
hipError_t launch_q1_resid_m(Prec pr, const void* st, const void* b, const void* x, void* r, int m, int R,
                             hipStream_t s);
hipError_t launch_q1_cheb_m(Prec pr, const void* st, const void* dinv, const void* b, const void* x, void* d,
                            void* xo, double c1, double c2, int m, int R, hipStream_t s);
hipError_t launch_q1_restrict_m(Prec pr, const void* rf, void* rc, int mf, int R, hipStream_t s);
hipError_t launch_q1_prolong_add_m(Prec pr, const void* ec, void* xf, int mf, int R, hipStream_t s);
hipError_t launch_pj_restrict_m(Prec pr, const void* rface, void* rv, int n, int R, hipStream_t s);
hipError_t launch_pj_prolong_add_m(Prec pr, const void* ev, void* xface, int n, int R, hipStream_t s);
hipError_t launch_dense_gemm_m(Prec pr, const double* A, const void* b, void* y, int m, int R, hipStream_t s);
struct ChainMultiArgs {
  const void* factors;
  int64_t cstride;
  const void* r;
  const void* x;     // nullptr: out = omega M^{-1} r
  void* out;         // may alias x
  double omega;
  int n;
  int R;             // right-hand sides (row stride of r, x, out)
  int rc;            // right-hand sides per workgroup (chain_multi_chunk)
  int nchunks;       // ceil(R / rc)
  int threads;       // workgroup size (0: smallest of 256, 512, 1024 that fits the items)
  int64_t lds_cap;   // LDS bytes a workgroup may use on this device (0: 64 KiB)
};
// Largest power-of-two chunk of columns for the chain solve; 0 if one column
// does not fit lds_cap bytes of LDS.
int chain_multi_chunk(int P, int n, int R, size_t elem_bytes, int64_t lds_cap);
hipError_t launch_chain_solve_m(Prec pr, int P, const ChainMultiArgs& a, hipStream_t s);
// out[r] = sum_i x[i][r] y[i][r] (FP64, deterministic); partial needs dots_m_grid(N) * R
int dots_m_grid(int64_t N);
hipError_t launch_dots_m(Prec pr, const void* x, const void* y, int64_t N, int R, double* partial, double* out,
                         hipStream_t s);
// y[i][r] += sign act[r] num[r] / den[r] x[i][r]  (ratio 0 when den[r] is not > 0; act may be null)
hipError_t launch_axpy_m(Prec pr, const double* num, const double* den, const double* act, double sign,
                         const void* x, void* y, int64_t N, int R, hipStream_t s);
// y[i][r] = x[i][r] + sign num[r] / den[r] y[i][r]
hipError_t launch_xpby_m(Prec pr, const void* x, const double* num, const double* den, double sign, void* y,
                         int64_t N, int R, hipStream_t s);
// sc = [5][R]: sc[0][r] = sc[3][r] - (sc[2][r] / sc[1][r]) sc[4][r]
hipError_t launch_fcg_scalars_m(double* sc, int R, hipStream_t s);

// ---- device setup (setup_dev.hip)
// Reference matrices of one degree for the element-block generator (FP64,
// device): pencil basis V [P2][P2] (column i), delta, mu [P2], the local U
// system D [P2][P2] and G [P2][P2], H [P2][4P], E [P2][4P], the trace mass Mb
// [4P][4P] and C^T A0^{-1} C [4P][4P]; so that with W = kappa H - E
//   K_e = tau Mb + kappa P1 - W^T (D + kappa G)^{-1} W.
struct ElemGenRef {
  const double *V, *delta, *mu, *Dm, *G, *H, *E, *Mb, *P1;
  double tau;
};
// EB [ne][4P][4P]: condensed blocks of every element (one thread per column)
hipError_t launch_elem_rows(int P, const ElemGenRef& r, const double* kappa, double* EB, int64_t ne, hipStream_t s);
// Kc = P4^T Kf P4 per element (P4 = blockdiag(Pp), Pp [Pfine x (Pfine - 1)])
hipError_t launch_elem_galerkin(int Pfine, const double* Pp, const double* Kf, double* Kc, int64_t ne,
                                hipStream_t s);
// face-major slab of level P from the element blocks, in matrix precision mp
// (zero padding included); slab64 (optional, mp != F64): the FP64 copy
hipError_t launch_pack_slab(Prec mp, int P, const double* EB, int n, int64_t nf, void* slab, double* slab64,
                            hipStream_t s);
// facet inverses in the slab layout (P^2 entries per face); *fail = 1 if a block is not SPD
hipError_t launch_face_dinv(Prec mp, int P, const double* EB, int n, int64_t nf, void* dinv, int* fail,
                            hipStream_t s);
// element-patch Schwarz: MB[e] = (R_e S R_e^T)^{-1} on the interior faces of element
// e (rows and columns of boundary faces zero), [ne][4P][4P]; *fail = 1 if not SPD
hipError_t launch_patch_inverse(int P, const double* EB, int n, double* MB, int* fail, hipStream_t s);
// chain cyclic-reduction factors of chains [chain0, chain0 + nchains), records
// in vector precision vp; work: nchains * chain_factor_work_doubles(P, n)
int64_t chain_factor_work_doubles(int P, int n);
hipError_t launch_chain_factor(Prec vp, int P, const double* EB, int n, int64_t chain0, int nchains, double* work,
                               void* fac, int64_t cstride, int* fail, hipStream_t s);
// Q1 stencils [9][Nv] (FP64): from the p = 0 blocks, Galerkin coarsening, and
// the cycle copies (vector precision stencil, 1 / diagonal, FP64 1 / diagonal)
hipError_t launch_q1_stencil0(const double* EB0, int n, double* st, hipStream_t s);
hipError_t launch_q1_galerkin(const double* stf, int mf, double* stc, hipStream_t s);
hipError_t launch_q1_finish(Prec vp, const double* st64, int64_t Nv, void* st, void* dinv, double* dinv64,
                            hipStream_t s);
hipError_t launch_vmul(const double* a, const double* b, double* out, int64_t n, hipStream_t s);  // out = a .* b

// deterministic reductions (FP64 vectors)
int reduce_grid(int64_t n);
hipError_t launch_dot_partials(const double* a, const double* b, int64_t n, double* partial,
                               hipStream_t s);
hipError_t launch_sum_partials(const double* partial, int np, double* out, hipStream_t s);
// up to three dot products x_j . y_j of vectors in precision pr, FP64 partials
// (dot j at partial[j * reduce_grid(n) + i]); the multi-sum writes out[j]
struct DotArgs {
  const void* x[3];
  const void* y[3];
  int ndots;
};
hipError_t launch_dots(Prec pr, const DotArgs& a, int64_t n, double* partial, hipStream_t s);
hipError_t launch_sum_partials_multi(const double* partial, int np, int ndots, double* out, hipStream_t s);
// vector updates (FP64, or vector precision pr)
hipError_t launch_axpy(double alpha, const double* x, double* y, int64_t n, hipStream_t s);   // y += a x
hipError_t launch_xpby(const double* x, double beta, double* y, int64_t n, hipStream_t s);    // y = x + b y
hipError_t launch_axpy(Prec pr, double alpha, const void* x, void* y, int64_t n, hipStream_t s);
hipError_t launch_xpby(Prec pr, const void* x, double beta, void* y, int64_t n, hipStream_t s);
hipError_t launch_zero(Prec pr, void* y, int64_t n, hipStream_t s);
// Updates whose coefficient is a ratio of device scalars, c = sign sc[num] / sc[den]
// (c = 0 when sc[den] is not > 0 or the ratio is not finite): no host round trip.
hipError_t launch_axpy_dev(Prec pr, const double* sc, int num, int den, double sign, const void* x, void* y,
                           int64_t n, hipStream_t s);                                          // y += c x
hipError_t launch_xpby_dev(Prec pr, const void* x, const double* sc, int num, int den, double sign, void* y,
                           int64_t n, hipStream_t s);                                          // y = x + c y
// Flexible-CG direction scalars on the device: with sc[1] = d.q, sc[2] = z.q,
// sc[3] = z.r, sc[4] = d.r:  sc[0] = sc[3] - (sc[2] / sc[1]) sc[4]  (the new d.r)
hipError_t launch_fcg_scalars(double* sc, hipStream_t s);
// e += (sc[0] / sc[1]) d and, when r is not null, r -= (sc[0] / sc[1]) q
hipError_t launch_fcg_update(Prec pr, const double* sc, const void* d, void* e, const void* q, void* r, int64_t n,
                             hipStream_t s);
// the three dots of a flexible CG step (sums into sc[2..4]) and sc[0] as
// launch_fcg_scalars, in one launch
hipError_t launch_sum_partials_fcg(const double* partial, int np, double* sc, hipStream_t s);
// r -= alpha q and per-workgroup sum of squares of the new r
hipError_t launch_axpy_norm(double alpha, const double* q, double* r, int64_t n, double* partial,
                            hipStream_t s);
// copies in vector precision, conversions between FP64 and FP32
hipError_t launch_copy(Prec pr, const void* x, void* y, int64_t n, hipStream_t s);
hipError_t launch_fill(double v, double* y, int64_t n, hipStream_t s);
hipError_t launch_to_f32(const double* x, float* y, int64_t n, hipStream_t s);
hipError_t launch_to_f64(const float* x, double* y, int64_t n, hipStream_t s);

}  // namespace hdg
