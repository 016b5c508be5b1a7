// Device (gfx950) setup of the trace operator and its multigrid hierarchy.
//
// The condensed element blocks of Sec. 3 (eq. shur0 substituted into shur1),
//   K_e = tau M + kappa C^T A0^{-1} C - W^T (D + kappa G)^{-1} W,  W = kappa H - E,
// are generated for every element at once (Sec. 8 notes that the local solves
// are independent and compute bound).  One thread forms one column of one
// element's block: the local U system (D + kappa G) x = W[:, c] is solved with
// the pencil basis V of the degree's reference matrices,
// (D + kappa G)^{-1} = V diag(1 / (delta + kappa mu)) V^T, followed by one step
// of iterative refinement against the explicit D + kappa G (the pencil alone
// loses accuracy at small kappa, where D + kappa G is ill conditioned); K is
// symmetric, so the column is also the row.  Coarse p-levels are then P4^T K P4
// element by element, and the face-major slabs, facet inverses, chain
// cyclic-reduction factors and the Q1 hierarchy are built from those blocks on
// the device.  Nothing here depends on the host beyond the small reference
// matrices and the coarsest Q1 inverse.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "kernels.hpp"

namespace hdg {

static constexpr int kSW = 256;

#define HDG_SETUP_DISPATCH_P(P, CALL)                 \
  switch (P) {                                        \
    case 1: { constexpr int PP = 1; CALL; } break;    \
    case 2: { constexpr int PP = 2; CALL; } break;    \
    case 3: { constexpr int PP = 3; CALL; } break;    \
    case 4: { constexpr int PP = 4; CALL; } break;    \
    case 5: { constexpr int PP = 5; CALL; } break;    \
    case 6: { constexpr int PP = 6; CALL; } break;    \
    case 7: { constexpr int PP = 7; CALL; } break;    \
    case 8: { constexpr int PP = 8; CALL; } break;    \
    case 9: { constexpr int PP = 9; CALL; } break;    \
    default: return hipErrorInvalidValue;             \
  }
static inline dim3 sgrid(int64_t n) { return dim3((unsigned)((n + kSW - 1) / kSW)); }

// ------------------------------------------------------------ element blocks
template <int P>
__global__ __launch_bounds__(kSW) void k_elem_rows(ElemGenRef r, const double* __restrict__ kappa,
                                                   double* __restrict__ EB, int64_t ne) {
  constexpr int P2 = P * P, F4 = 4 * P;
  // loops over the P2 unknowns unrolled for small degrees only (code size)
  constexpr int UR = P2 <= 25 ? P2 : 1;
  const int64_t t = (int64_t)blockIdx.x * kSW + threadIdx.x;
  if (t >= ne * F4) return;
  const int64_t e = t / F4;
  const int c = (int)(t - e * F4);
  const double kap = kappa[e];
  double w[P2], x[P2], s[P2], d[P2];
#pragma unroll UR
  for (int l = 0; l < P2; ++l) w[l] = kap * r.H[l * F4 + c] - r.E[l * F4 + c];
#pragma unroll UR
  for (int i = 0; i < P2; ++i) d[i] = 1.0 / (r.delta[i] + kap * r.mu[i]);
  // x = V diag(d) V^T w
#pragma unroll UR
  for (int i = 0; i < P2; ++i) {
    double a = 0.0;
#pragma unroll UR
    for (int l = 0; l < P2; ++l) a += r.V[l * P2 + i] * w[l];
    s[i] = a * d[i];
  }
#pragma unroll UR
  for (int l = 0; l < P2; ++l) {
    double a = 0.0;
#pragma unroll UR
    for (int i = 0; i < P2; ++i) a += r.V[l * P2 + i] * s[i];
    x[l] = a;
  }
  // one refinement step: x += V diag(d) V^T (w - (D + kappa G) x)
  double res[P2];
#pragma unroll UR
  for (int l = 0; l < P2; ++l) {
    double a = w[l];
#pragma unroll UR
    for (int q = 0; q < P2; ++q) a -= (r.Dm[l * P2 + q] + kap * r.G[l * P2 + q]) * x[q];
    res[l] = a;
  }
#pragma unroll UR
  for (int i = 0; i < P2; ++i) {
    double a = 0.0;
#pragma unroll UR
    for (int l = 0; l < P2; ++l) a += r.V[l * P2 + i] * res[l];
    s[i] = a * d[i];
  }
#pragma unroll UR
  for (int l = 0; l < P2; ++l) {
    double a = 0.0;
#pragma unroll UR
    for (int i = 0; i < P2; ++i) a += r.V[l * P2 + i] * s[i];
    x[l] += a;
  }
  double* out = EB + (e * F4 + c) * F4;
  for (int a = 0; a < F4; ++a) {
    double acc = 0.0;
#pragma unroll UR
    for (int l = 0; l < P2; ++l) acc += (kap * r.H[l * F4 + a] - r.E[l * F4 + a]) * x[l];
    out[a] = r.tau * r.Mb[a * F4 + c] + kap * r.P1[a * F4 + c] - acc;
  }
}

hipError_t launch_elem_rows(int P, const ElemGenRef& r, const double* kappa, double* EB, int64_t ne,
                            hipStream_t s) {
  if (ne == 0) return hipSuccess;
  HDG_SETUP_DISPATCH_P(P, hipLaunchKernelGGL(k_elem_rows<PP>, sgrid(ne * 4 * PP), dim3(kSW), 0, s, r, kappa, EB, ne));
  return hipGetLastError();
}

// Kc = P4^T Kf P4 per element, P4 = blockdiag(Pp) [4(p+1) x 4p]; thread = (element, coarse row)
template <int PF>
__global__ __launch_bounds__(kSW) void k_elem_galerkin(const double* __restrict__ Pp, const double* __restrict__ Kf,
                                                       double* __restrict__ Kc, int64_t ne) {
  constexpr int PC = PF - 1, FF = 4 * PF, FC = 4 * PC;
  const int64_t t = (int64_t)blockIdx.x * kSW + threadIdx.x;
  if (t >= ne * FC) return;
  const int64_t e = t / FC;
  const int rc = (int)(t - e * FC);
  const int lf = rc / PC, b = rc - lf * PC;
  const double* K = Kf + e * FF * FF;
  double row[FF];  // sum_a Pp[a][b] Kf[lf PF + a][:]
#pragma unroll
  for (int col = 0; col < FF; ++col) {
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < PF; ++a) acc += Pp[a * PC + b] * K[(lf * PF + a) * FF + col];
    row[col] = acc;
  }
  double* out = Kc + (e * FC + rc) * FC;
#pragma unroll
  for (int lf2 = 0; lf2 < 4; ++lf2)
#pragma unroll
    for (int b2 = 0; b2 < PC; ++b2) {
      double acc = 0.0;
#pragma unroll
      for (int a = 0; a < PF; ++a) acc += row[lf2 * PF + a] * Pp[a * PC + b2];
      out[lf2 * PC + b2] = acc;
    }
}

hipError_t launch_elem_galerkin(int Pfine, const double* Pp, const double* Kf, double* Kc, int64_t ne,
                                hipStream_t s) {
  if (ne == 0) return hipSuccess;
  if (Pfine < 2) return hipErrorInvalidValue;
  HDG_SETUP_DISPATCH_P(Pfine, if constexpr (PP >= 2) hipLaunchKernelGGL(k_elem_galerkin<PP>, sgrid(ne * 4 * (PP - 1)),
                                                                        dim3(kSW), 0, s, Pp, Kf, Kc, ne));
  return hipGetLastError();
}

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ void elem_face_pair(int n, int64_t f, int64_t& lo, int64_t& hi, int& llo, int& lhi) {
  const int64_t nv = (int64_t)n * (n - 1);
  if (f < nv) {  // vertical, between (i-1, j) and (i, j)
    const int64_t j = f / (n - 1), i = f - j * (n - 1) + 1;
    lo = (i - 1) + (int64_t)n * j;
    hi = i + (int64_t)n * j;
    llo = 1;
    lhi = 0;
  } else {       // horizontal, between (i, j-1) and (i, j)
    const int64_t q = f - nv, jm1 = q / n, i = q - jm1 * n;
    lo = i + (int64_t)n * jm1;
    hi = i + (int64_t)n * (jm1 + 1);
    llo = 3;
    lhi = 2;
  }
}

__device__ __forceinline__ bool elem_face_interior(int n, int64_t e, int lf) {
  const int64_t j = e / n, i = e - j * n;
  switch (lf) {
    case 0: return i >= 1;
    case 1: return i <= n - 2;
    case 2: return j >= 1;
    default: return j <= n - 2;
  }
}

// the 3 local faces != lf in increasing order
__device__ __forceinline__ int other_face(int lf, int s) { return s < lf ? s : s + 1; }

template <typename TM>
__device__ __forceinline__ void store_as(TM* p, double v);
template <>
__device__ __forceinline__ void store_as<double>(double* p, double v) { *p = v; }
template <>
__device__ __forceinline__ void store_as<float>(float* p, double v) { *p = (float)v; }
template <>
__device__ __forceinline__ void store_as<uint16_t>(uint16_t* p, double v) {  // bfloat16, round to nearest even
  const float f = (float)v;
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);
  *p = (uint16_t)(u >> 16);
}

// ------------------------------------------------------------ face slabs
// Entry e of face f in the tile-interleaved layout (V entries per 16 bytes):
// ((tile NQ + e / V) 64 + lane) V + e % V.  Thread = (16-byte word q, face f).
template <int P, typename TM>
__global__ __launch_bounds__(kSW) void k_pack_slab(const double* __restrict__ EB, int n, int64_t nf, TM* __restrict__ slab,
                                                   double* __restrict__ slab64) {
  constexpr int P2 = P * P, F4 = 4 * P, NE = 7 * P2;
  constexpr int V = 16 / (int)sizeof(TM), NQ = (NE + V - 1) / V;
  constexpr int NQ64 = (NE + 1) / 2;
  const int64_t ntiles = (nf + 63) / 64;
  const int64_t t = (int64_t)blockIdx.x * kSW + threadIdx.x;
  if (t >= ntiles * 64 * NQ) return;
  const int64_t tile = t / (64 * NQ);
  const int q = (int)((t / 64) % NQ);
  const int lane = (int)(t & 63);
  const int64_t f = tile * 64 + lane;
  const int64_t base = ((tile * NQ + q) * 64 + lane) * V;
  if (f >= nf) {
#pragma unroll
    for (int u = 0; u < V; ++u) store_as<TM>(slab + base + u, 0.0);
    return;
  }
  int64_t lo, hi;
  int llo, lhi;
  elem_face_pair(n, f, lo, hi, llo, lhi);
  const double* Klo = EB + lo * F4 * F4;
  const double* Khi = EB + hi * F4 * F4;
#pragma unroll
  for (int u = 0; u < V; ++u) {
    const int e = q * V + u;
    double v = 0.0;
    if (e < NE) {
      const int sl = e / P2, ac = e - sl * P2, a = ac / P, c = ac - a * P;
      if (sl == 0) {
        v = Klo[(llo * P + a) * F4 + llo * P + c] + Khi[(lhi * P + a) * F4 + lhi * P + c];
      } else if (sl <= 3) {
        const int g = other_face(llo, sl - 1);
        if (elem_face_interior(n, lo, g)) v = Klo[(llo * P + a) * F4 + g * P + c];
      } else {
        const int g = other_face(lhi, sl - 4);
        if (elem_face_interior(n, hi, g)) v = Khi[(lhi * P + a) * F4 + g * P + c];
      }
    }
    store_as<TM>(slab + base + u, v);
    if (slab64 != nullptr && e < 2 * NQ64) {
      // FP64 copy of the same entry (2 entries per 16 bytes)
      const int64_t b64 = ((tile * NQ64 + e / 2) * 64 + lane) * 2 + (e & 1);
      slab64[b64] = v;
    }
  }
}

hipError_t launch_pack_slab(Prec mp, int P, const double* EB, int n, int64_t nf, void* slab, double* slab64,
                            hipStream_t s) {
  if (nf == 0) return hipSuccess;
  const int64_t ntiles = (nf + 63) / 64;
  const int V = mat_lanes16(mp);
  const int64_t nq = (7 * P * P + V - 1) / V;
  switch (mp) {
    case Prec::F64:
      HDG_SETUP_DISPATCH_P(P, hipLaunchKernelGGL((k_pack_slab<PP, double>), sgrid(ntiles * 64 * nq), dim3(kSW), 0, s,
                                                 EB, n, nf, (double*)slab, nullptr));
      break;
    case Prec::F32:
      HDG_SETUP_DISPATCH_P(P, hipLaunchKernelGGL((k_pack_slab<PP, float>), sgrid(ntiles * 64 * nq), dim3(kSW), 0, s,
                                                 EB, n, nf, (float*)slab, slab64));
      break;
    case Prec::BF16:
      HDG_SETUP_DISPATCH_P(P, hipLaunchKernelGGL((k_pack_slab<PP, uint16_t>), sgrid(ntiles * 64 * nq), dim3(kSW), 0,
                                                 s, EB, n, nf, (uint16_t*)slab, slab64));
      break;
  }
  return hipGetLastError();
}

// In-register Cholesky inverse of an SPD P x P matrix (row major), in the order
// of operations of the host setup (factor, then forward and backward
// substitution on the identity).  Returns false if a pivot is not positive.
template <int P>
__device__ bool spd_inverse(const double* A, double* X) {
  double L[P * P];
#pragma unroll
  for (int i = 0; i < P * P; ++i) L[i] = A[i];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    double d = L[j * P + j];
#pragma unroll
    for (int k = 0; k < j; ++k) d -= L[j * P + k] * L[j * P + k];
    if (!(d > 0.0)) return false;
    d = sqrt(d);
    L[j * P + j] = d;
#pragma unroll
    for (int i = j + 1; i < P; ++i) {
      double s = L[i * P + j];
#pragma unroll
      for (int k = 0; k < j; ++k) s -= L[i * P + k] * L[j * P + k];
      L[i * P + j] = s / d;
    }
  }
#pragma unroll
  for (int i = 0; i < P * P; ++i) X[i] = (i / P == i % P) ? 1.0 : 0.0;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const double inv = 1.0 / L[i * P + i];
#pragma unroll
    for (int c = 0; c < P; ++c) {
      double s = X[i * P + c];
#pragma unroll
      for (int k = 0; k < i; ++k) s -= L[i * P + k] * X[k * P + c];
      X[i * P + c] = s * inv;
    }
  }
#pragma unroll
  for (int i = P - 1; i >= 0; --i) {
    const double inv = 1.0 / L[i * P + i];
#pragma unroll
    for (int c = 0; c < P; ++c) {
      double s = X[i * P + c];
#pragma unroll
      for (int k = i + 1; k < P; ++k) s -= L[k * P + i] * X[k * P + c];
      X[i * P + c] = s * inv;
    }
  }
  return true;
}

// Facet inverses (facet Schwarz): the summed diagonal block of each face,
// inverted, in the slab's layout with P^2 entries per face.  A block that is not
// SPD sets *fail.
template <int P, typename TM>
__global__ __launch_bounds__(kSW) void k_face_dinv(const double* __restrict__ EB, int n, int64_t nf, TM* __restrict__ dinv,
                                                   int* fail) {
  constexpr int P2 = P * P, F4 = 4 * P;
  constexpr int V = 16 / (int)sizeof(TM), NQD = (P2 + V - 1) / V;
  const int64_t f = (int64_t)blockIdx.x * kSW + threadIdx.x;
  const int64_t ntiles = (nf + 63) / 64;
  if (f >= ntiles * 64) return;
  const int64_t tile = f >> 6;
  const int lane = (int)(f & 63);
  double X[P2];
#pragma unroll
  for (int i = 0; i < P2; ++i) X[i] = 0.0;
  if (f < nf) {
    int64_t lo, hi;
    int llo, lhi;
    elem_face_pair(n, f, lo, hi, llo, lhi);
    double D[P2];
#pragma unroll
    for (int a = 0; a < P; ++a)
#pragma unroll
      for (int c = 0; c < P; ++c)
        D[a * P + c] = EB[(lo * F4 + llo * P + a) * F4 + llo * P + c] + EB[(hi * F4 + lhi * P + a) * F4 + lhi * P + c];
    if (!spd_inverse<P>(D, X)) *fail = 1;
  }
#pragma unroll
  for (int e = 0; e < NQD * V; ++e)
    store_as<TM>(dinv + ((tile * NQD + e / V) * 64 + lane) * V + e % V, e < P2 ? X[e] : 0.0);
}

hipError_t launch_face_dinv(Prec mp, int P, const double* EB, int n, int64_t nf, void* dinv, int* fail,
                            hipStream_t s) {
  if (nf == 0) return hipSuccess;
  const int64_t nt = (nf + 63) / 64 * 64;
  switch (mp) {
    case Prec::F64:
      HDG_SETUP_DISPATCH_P(P, hipLaunchKernelGGL((k_face_dinv<PP, double>), sgrid(nt), dim3(kSW), 0, s, EB, n, nf,
                                                 (double*)dinv, fail));
      break;
    case Prec::F32:
      HDG_SETUP_DISPATCH_P(P, hipLaunchKernelGGL((k_face_dinv<PP, float>), sgrid(nt), dim3(kSW), 0, s, EB, n, nf,
                                                 (float*)dinv, fail));
      break;
    case Prec::BF16:
      HDG_SETUP_DISPATCH_P(P, hipLaunchKernelGGL((k_face_dinv<PP, uint16_t>), sgrid(nt), dim3(kSW), 0, s, EB, n, nf,
                                                 (uint16_t*)dinv, fail));
      break;
  }
  return hipGetLastError();
}

// ------------------------------------------------ element-patch Schwarz
// Subdomain of element e: its interior faces.  S restricted to them is e's own
// block plus, on the diagonal block of each face, the neighbour's diagonal block
// of that face (two distinct faces share one element at most).  The inverse is
// stored as an element block (zero rows and columns for boundary faces), so the
// smoother sum_e R_e^T (R_e S R_e^T)^{-1} R_e has the layout of S and is packed
// and applied face by face like it.  Thread = element.
template <int P>
__global__ __launch_bounds__(kSW) void k_patch_inverse(const double* __restrict__ EB, int n, double* __restrict__ MB,
                                                       int* fail) {
  constexpr int F4 = 4 * P, F2 = F4 * F4;
  const int64_t ne = (int64_t)n * n;
  const int64_t e = (int64_t)blockIdx.x * kSW + threadIdx.x;
  if (e >= ne) return;
  const int64_t j = e / n, i = e - j * n;
  bool in[4];
  int64_t nb[4];
  in[0] = i >= 1, nb[0] = e - 1;        // left: neighbour's right face (local 1)
  in[1] = i <= n - 2, nb[1] = e + 1;    // right: neighbour's local 0
  in[2] = j >= 1, nb[2] = e - n;        // bottom: neighbour's local 3
  in[3] = j <= n - 2, nb[3] = e + n;    // top: neighbour's local 2
  double A[F2], X[F2];
  const double* K = EB + e * F2;
  for (int r = 0; r < F4; ++r)
    for (int c = 0; c < F4; ++c) {
      const bool ok = in[r / P] && in[c / P];
      A[r * F4 + c] = ok ? K[r * F4 + c] : (r == c ? 1.0 : 0.0);
    }
  for (int lf = 0; lf < 4; ++lf) {
    if (!in[lf]) continue;
    const int nlf = lf ^ 1;  // the same face seen from the neighbour
    const double* Kn = EB + nb[lf] * F2;
    for (int a = 0; a < P; ++a)
      for (int c = 0; c < P; ++c) A[(lf * P + a) * F4 + lf * P + c] += Kn[(nlf * P + a) * F4 + nlf * P + c];
  }
  if (!spd_inverse<F4>(A, X)) *fail = 1;
  double* out = MB + e * F2;
  for (int r = 0; r < F4; ++r)
    for (int c = 0; c < F4; ++c) out[r * F4 + c] = (in[r / P] && in[c / P]) ? X[r * F4 + c] : 0.0;
}

hipError_t launch_patch_inverse(int P, const double* EB, int n, double* MB, int* fail, hipStream_t s) {
  const int64_t ne = (int64_t)n * n;
  if (ne == 0) return hipSuccess;
  HDG_SETUP_DISPATCH_P(P, hipLaunchKernelGGL(k_patch_inverse<PP>, sgrid(ne), dim3(kSW), 0, s, EB, n, MB, fail));
  return hipGetLastError();
}

// ------------------------------------------------- chain cyclic reduction
// Factors of the block-tridiagonal matrix of every chain of faces (the SPD
// principal submatrix of S on the vertical faces of an element row, or the
// horizontal faces of an element column), in the record layout the chain
// solve reads: per level of size ml the odd positions' records
// [Dinv, W = Dinv A, Z = Dinv C] as 3 P^2 arrays over floor(ml/2) columns, the
// last level Dinv of its single block.  One workgroup per chain; the current
// level's blocks (A, D, C per position, FP64) live in `work`, the next level's
// in the second half.  The even positions of a level reduce with the odd
// neighbours' W and Z (A_j W_{j-1}, A_j Z_{j-1}, C_j W_{j+1}, C_j Z_{j+1}).
template <int P>
__device__ __forceinline__ void mat_mul(const double* X, const double* Y, double* Z) {
#pragma unroll
  for (int a = 0; a < P; ++a)
#pragma unroll
    for (int b = 0; b < P; ++b) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < P; ++q) s += X[a * P + q] * Y[q * P + b];
      Z[a * P + b] = s;
    }
}

template <int P, typename TV>
__global__ __launch_bounds__(kSW) void k_chain_factor(const double* __restrict__ EB, int n, int64_t chain0,
                                                      double* __restrict__ work, int64_t wstride, TV* __restrict__ fac,
                                                      int64_t cstride, int* fail) {
  constexpr int P2 = P * P, F4 = 4 * P, B3 = 3 * P2;
  const int64_t c = chain0 + blockIdx.x;
  const int m = n - 1;
  double* cur = work + (int64_t)blockIdx.x * wstride;
  double* nxt = cur + (int64_t)B3 * m;
  TV* F = fac + c * cstride;
  const bool vert = c < n;
  const int t = threadIdx.x, nt = blockDim.x;
  // level 0: [A | D | C] of every position from the element blocks
  for (int i = t; i < m; i += nt) {
    int64_t lo, hi;
    int llo, lhi, lsub, lsup;
    if (vert) {  // row c: between (i, c) and (i+1, c); previous face = lo's left, next = hi's right
      lo = i + (int64_t)n * c;
      hi = lo + 1;
      llo = 1, lhi = 0, lsub = 0, lsup = 1;
    } else {     // column c - n: between (c', i) and (c', i+1); previous = lo's bottom, next = hi's top
      lo = (c - n) + (int64_t)n * i;
      hi = lo + n;
      llo = 3, lhi = 2, lsub = 2, lsup = 3;
    }
    double* blk = cur + (int64_t)i * B3;
#pragma unroll
    for (int a = 0; a < P; ++a)
#pragma unroll
      for (int b = 0; b < P; ++b) {
        blk[a * P + b] = i >= 1 ? EB[(lo * F4 + llo * P + a) * F4 + lsub * P + b] : 0.0;
        blk[P2 + a * P + b] =
            EB[(lo * F4 + llo * P + a) * F4 + llo * P + b] + EB[(hi * F4 + lhi * P + a) * F4 + lhi * P + b];
        blk[2 * P2 + a * P + b] = i + 1 < m ? EB[(hi * F4 + lhi * P + a) * F4 + lsup * P + b] : 0.0;
      }
  }
  __syncthreads();
  int ml = m;
  int64_t off = 0;
  while (ml > 1) {
    const int no = ml / 2;
    for (int o = t; o < no; o += nt) {  // odd positions j = 2o + 1
      double* blk = cur + (int64_t)(2 * o + 1) * B3;
      double Di[P2], W[P2], Z[P2];
      if (!spd_inverse<P>(blk + P2, Di)) *fail = 1;
      mat_mul<P>(Di, blk, W);
      mat_mul<P>(Di, blk + 2 * P2, Z);
#pragma unroll
      for (int e = 0; e < P2; ++e) {
        F[off + (int64_t)e * no + o] = (TV)Di[e];
        F[off + (int64_t)(P2 + e) * no + o] = (TV)W[e];
        F[off + (int64_t)(2 * P2 + e) * no + o] = (TV)Z[e];
        blk[e] = W[e];            // A slot now holds W
        blk[2 * P2 + e] = Z[e];   // C slot now holds Z
      }
    }
    __syncthreads();
    const int ne = (ml + 1) / 2;
    for (int o = t; o < ne; o += nt) {  // even positions j = 2o
      const int j = 2 * o;
      const double* blk = cur + (int64_t)j * B3;
      double Dn[P2], An[P2], Cn[P2], T[P2];
#pragma unroll
      for (int e = 0; e < P2; ++e) {
        Dn[e] = blk[P2 + e];
        An[e] = 0.0;
        Cn[e] = 0.0;
      }
      if (j >= 1) {
        const double* L = cur + (int64_t)(j - 1) * B3;  // W_{j-1} in A slot, Z_{j-1} in C slot
        mat_mul<P>(blk, L + 2 * P2, T);
#pragma unroll
        for (int e = 0; e < P2; ++e) Dn[e] -= T[e];
        mat_mul<P>(blk, L, T);
#pragma unroll
        for (int e = 0; e < P2; ++e) An[e] = -T[e];
      }
      if (j + 1 < ml) {
        const double* R = cur + (int64_t)(j + 1) * B3;
        mat_mul<P>(blk + 2 * P2, R, T);
#pragma unroll
        for (int e = 0; e < P2; ++e) Dn[e] -= T[e];
        mat_mul<P>(blk + 2 * P2, R + 2 * P2, T);
#pragma unroll
        for (int e = 0; e < P2; ++e) Cn[e] = -T[e];
      }
      double* out = nxt + (int64_t)o * B3;
#pragma unroll
      for (int e = 0; e < P2; ++e) {
        out[e] = An[e];
        out[P2 + e] = Dn[e];
        out[2 * P2 + e] = Cn[e];
      }
    }
    __syncthreads();
    double* sw = cur;
    cur = nxt;
    nxt = sw;
    off += (int64_t)B3 * no;
    ml = ne;
  }
  if (t == 0) {
    double Di[P2];
    if (!spd_inverse<P>(cur + P2, Di)) *fail = 1;
#pragma unroll
    for (int e = 0; e < P2; ++e) F[off + e] = (TV)Di[e];
  }
}

int64_t chain_factor_work_doubles(int P, int n) {
  const int64_t m = n - 1;
  return (int64_t)3 * P * P * (m + (m + 1) / 2);
}

hipError_t launch_chain_factor(Prec vp, int P, const double* EB, int n, int64_t chain0, int nchains, double* work,
                               void* fac, int64_t cstride, int* fail, hipStream_t s) {
  if (nchains <= 0) return hipSuccess;
  const int64_t ws = chain_factor_work_doubles(P, n);
  if (vp == Prec::F64) {
    HDG_SETUP_DISPATCH_P(P, hipLaunchKernelGGL((k_chain_factor<PP, double>), dim3((unsigned)nchains), dim3(kSW), 0, s,
                                               EB, n, chain0, work, ws, (double*)fac, cstride, fail));
  } else {
    HDG_SETUP_DISPATCH_P(P, hipLaunchKernelGGL((k_chain_factor<PP, float>), dim3((unsigned)nchains), dim3(kSW), 0, s,
                                               EB, n, chain0, work, ws, (float*)fac, cstride, fail));
  }
  return hipGetLastError();
}

// ------------------------------------- partitioned chain solve (P = 1)
// At P = 1 a chain matrix is scalar tridiagonal and SPD: diagonal D_i and
// coupling E_i between positions i and i + 1 (symmetric; E_i is taken from the
// element on the chain's high side, as in the cyclic reduction above).  The
// chain is split into nseg <= 64 segments of >= 2 positions, one per lane of
// the solving wavefront.  Each segment's interior (all but its first and last
// position) is factored by Gaussian elimination: pivots piv_j, stored as
// ip_j = 1 / piv_j and ch_j = E_j ip_j.  Eliminating the interiors leaves a
// tridiagonal system on the segment ends (first F_k, last L_k of segment k);
// eliminating the F_k leaves a tridiagonal system on the L_k, one per lane,
// solved by parallel cyclic reduction over the lanes (6 levels).  Everything
// that depends on the matrix only is computed here, per lane:
//   0 eF = E_o, 1 eL = E_{l-1} (o, l: the segment's first and last position),
//   2 muF, 3 nuF (the F-elimination's multipliers of gF_k, gF_{k+1}),
//   4 1 / betaF, 5 alphaF, 6 gammaF (row F_k: alphaF L_{k-1} + betaF F_k + gammaF L_k),
//   7 + 2 h, 8 + 2 h: the cyclic reduction's multipliers of level h (lanes k - 2^h, k + 2^h),
//   19 1 / b (the decoupled L_k rows).
// Record of a chain: ch[LMAX][64], ip[LMAX][64], scalars[20][64], lane-minor.
template <typename TV>
__global__ __launch_bounds__(64) void k_chain_tri_factor(const double* __restrict__ EB, int n, TV* __restrict__ tri,
                                                         int lmax, int64_t tstride, int* fail) {
  const int64_t c = blockIdx.x;
  const int m = n - 1, k = threadIdx.x;
  const bool vert = c < n;
  const int nseg = min(64, m / 2), base = m / nseg, extra = m % nseg;
  const int L = k < nseg ? base + (k < extra ? 1 : 0) : 0;
  const int o = k * base + min(k, extra), l = o + L - 1;
  TV* R = tri + c * tstride;
  // D_i and E_i of position i (E_{m-1} = 0)
  auto entries = [&](int i, double& D, double& E) {
    int64_t lo, hi;
    int llo, lhi, lsup;
    if (vert) {  // row c: between (i, c) and (i+1, c); next face = hi's right
      lo = i + (int64_t)n * c;
      hi = lo + 1;
      llo = 1, lhi = 0, lsup = 1;
    } else {     // column c - n: between (c', i) and (c', i+1); next face = hi's top
      lo = (c - n) + (int64_t)n * i;
      hi = lo + n;
      llo = 3, lhi = 2, lsup = 3;
    }
    D = EB[(lo * 4 + llo) * 4 + llo] + EB[(hi * 4 + lhi) * 4 + lhi];
    E = i + 1 < m ? EB[(hi * 4 + lhi) * 4 + lsup] : 0.0;
  };
  __shared__ double sa[64], sb[64], sc[64], saF[64], sbF[64], sgF[64];
  double ch[32], ip[32];
  for (int j = 0; j < 32; ++j) ch[j] = ip[j] = 0.0;
  double aF = 0.0, bF = 1.0, gF = 0.0, aL = 0.0, bL = 1.0, gL = 0.0, eF = 0.0, eL = 0.0;
  bool bad = false;
  if (L >= 2) {
    double Do, Dl, El, dummy;
    entries(o, Do, eF);
    entries(l, Dl, El);
    entries(l - 1, dummy, eL);
    if (k > 0) entries(o - 1, dummy, aF);
    gL = El;
    if (L == 2) {
      bF = Do, gF = eF, aL = eF, bL = Dl;
    } else {
      // interior LU, then the spikes' end values: sigma = T_J^{-1} (E_o e_1),
      // tau = T_J^{-1} (E_{l-1} e_{L-2})
      double Eprev = eF;
      for (int j = 1; j <= L - 2; ++j) {
        double Dj, Ej;
        entries(o + j, Dj, Ej);
        const double piv = j == 1 ? Dj : Dj - Eprev * ch[j - 1];
        if (!(piv > 0.0) || !isfinite(piv)) bad = true;
        ip[j] = 1.0 / piv;
        ch[j] = j <= L - 3 ? Ej * ip[j] : 0.0;
        Eprev = Ej;
      }
      double s[32];
      s[1] = eF;
      for (int j = 2; j <= L - 2; ++j) s[j] = -ch[j - 1] * s[j - 1];
      double sig = s[L - 2] * ip[L - 2];
      const double sigL = sig;
      for (int j = L - 3; j >= 1; --j) sig = s[j] * ip[j] - ch[j] * sig;
      double tau = eL * ip[L - 2];
      const double tauL = tau;
      for (int j = L - 3; j >= 1; --j) tau = -ch[j] * tau;
      bF = Do - eF * sig;
      gF = -eF * tau;
      aL = -eL * sigL;
      bL = Dl - eL * tauL;
    }
    if (!(bF > 0.0) || !isfinite(bF)) bad = true;
  }
  saF[k] = aF, sbF[k] = bF, sgF[k] = gF;
  __syncthreads();
  const bool nxt = k + 1 < nseg;
  const double muF = L >= 2 ? aL / bF : 0.0;
  const double nuF = L >= 2 && nxt ? gL / sbF[k + 1] : 0.0;
  double a = L >= 2 ? -muF * aF : 0.0;
  double b = L >= 2 ? bL - muF * gF - (nxt ? nuF * saF[k + 1] : 0.0) : 1.0;
  double cc = L >= 2 && nxt ? -nuF * sgF[k + 1] : 0.0;
  double pm[6], pn[6];
  for (int h = 0; h < 6; ++h) {
    const int d = 1 << h;
    sa[k] = a, sb[k] = b, sc[k] = cc;
    __syncthreads();
    const bool lo_ok = L >= 2 && k - d >= 0, hi_ok = L >= 2 && k + d < nseg;
    const double mu = lo_ok ? a / sb[k - d] : 0.0;
    const double nu = hi_ok ? cc / sb[k + d] : 0.0;
    const double na = lo_ok ? -mu * sa[k - d] : 0.0;
    const double nc = hi_ok ? -nu * sc[k + d] : 0.0;
    const double nb = b - (lo_ok ? mu * sc[k - d] : 0.0) - (hi_ok ? nu * sa[k + d] : 0.0);
    __syncthreads();
    pm[h] = mu, pn[h] = nu;
    a = na, b = nb, cc = nc;
  }
  if (L >= 2 && (!(b > 0.0) || !isfinite(b))) bad = true;
  if (bad) *fail = 1;
  for (int j = 0; j < lmax; ++j) {
    R[(int64_t)j * 64 + k] = (TV)ch[j];
    R[(int64_t)(lmax + j) * 64 + k] = (TV)ip[j];
  }
  TV* S = R + (int64_t)2 * lmax * 64;
  const double sv[7] = {eF, eL, muF, nuF, L >= 2 ? 1.0 / bF : 0.0, aF, gF};
  for (int q = 0; q < 7; ++q) S[q * 64 + k] = (TV)sv[q];
  for (int h = 0; h < 6; ++h) {
    S[(7 + 2 * h) * 64 + k] = (TV)pm[h];
    S[(8 + 2 * h) * 64 + k] = (TV)pn[h];
  }
  S[19 * 64 + k] = (TV)(L >= 2 ? 1.0 / b : 0.0);
}

hipError_t launch_chain_tri_factor(Prec vp, const double* EB, int n, void* tri, int* fail, hipStream_t s) {
  const int lmax = chain_tri_lmax(n);
  if (lmax == 0) return hipErrorInvalidValue;
  const int64_t ts = chain_tri_stride(n);
  if (vp == Prec::F64)
    hipLaunchKernelGGL((k_chain_tri_factor<double>), dim3((unsigned)(2 * n)), dim3(64), 0, s, EB, n, (double*)tri,
                       lmax, ts, fail);
  else
    hipLaunchKernelGGL((k_chain_tri_factor<float>), dim3((unsigned)(2 * n)), dim3(64), 0, s, EB, n, (float*)tri,
                       lmax, ts, fail);
  return hipGetLastError();
}

// ---------------------------------------------------------------- Q1 levels
// Stencil of P_J^T S0 P_J on the interior vertices of the n x n mesh from the
// p = 0 element blocks (4 x 4): a vertex gathers, from its 4 elements in order,
// 1/4 of K[f1][f2] for every interior face f1 it ends and every interior end w
// of every interior face f2 (P_J maps vertex values to face means).
__global__ __launch_bounds__(kSW) void k_q1_stencil0(const double* __restrict__ EB0, int n, double* __restrict__ st) {
  const int64_t Nv = (int64_t)(n - 1) * (n - 1);
  const int64_t v = (int64_t)blockIdx.x * kSW + threadIdx.x;
  if (v >= Nv) return;
  const int vi = (int)(v % (n - 1)) + 1, vj = (int)(v / (n - 1)) + 1;
  double acc[9];
#pragma unroll
  for (int s = 0; s < 9; ++s) acc[s] = 0.0;
  for (int ej = vj - 1; ej <= vj; ++ej)
    for (int ei = vi - 1; ei <= vi; ++ei) {
      const int64_t e = ei + (int64_t)n * ej;
      const double* K = EB0 + e * 16;
      // face ends: left (ei, ej)-(ei, ej+1), right (ei+1, ej)-(ei+1, ej+1),
      // bottom (ei, ej)-(ei+1, ej), top (ei, ej+1)-(ei+1, ej+1)
      const int ex[4][2] = {{ei, ei}, {ei + 1, ei + 1}, {ei, ei + 1}, {ei, ei + 1}};
      const int ey[4][2] = {{ej, ej + 1}, {ej, ej + 1}, {ej, ej}, {ej + 1, ej + 1}};
      bool inter[4];
#pragma unroll
      for (int lf = 0; lf < 4; ++lf) inter[lf] = elem_face_interior(n, e, lf);
      for (int f1 = 0; f1 < 4; ++f1) {
        if (!inter[f1]) continue;
        for (int f2 = 0; f2 < 4; ++f2) {
          if (!inter[f2]) continue;
          const double kv = K[f1 * 4 + f2];
          for (int a = 0; a < 2; ++a) {
            if (ex[f1][a] != vi || ey[f1][a] != vj) continue;
            for (int b = 0; b < 2; ++b) {
              const int wi = ex[f2][b], wj = ey[f2][b];
              if (wi <= 0 || wj <= 0 || wi >= n || wj >= n) continue;
              acc[(wi - vi + 1) + 3 * (wj - vj + 1)] += 0.25 * kv;
            }
          }
        }
      }
    }
#pragma unroll
  for (int s = 0; s < 9; ++s) st[s * Nv + v] = acc[s];
}

hipError_t launch_q1_stencil0(const double* EB0, int n, double* st, hipStream_t s) {
  const int64_t Nv = (int64_t)(n - 1) * (n - 1);
  if (Nv == 0) return hipSuccess;
  hipLaunchKernelGGL(k_q1_stencil0, sgrid(Nv), dim3(kSW), 0, s, EB0, n, st);
  return hipGetLastError();
}

// Galerkin coarse stencil I^T A I with bilinear I (coarse vertex (I, J) at fine
// (2I, 2J), weights 1 and 1/2): thread = coarse interior vertex.
__global__ __launch_bounds__(kSW) void k_q1_galerkin(const double* __restrict__ stf, int mf, double* __restrict__ stc) {
  const int mc = mf / 2;
  const int64_t Nf = (int64_t)(mf - 1) * (mf - 1), Nc = (int64_t)(mc - 1) * (mc - 1);
  const int64_t V = (int64_t)blockIdx.x * kSW + threadIdx.x;
  if (V >= Nc) return;
  const int I = (int)(V % (mc - 1)) + 1, J = (int)(V / (mc - 1)) + 1;
  double acc[9];
#pragma unroll
  for (int s = 0; s < 9; ++s) acc[s] = 0.0;
  for (int dj = -1; dj <= 1; ++dj)
    for (int di = -1; di <= 1; ++di) {
      const int vi = 2 * I + di, vj = 2 * J + dj;   // interior of the fine mesh
      const double wv = (di == 0 ? 1.0 : 0.5) * (dj == 0 ? 1.0 : 0.5);
      const int64_t v = (int64_t)(vi - 1) + (int64_t)(mf - 1) * (vj - 1);
      for (int ej = -1; ej <= 1; ++ej)
        for (int ei = -1; ei <= 1; ++ei) {
          const double a = stf[((ei + 1) + 3 * (ej + 1)) * Nf + v];
          if (a == 0.0) continue;
          const int wi = vi + ei, wj = vj + ej;
          // coarse vertices whose hat function is nonzero at fine (wi, wj)
          int ci[2], cj[2];
          double cwi[2], cwj[2];
          int nci = 0, ncj = 0;
          if (wi % 2 == 0) { ci[0] = wi / 2; cwi[0] = 1.0; nci = 1; }
          else { ci[0] = wi / 2; ci[1] = wi / 2 + 1; cwi[0] = cwi[1] = 0.5; nci = 2; }
          if (wj % 2 == 0) { cj[0] = wj / 2; cwj[0] = 1.0; ncj = 1; }
          else { cj[0] = wj / 2; cj[1] = wj / 2 + 1; cwj[0] = cwj[1] = 0.5; ncj = 2; }
          for (int y = 0; y < ncj; ++y)
            for (int x = 0; x < nci; ++x) {
              const int WI = ci[x], WJ = cj[y];
              if (WI <= 0 || WJ <= 0 || WI >= mc || WJ >= mc) continue;
              acc[(WI - I + 1) + 3 * (WJ - J + 1)] += wv * a * cwi[x] * cwj[y];
            }
        }
    }
#pragma unroll
  for (int s = 0; s < 9; ++s) stc[s * Nc + V] = acc[s];
}

hipError_t launch_q1_galerkin(const double* stf, int mf, double* stc, hipStream_t s) {
  const int mc = mf / 2;
  const int64_t Nc = (int64_t)(mc - 1) * (mc - 1);
  if (Nc <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_q1_galerkin, sgrid(Nc), dim3(kSW), 0, s, stf, mf, stc);
  return hipGetLastError();
}

// Cycle copies of a Q1 level: the stencil in vector precision and 1 / diagonal.
template <typename TV>
__global__ __launch_bounds__(kSW) void k_q1_finish(const double* __restrict__ st64, int64_t Nv, TV* __restrict__ st,
                                                   TV* __restrict__ dinv, double* __restrict__ dinv64) {
  const int64_t v = (int64_t)blockIdx.x * kSW + threadIdx.x;
  if (v >= Nv) return;
  // the cycle keeps the symmetric operator's five entries of directions 4 ... 8
#pragma unroll
  for (int s = 0; s < 5; ++s) st[s * Nv + v] = (TV)st64[(4 + s) * Nv + v];
  const double d = 1.0 / st64[4 * Nv + v];
  dinv[v] = (TV)d;
  dinv64[v] = d;
}

hipError_t launch_q1_finish(Prec vp, const double* st64, int64_t Nv, void* st, void* dinv, double* dinv64,
                            hipStream_t s) {
  if (Nv == 0) return hipSuccess;
  if (vp == Prec::F64)
    hipLaunchKernelGGL(k_q1_finish<double>, sgrid(Nv), dim3(kSW), 0, s, st64, Nv, (double*)st, (double*)dinv, dinv64);
  else
    hipLaunchKernelGGL(k_q1_finish<float>, sgrid(Nv), dim3(kSW), 0, s, st64, Nv, (float*)st, (float*)dinv, dinv64);
  return hipGetLastError();
}

// out = a .* b (FP64)
__global__ __launch_bounds__(kSW) void k_vmul(const double* __restrict__ a, const double* __restrict__ b,
                                              double* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kSW + threadIdx.x;
  if (i < n) out[i] = a[i] * b[i];
}

hipError_t launch_vmul(const double* a, const double* b, double* out, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_vmul, sgrid(n), dim3(kSW), 0, s, a, b, out, n);
  return hipGetLastError();
}

}  // namespace hdg
