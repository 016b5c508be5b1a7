// gfx950 kernels of the multigrid cycle for many right-hand sides at once.
//
// Every vector is [rows][R]: the R right-hand sides of one trace DoF, Q1 vertex
// or face are contiguous, so a thread takes one (row, right-hand side) pair
// with the right-hand side fastest and every access of a wavefront is
// contiguous.  Each kernel applies the same operation as its single-vector
// counterpart in kernels.hip to every column; operators (blocks, smoother
// factors, stencils, transfer tables) are read once per launch for all columns.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "kernels.hpp"

namespace hdg {

static constexpr int kMW = 256;
static inline dim3 grid_m(int64_t n) { return dim3((unsigned)((n + kMW - 1) / kMW)); }

#define HDG_MDISPATCH_T(pr, CALL)                     \
  if ((pr) == Prec::F64) { using TT = double; CALL; } \
  else { using TT = float; CALL; }

#define HDG_MDISPATCH_P(P, CALL)                      \
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

// ------------------------------------------------------------- p-transfers
template <int P, typename T>
__global__ __launch_bounds__(kMW) void k_p_restrict_m(const T* pm, const T* rf, T* rc, int64_t nf, int R) {
  const int64_t idx = (int64_t)blockIdx.x * kMW + threadIdx.x;
  if (idx >= nf * R) return;
  const int64_t f = idx / R;
  const int r = (int)(idx - f * R);
  T v[P];
#pragma unroll
  for (int a = 0; a < P; ++a) v[a] = rf[(f * P + a) * R + r];
#pragma unroll
  for (int c = 0; c < P - 1; ++c) {
    T s = T(0);
#pragma unroll
    for (int a = 0; a < P; ++a) s += pm[a * (P - 1) + c] * v[a];
    rc[(f * (P - 1) + c) * R + r] = s;
  }
}

template <int P, typename T>
__global__ __launch_bounds__(kMW) void k_p_prolong_add_m(const T* pm, const T* ec, T* xf, int64_t nf, int R) {
  const int64_t idx = (int64_t)blockIdx.x * kMW + threadIdx.x;
  if (idx >= nf * R) return;
  const int64_t f = idx / R;
  const int r = (int)(idx - f * R);
  T e[P - 1];
#pragma unroll
  for (int c = 0; c < P - 1; ++c) e[c] = ec[(f * (P - 1) + c) * R + r];
#pragma unroll
  for (int a = 0; a < P; ++a) {
    T s = xf[(f * P + a) * R + r];
#pragma unroll
    for (int c = 0; c < P - 1; ++c) s += pm[a * (P - 1) + c] * e[c];
    xf[(f * P + a) * R + r] = s;
  }
}

hipError_t launch_p_prolong_add_m(Prec pr, int P, const void* pm, const void* ec, void* xf, int64_t nf, int R,
                                  hipStream_t s) {
  if (P < 2) return hipErrorInvalidValue;
  if (nf == 0) return hipSuccess;
  HDG_MDISPATCH_T(pr, HDG_MDISPATCH_P(P, if constexpr (PP >= 2) hipLaunchKernelGGL(
                                             (k_p_prolong_add_m<PP, TT>), grid_m(nf * R), dim3(kMW), 0, s,
                                             (const TT*)pm, (const TT*)ec, (TT*)xf, nf, R)));
  return hipGetLastError();
}
hipError_t launch_p_restrict_m(Prec pr, int P, const void* pm, const void* rf, void* rc, int64_t nf, int R,
                               hipStream_t s) {
  if (P < 2) return hipErrorInvalidValue;
  if (nf == 0) return hipSuccess;
  HDG_MDISPATCH_T(pr, HDG_MDISPATCH_P(P, if constexpr (PP >= 2) hipLaunchKernelGGL(
                                             (k_p_restrict_m<PP, TT>), grid_m(nf * R), dim3(kMW), 0, s,
                                             (const TT*)pm, (const TT*)rf, (TT*)rc, nf, R)));
  return hipGetLastError();
}

// ------------------------------------------------------------------ Q1 levels
template <typename T>
__device__ __forceinline__ T q1_apply_m(const T* st, const T* x, int m, int64_t Nv, int i, int j, int64_t v, int R,
                                        int r) {
  T s = T(0);
#pragma unroll
  for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
    for (int di = -1; di <= 1; ++di) {
      const int ii = i + di, jj = j + dj;  // clamped and zeroed outside, as in q1_apply
      const bool ok = ii >= 1 && jj >= 1 && ii <= m - 1 && jj <= m - 1;
      const int ic = min(max(ii, 1), m - 1), jc = min(max(jj, 1), m - 1);
      const T xv = x[((ic - 1) + (int64_t)(m - 1) * (jc - 1)) * R + r];
      // symmetric 5-entry stencil: directions 4 ... 8 at the vertex, the others
      // mirrored from the (clamped) neighbour
      const int d = (di + 1) + 3 * (dj + 1);
      const T a = d >= 4 ? st[(int64_t)(d - 4) * Nv + v]
                         : st[(int64_t)(4 - d) * Nv + (ic - 1) + (int64_t)(m - 1) * (jc - 1)];
      s += a * (ok ? xv : T(0));
    }
  return s;
}

template <typename T>
__global__ __launch_bounds__(kMW) void k_q1_resid_m(const T* st, const T* b, const T* x, T* rr, int m, int R) {
  const int64_t Nv = (int64_t)(m - 1) * (m - 1);
  const int64_t idx = (int64_t)blockIdx.x * kMW + threadIdx.x;
  if (idx >= Nv * R) return;
  const int64_t v = idx / R;
  const int r = (int)(idx - v * R);
  const int i = (int)(v % (m - 1)) + 1, j = (int)(v / (m - 1)) + 1;
  rr[idx] = b[idx] - q1_apply_m(st, x, m, Nv, i, j, v, R, r);
}

template <typename T>
__global__ __launch_bounds__(kMW) void k_q1_cheb_m(const T* st, const T* dinv, const T* b, const T* x, T* d, T* xo,
                                                   double c1, double c2, int m, int R) {
  const int64_t Nv = (int64_t)(m - 1) * (m - 1);
  const int64_t idx = (int64_t)blockIdx.x * kMW + threadIdx.x;
  if (idx >= Nv * R) return;
  const int64_t v = idx / R;
  const int r = (int)(idx - v * R);
  const int i = (int)(v % (m - 1)) + 1, j = (int)(v / (m - 1)) + 1;
  const T ax = x ? q1_apply_m(st, x, m, Nv, i, j, v, R, r) : T(0);
  const T z = dinv[v] * (b[idx] - ax);
  const T dn = (c1 != 0.0 ? T(c1) * d[idx] : T(0)) + T(c2) * z;
  d[idx] = dn;
  xo[idx] = (x ? x[idx] : T(0)) + dn;
}

template <typename T>
__global__ __launch_bounds__(kMW) void k_q1_restrict_m(const T* rf, T* rc, int mf, int R) {
  const int mc = mf / 2;
  const int64_t Nc = (int64_t)(mc - 1) * (mc - 1);
  const int64_t idx = (int64_t)blockIdx.x * kMW + threadIdx.x;
  if (idx >= Nc * R) return;
  const int64_t v = idx / R;
  const int r = (int)(idx - v * R);
  const int I = (int)(v % (mc - 1)) + 1, J = (int)(v / (mc - 1)) + 1;
  T s = T(0);
#pragma unroll
  for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
    for (int di = -1; di <= 1; ++di) {
      const T w = T((di == 0 ? 1.0 : 0.5) * (dj == 0 ? 1.0 : 0.5));
      const int fi = 2 * I + di, fj = 2 * J + dj;
      s += w * rf[((fi - 1) + (int64_t)(mf - 1) * (fj - 1)) * R + r];
    }
  rc[idx] = s;
}

template <typename T>
__global__ __launch_bounds__(kMW) void k_q1_prolong_add_m(const T* ec, T* xf, int mf, int R) {
  const int mc = mf / 2;
  const int64_t Nf = (int64_t)(mf - 1) * (mf - 1);
  const int64_t idx = (int64_t)blockIdx.x * kMW + threadIdx.x;
  if (idx >= Nf * R) return;
  const int64_t v = idx / R;
  const int r = (int)(idx - v * R);
  const int I = (int)(v % (mf - 1)) + 1, J = (int)(v / (mf - 1)) + 1;
  // bilinear weights over the 2 x 2 coarse vertices around (I, J): an even index
  // has one parent (the second weight is 0); parents outside the interior read
  // a clamped vertex and are zeroed, so no load sits under a branch
  const int xi[2] = {I / 2, I / 2 + (I & 1)}, yi[2] = {J / 2, J / 2 + (J & 1)};
  const T wx[2] = {(I & 1) ? T(0.5) : T(1), (I & 1) ? T(0.5) : T(0)};
  const T wy[2] = {(J & 1) ? T(0.5) : T(1), (J & 1) ? T(0.5) : T(0)};
  T s = T(0);
#pragma unroll
  for (int bb = 0; bb < 2; ++bb)
#pragma unroll
    for (int aa = 0; aa < 2; ++aa) {
      const int ci = xi[aa], cj = yi[bb];
      const bool ok = ci >= 1 && cj >= 1 && ci <= mc - 1 && cj <= mc - 1;
      const int cic = min(max(ci, 1), mc - 1), cjc = min(max(cj, 1), mc - 1);
      const T e = ec[((cic - 1) + (int64_t)(mc - 1) * (cjc - 1)) * R + r];
      s += wx[aa] * wy[bb] * (ok ? e : T(0));
    }
  xf[idx] += s;
}

template <typename T>
__global__ __launch_bounds__(kMW) void k_pj_restrict_m(const T* rface, T* rv, int n, int R) {
  const int64_t Nv = (int64_t)(n - 1) * (n - 1);
  const int64_t idx = (int64_t)blockIdx.x * kMW + threadIdx.x;
  if (idx >= Nv * R) return;
  const int64_t v = idx / R;
  const int r = (int)(idx - v * R);
  const int i = (int)(v % (n - 1)) + 1, j = (int)(v / (n - 1)) + 1;
  const int64_t nv = (int64_t)n * (n - 1);
  const T s = rface[((i - 1) + (int64_t)(n - 1) * j) * R + r] + rface[((i - 1) + (int64_t)(n - 1) * (j - 1)) * R + r] +
              rface[(nv + i + (int64_t)n * (j - 1)) * R + r] + rface[(nv + (i - 1) + (int64_t)n * (j - 1)) * R + r];
  rv[idx] = T(0.5) * s;
}

template <typename T>
__global__ __launch_bounds__(kMW) void k_pj_prolong_add_m(const T* ev, T* xface, int n, int R) {
  const int64_t nf = 2LL * n * (n - 1), nv = (int64_t)n * (n - 1);
  const int64_t idx = (int64_t)blockIdx.x * kMW + threadIdx.x;
  if (idx >= nf * R) return;
  const int64_t f = idx / R;
  const int r = (int)(idx - f * R);
  int ai, aj, bi, bj;
  if (f < nv) {
    const int j = (int)(f / (n - 1)), i = (int)(f % (n - 1)) + 1;
    ai = i; aj = j; bi = i; bj = j + 1;
  } else {
    const int64_t q = f - nv;
    const int j = (int)(q / n) + 1, i = (int)(q % n);
    ai = i; aj = j; bi = i + 1; bj = j;
  }
  T s = T(0);
  {  // end vertices on the boundary read a clamped vertex and are zeroed
    const bool oa = ai >= 1 && aj >= 1 && ai <= n - 1 && aj <= n - 1;
    const bool ob = bi >= 1 && bj >= 1 && bi <= n - 1 && bj <= n - 1;
    const T ea = ev[((min(max(ai, 1), n - 1) - 1) + (int64_t)(n - 1) * (min(max(aj, 1), n - 1) - 1)) * R + r];
    const T eb = ev[((min(max(bi, 1), n - 1) - 1) + (int64_t)(n - 1) * (min(max(bj, 1), n - 1) - 1)) * R + r];
    s += oa ? ea : T(0);
    s += ob ? eb : T(0);
  }
  xface[idx] += T(0.5) * s;
}

// Y = A B with the FP64 dense coarsest inverse A (m x m) and B [m][R]: one
// workgroup per row; lanes run over right-hand sides, FP64 accumulation in
// column order.
template <typename T>
__global__ __launch_bounds__(64) void k_dense_gemm_m(const double* A, const T* B, T* Y, int m, int R) {
  const int row = blockIdx.x;
  for (int r = threadIdx.x; r < R; r += 64) {
    double s = 0.0;
    for (int c = 0; c < m; ++c) s += A[(int64_t)row * m + c] * (double)B[(int64_t)c * R + r];
    Y[(int64_t)row * R + r] = T(s);
  }
}

hipError_t launch_q1_resid_m(Prec pr, const void* st, const void* b, const void* x, void* r, int m, int R,
                             hipStream_t s) {
  HDG_MDISPATCH_T(pr, hipLaunchKernelGGL(k_q1_resid_m<TT>, grid_m((int64_t)(m - 1) * (m - 1) * R), dim3(kMW), 0, s,
                                         (const TT*)st, (const TT*)b, (const TT*)x, (TT*)r, m, R));
  return hipGetLastError();
}
hipError_t launch_q1_cheb_m(Prec pr, const void* st, const void* dinv, const void* b, const void* x, void* d,
                            void* xo, double c1, double c2, int m, int R, hipStream_t s) {
  HDG_MDISPATCH_T(pr, hipLaunchKernelGGL(k_q1_cheb_m<TT>, grid_m((int64_t)(m - 1) * (m - 1) * R), dim3(kMW), 0, s,
                                         (const TT*)st, (const TT*)dinv, (const TT*)b, (const TT*)x, (TT*)d,
                                         (TT*)xo, c1, c2, m, R));
  return hipGetLastError();
}
hipError_t launch_q1_restrict_m(Prec pr, const void* rf, void* rc, int mf, int R, hipStream_t s) {
  const int mc = mf / 2;
  HDG_MDISPATCH_T(pr, hipLaunchKernelGGL(k_q1_restrict_m<TT>, grid_m((int64_t)(mc - 1) * (mc - 1) * R), dim3(kMW),
                                         0, s, (const TT*)rf, (TT*)rc, mf, R));
  return hipGetLastError();
}
hipError_t launch_q1_prolong_add_m(Prec pr, const void* ec, void* xf, int mf, int R, hipStream_t s) {
  HDG_MDISPATCH_T(pr, hipLaunchKernelGGL(k_q1_prolong_add_m<TT>, grid_m((int64_t)(mf - 1) * (mf - 1) * R),
                                         dim3(kMW), 0, s, (const TT*)ec, (TT*)xf, mf, R));
  return hipGetLastError();
}
hipError_t launch_pj_restrict_m(Prec pr, const void* rface, void* rv, int n, int R, hipStream_t s) {
  HDG_MDISPATCH_T(pr, hipLaunchKernelGGL(k_pj_restrict_m<TT>, grid_m((int64_t)(n - 1) * (n - 1) * R), dim3(kMW), 0,
                                         s, (const TT*)rface, (TT*)rv, n, R));
  return hipGetLastError();
}
hipError_t launch_pj_prolong_add_m(Prec pr, const void* ev, void* xface, int n, int R, hipStream_t s) {
  HDG_MDISPATCH_T(pr, hipLaunchKernelGGL(k_pj_prolong_add_m<TT>, grid_m(2LL * n * (n - 1) * R), dim3(kMW), 0, s,
                                         (const TT*)ev, (TT*)xface, n, R));
  return hipGetLastError();
}
hipError_t launch_dense_gemm_m(Prec pr, const double* A, const void* b, void* y, int m, int R, hipStream_t s) {
  HDG_MDISPATCH_T(pr, hipLaunchKernelGGL(k_dense_gemm_m<TT>, dim3((unsigned)m), dim3(64), 0, s, A, (const TT*)b,
                                         (TT*)y, m, R));
  return hipGetLastError();
}

// ----------------------------------------------------------- chain Schwarz
// out = x + omega M^{-1} r for R right-hand sides: the block cyclic reduction of
// k_chain for a chunk of RC (a power of two) right-hand sides per workgroup.
// The chunk sits in LDS in k_chain's level order: word w (a position's row)
// holds the RC columns at w RCP + c, RCP = RC + 1 (odd) for RC > 1, so lanes
// whose words are consecutive fall in different banks.  Forward reduction:
// a work item is one (row, position) pair, which loads its factor row once and
// loops over the columns.  Back substitution: a work item is one (position,
// column) pair, column fastest, computing every row of its position for its
// column; it owns those values, so results are written as soon as they are
// computed (the RC lanes of one position load the same factor entries, one
// transaction for all).  Factors come by buffer loads (one register offset per
// lane, a wave-uniform offset per entry), unconditional at clamped indices and
// masked afterwards (the factors are finite).  The chunks of one chain are
// consecutive workgroups of one XCD (workgroups are dealt round-robin to the
// 8 XCDs), so the factor re-reads of later chunks come from that XCD's L2.
// At most 256 threads and at least 2 waves per SIMD (256 registers): a chunk
// of up to 64 KiB of LDS allows 2 workgroups per CU, so more registers cost no
// occupancy.
template <int P, typename T>
__global__ __launch_bounds__(256, 2) void k_chain_m(ChainMultiArgs a) {
  constexpr int P2 = P * P;
  constexpr int S = (int)sizeof(T);
  extern __shared__ unsigned char lds_raw_m[];
  T* Rl = reinterpret_cast<T*>(lds_raw_m);
  const T* rin = static_cast<const T*>(a.r);
  const T* xin = static_cast<const T*>(a.x);
  T* out = static_cast<T*>(a.out);
  const int64_t nch = 2LL * a.n;
  const int64_t npairs = nch * a.nchunks;
  int64_t pair = blockIdx.x;
  if (npairs % 8 == 0) pair = (int64_t)(blockIdx.x & 7) * (npairs >> 3) + (blockIdx.x >> 3);
  const int64_t c = pair / a.nchunks;
  const int chunk = (int)(pair - c * a.nchunks);
  const int RC = a.rc;
  const int lg = __builtin_ctz((unsigned)RC);
  const int RCP = RC == 1 ? 1 : RC + 1;
  const int R = a.R;
  const int col0 = chunk * RC;
  const int m = a.n - 1;
  const int64_t nv = (int64_t)a.n * (a.n - 1);
  const bool vert = c < a.n;
  const int64_t base = vert ? c * (a.n - 1) : nv + (c - a.n);
  const int64_t stride = vert ? 1 : a.n;
  const T* F = static_cast<const T*>(a.factors) + c * a.cstride;
  const __amdgpu_buffer_rsrc_t fr = buffer_rsrc(F, (int)(a.cstride * S));
  const int t = threadIdx.x;
  const int nt = blockDim.x;
  auto slot = [m](int l, int pos, int& rs) -> int {  // as in k_chain
    if (pos == 0) {
      rs = 1;
      return P * (m - 1);
    }
    const int z = __builtin_ctz((unsigned)pos);
    const int lv = l + z;
    const int mlv = (m + (1 << lv) - 1) >> lv;
    rs = mlv >> 1;
    return P * (m - mlv) + (pos >> (z + 1));
  };
  // chunk in: lanes over (position, column), column fastest
  for (int j = t; j < m * RC; j += nt) {
    const int i = j >> lg, q0 = j & (RC - 1);
    const int col = col0 + q0;
    int rs;
    const int w = slot(0, i, rs);
    T v[P];
#pragma unroll
    for (int r = 0; r < P; ++r) v[r] = col < R ? rin[((base + stride * i) * P + r) * R + col] : T(0);
#pragma unroll
    for (int r = 0; r < P; ++r) Rl[(w + r * rs) * RCP + q0] = v[r];
  }
  lds_barrier();
  // forward reduction: M-_j = Z_{j-1}^T, M+_j = W_{j+1}^T
  int ml = m, lev = 0;
  int64_t off = 0;
  while (ml > 1) {
    const int ne = (ml + 1) >> 1, no = ml >> 1;
    const int ob = P * (m - ml);
    const int ob8 = (int)off * S;  // byte offset of the level's records
#pragma unroll
    for (int r = 0; r < P; ++r)
      for (int tt = t; tt < ne; tt += nt) {
        const int zi = min(max(tt - 1, 0), no - 1), wi = min(tt, no - 1);
        const bool zok = tt >= 1, wok = tt < no;
        T zm[P], wp[P];  // row r of M-_j and M+_j
#pragma unroll
        for (int q = 0; q < P; ++q) {
          const T z = buffer_load<T>(fr, zi * S, ob8 + (2 * P2 + q * P + r) * no * S);
          const T w = buffer_load<T>(fr, wi * S, ob8 + (P2 + q * P + r) * no * S);
          zm[q] = zok ? z : T(0);
          wp[q] = wok ? w : T(0);
        }
        int rs;
        const int wo = (slot(lev + 1, tt, rs) + r * rs) * RCP;
        for (int q0 = 0; q0 < RC; ++q0) {
          T v = Rl[wo + q0];
#pragma unroll
          for (int q = 0; q < P; ++q)
            v -= zm[q] * Rl[(ob + q * no + zi) * RCP + q0] + wp[q] * Rl[(ob + q * no + wi) * RCP + q0];
          Rl[wo + q0] = v;
        }
      }
    off += (int64_t)3 * P2 * no;
    ml = ne;
    ++lev;
    lds_barrier();
  }
  // last level: x_0 = Dinv r_0 for every column of the chunk
  {
    const int top = P * (m - 1);
    for (int q0 = t; q0 < RC; q0 += nt) {
      T v[P], xr[P];
#pragma unroll
      for (int q = 0; q < P; ++q) v[q] = Rl[(top + q) * RCP + q0];
#pragma unroll
      for (int r = 0; r < P; ++r) {
        xr[r] = T(0);
#pragma unroll
        for (int q = 0; q < P; ++q) xr[r] += F[off + r * P + q] * v[q];
      }
#pragma unroll
      for (int r = 0; r < P; ++r) Rl[(top + r) * RCP + q0] = xr[r];
    }
  }
  lds_barrier();
  // back substitution: x_j = Dinv_j r_j - W_j x_{j-1} - Z_j x_{j+1} (j odd)
  while (lev > 0) {
    --lev;
    ml = (m + (1 << lev) - 1) >> lev;
    const int no = ml >> 1;
    const int ob = P * (m - ml);
    int64_t lo = 0;
    for (int l = 0, s = m; l < lev; ++l, s = (s + 1) >> 1) lo += (int64_t)3 * P2 * (s >> 1);
    const int lo8 = (int)lo * S;
    for (int j = t; j < no * RC; j += nt) {
      const int tt = j >> lg, q0 = j & (RC - 1);
      int rl, rr;
      const int wl = slot(lev + 1, tt, rl);
      const bool right = 2 * tt + 2 < ml;
      const int wr = right ? slot(lev + 1, tt + 1, rr) : (rr = rl, wl);
      T own[P], xl[P], xrt[P];
#pragma unroll
      for (int q = 0; q < P; ++q) {
        own[q] = Rl[(ob + q * no + tt) * RCP + q0];
        xl[q] = Rl[(wl + q * rl) * RCP + q0];
        const T x = Rl[(wr + q * rr) * RCP + q0];
        xrt[q] = right ? x : T(0);
      }
      T res[P];
#pragma unroll
      for (int r = 0; r < P; ++r) {
        T s = T(0);
#pragma unroll
        for (int q = 0; q < P; ++q)
          s += buffer_load<T>(fr, tt * S, lo8 + (r * P + q) * no * S) * own[q] -
               buffer_load<T>(fr, tt * S, lo8 + (P2 + r * P + q) * no * S) * xl[q] -
               buffer_load<T>(fr, tt * S, lo8 + (2 * P2 + r * P + q) * no * S) * xrt[q];
        res[r] = s;
      }
#pragma unroll
      for (int r = 0; r < P; ++r) Rl[(ob + r * no + tt) * RCP + q0] = res[r];
    }
    lds_barrier();
  }
  for (int j = t; j < m * RC; j += nt) {
    const int i = j >> lg, q0 = j & (RC - 1);
    const int col = col0 + q0;
    if (col >= R) continue;
    int rs;
    const int w = slot(0, i, rs);
#pragma unroll
    for (int r = 0; r < P; ++r) {
      const int64_t g = ((base + stride * i) * P + r) * R + col;
      out[g] = (xin ? xin[g] : T(0)) + T(a.omega) * Rl[(w + r * rs) * RCP + q0];
    }
  }
}

// LDS bytes of a chunk of rc right-hand sides (column stride rc + 1 for rc > 1)
static size_t chain_multi_lds(int P, int n, int rc, size_t es) {
  return (size_t)(n - 1) * P * (size_t)(rc == 1 ? 1 : rc + 1) * es;
}

// Largest power-of-two chunk (at most 16 and at most R rounded up to a power
// of two) whose right-hand sides fit 64 KiB of LDS (2 workgroups per CU), or
// one column up to lds_cap; 0 if one column does not fit lds_cap.
int chain_multi_chunk(int P, int n, int R, size_t es, int64_t lds_cap) {
  const int64_t cap = lds_cap > 0 ? lds_cap : 65536;
  if ((int64_t)chain_multi_lds(P, n, 1, es) > cap) return 0;
  int rc = 1;
  while (rc < 16 && rc < R && chain_multi_lds(P, n, 2 * rc, es) <= 65536) rc *= 2;
  return rc;
}

hipError_t launch_chain_solve_m(Prec pr, int P, const ChainMultiArgs& a, hipStream_t s) {
  if (a.rc < 1 || (a.rc & (a.rc - 1)) || a.nchunks * a.rc < a.R) return hipErrorInvalidValue;
  const size_t lds = chain_multi_lds(P, a.n, a.rc, vec_bytes(pr));
  if ((int64_t)lds > (a.lds_cap > 0 ? a.lds_cap : 65536)) return hipErrorInvalidValue;
  const bool big = lds > 65536;  // beyond 64 KiB a kernel's dynamic LDS is raised explicitly
  // one (position, column) pair per lane: the first forward level has
  // ceil((n-1)/2) positions
  const int64_t items = (int64_t)(a.n / 2) * a.rc;
  int threads = a.threads > 0 ? a.threads : 64;
  while (a.threads <= 0 && threads < 256 && threads < items) threads *= 2;
  if (threads > 256 || threads % 64) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(2LL * a.n * a.nchunks));
  if (pr == Prec::F64) {
    HDG_MDISPATCH_P(P, if (big && hipFuncSetAttribute(reinterpret_cast<const void*>(&k_chain_m<PP, double>),
                                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
                         return hipErrorInvalidValue;
                    hipLaunchKernelGGL((k_chain_m<PP, double>), grid, dim3(threads), lds, s, a));
  } else {
    HDG_MDISPATCH_P(P, if (big && hipFuncSetAttribute(reinterpret_cast<const void*>(&k_chain_m<PP, float>),
                                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
                         return hipErrorInvalidValue;
                    hipLaunchKernelGGL((k_chain_m<PP, float>), grid, dim3(threads), lds, s, a));
  }
  return hipGetLastError();
}

// -------------------------------------------------- per-column reductions
// partial[b][r] = sum over this block's rows of x[i][r] y[i][r] (FP64); the
// block's threads take (row offset, column) = (t / R, t % R), R <= 256.
template <typename T>
__global__ __launch_bounds__(kMW) void k_dots_m(const T* x, const T* y, int64_t N, int R, double* partial) {
  __shared__ double acc[kMW];
  const int t = threadIdx.x;
  const int rpi = kMW / R;  // rows per iteration
  double s = 0.0;
  if (t < rpi * R) {
    const int r = t % R, row0 = t / R;
    for (int64_t i = (int64_t)blockIdx.x * rpi + row0; i < N; i += (int64_t)gridDim.x * rpi)
      s += (double)x[i * R + r] * (double)y[i * R + r];
  }
  acc[t] = s;
  __syncthreads();
  if (t < R) {
    double v = 0.0;
    for (int q = 0; q < rpi; ++q) v += acc[q * R + t];
    partial[(int64_t)blockIdx.x * R + t] = v;
  }
}
__global__ __launch_bounds__(kMW) void k_sum_m(const double* partial, int nb, int R, double* out) {
  for (int r = threadIdx.x; r < R; r += kMW) {
    double v = 0.0;
    for (int b = 0; b < nb; ++b) v += partial[(int64_t)b * R + r];
    out[r] = v;
  }
}

int dots_m_grid(int64_t N) {
  int64_t g = (N + 255) / 256;
  return (int)(g < 1 ? 1 : (g > 512 ? 512 : g));
}
hipError_t launch_dots_m(Prec pr, const void* x, const void* y, int64_t N, int R, double* partial, double* out,
                         hipStream_t s) {
  if (R < 1 || R > kMW) return hipErrorInvalidValue;
  const int g = dots_m_grid(N);
  HDG_MDISPATCH_T(pr, hipLaunchKernelGGL(k_dots_m<TT>, dim3(g), dim3(kMW), 0, s, (const TT*)x, (const TT*)y, N, R,
                                         partial));
  hipLaunchKernelGGL(k_sum_m, dim3(1), dim3(kMW), 0, s, partial, g, R, out);
  return hipGetLastError();
}

__device__ __forceinline__ double ratio_or_zero_m(double a, double b) {
  const double r = a / b;
  return (b > 0.0 && isfinite(r)) ? r : 0.0;
}
// y[i][r] += sign act[r] num[r] / den[r] x[i][r]
template <typename T>
__global__ __launch_bounds__(kMW) void k_axpy_m(const double* num, const double* den, const double* act,
                                                double sign, const T* x, T* y, int64_t N, int R) {
  const int64_t idx = (int64_t)blockIdx.x * kMW + threadIdx.x;
  if (idx >= N * R) return;
  const int r = (int)(idx % R);
  const double c = sign * ratio_or_zero_m(num[r], den[r]) * (act ? act[r] : 1.0);
  y[idx] += T(c) * x[idx];
}
// y[i][r] = x[i][r] + sign num[r] / den[r] y[i][r]
template <typename T>
__global__ __launch_bounds__(kMW) void k_xpby_m(const T* x, const double* num, const double* den, double sign, T* y,
                                                int64_t N, int R) {
  const int64_t idx = (int64_t)blockIdx.x * kMW + threadIdx.x;
  if (idx >= N * R) return;
  const int r = (int)(idx % R);
  y[idx] = x[idx] + T(sign * ratio_or_zero_m(num[r], den[r])) * y[idx];
}
// d.r of the new direction: s0 = s3 - (s2 / s1) s4 per column (sc = [5][R])
__global__ void k_fcg_scalars_m(double* sc, int R) {
  for (int r = threadIdx.x; r < R; r += blockDim.x)
    sc[r] = sc[3 * R + r] - ratio_or_zero_m(sc[2 * R + r], sc[R + r]) * sc[4 * R + r];
}

hipError_t launch_axpy_m(Prec pr, const double* num, const double* den, const double* act, double sign,
                         const void* x, void* y, int64_t N, int R, hipStream_t s) {
  if (N * R == 0) return hipSuccess;
  HDG_MDISPATCH_T(pr, hipLaunchKernelGGL(k_axpy_m<TT>, grid_m(N * R), dim3(kMW), 0, s, num, den, act, sign,
                                         (const TT*)x, (TT*)y, N, R));
  return hipGetLastError();
}
hipError_t launch_xpby_m(Prec pr, const void* x, const double* num, const double* den, double sign, void* y,
                         int64_t N, int R, hipStream_t s) {
  if (N * R == 0) return hipSuccess;
  HDG_MDISPATCH_T(pr, hipLaunchKernelGGL(k_xpby_m<TT>, grid_m(N * R), dim3(kMW), 0, s, (const TT*)x, num, den, sign,
                                         (TT*)y, N, R));
  return hipGetLastError();
}
hipError_t launch_fcg_scalars_m(double* sc, int R, hipStream_t s) {
  hipLaunchKernelGGL(k_fcg_scalars_m, dim3(1), dim3(256), 0, s, sc, R);
  return hipGetLastError();
}

}  // namespace hdg
