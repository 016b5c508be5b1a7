// gfx950 kernels of the HDG trace operator and its multigrid.
//
// Trace apply (Sec. 8, Alg. algo_mv): one lane per interior face, 64 faces per
// wavefront.  The face's 7 blocks (its own summed diagonal block plus the 6
// blocks coupling it to the other faces of its two elements) are streamed from
// a tile-interleaved layout so that every 16-byte load of a wavefront reads
// 1 KiB of contiguous memory; the 7 (p+1) neighbour trace values are gathered
// from x (L2 / MALL resident).  Each face writes only its own outputs: no
// atomics, no barriers, no coloring.  Consecutive workgroups take consecutive
// tiles: the hardware deals them round-robin to the 8 XCDs, so all XCDs stream
// neighbouring regions of the block array at any time (measured faster than
// giving each XCD its own contiguous range, which favours x reuse in its L2).
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace hdg {

typedef double dbl2 __attribute__((ext_vector_type(2)));

static constexpr int kWG = 256;

// Face neighbours (App. numbering): g[0] = f, g[1..3] = other faces of the lo
// element in local order, g[4..6] = other faces of the hi element; -1 = boundary.
__device__ __forceinline__ void face_neighbours(int n, int64_t nv, int64_t f, int64_t g[7]) {
  g[0] = f;
  if (f < nv) {  // vertical: lo (i-1, j), hi (i, j); others: lo {L,B,T}, hi {R,B,T}
    const int64_t j = f / (n - 1), i = f - j * (n - 1) + 1;
    g[1] = (i >= 2) ? f - 1 : -1;
    g[2] = (j >= 1) ? nv + (i - 1) + (int64_t)n * (j - 1) : -1;
    g[3] = (j <= n - 2) ? nv + (i - 1) + (int64_t)n * j : -1;
    g[4] = (i <= n - 2) ? f + 1 : -1;
    g[5] = (j >= 1) ? nv + i + (int64_t)n * (j - 1) : -1;
    g[6] = (j <= n - 2) ? nv + i + (int64_t)n * j : -1;
  } else {       // horizontal: lo (i, j-1), hi (i, j); others: lo {L,R,B}, hi {L,R,T}
    const int64_t q = f - nv, jm1 = q / n, i = q - jm1 * n, j = jm1 + 1;
    g[1] = (i >= 1) ? (i - 1) + (int64_t)(n - 1) * (j - 1) : -1;
    g[2] = (i <= n - 2) ? i + (int64_t)(n - 1) * (j - 1) : -1;
    g[3] = (j >= 2) ? f - n : -1;
    g[4] = (i >= 1) ? (i - 1) + (int64_t)(n - 1) * j : -1;
    g[5] = (i <= n - 2) ? i + (int64_t)(n - 1) * j : -1;
    g[6] = (j <= n - 2) ? f + n : -1;
  }
}

// Deterministic workgroup sum (fixed shuffle tree, then the 4 wave sums in order).
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double ws[kWG / 64];
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kWG / 64; ++w) s += ws[w];
  return s;
}

int trace_grid(int64_t ntiles) { return (int)((ntiles + 3) / 4); }
int trace_partials(int64_t ntiles) { return 4 * trace_grid(ntiles); }

template <int P, int MODE>
__global__ __launch_bounds__(kWG) void k_trace(TraceArgs a) {
  constexpr int P2 = P * P;
  constexpr int NE = 7 * P2;
  constexpr int NQ = (NE + 1) / 2;
  constexpr int NQD = (P2 + 1) / 2;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t tile = (int64_t)blockIdx.x * (kWG / 64) + wave;
  const int64_t nv = (int64_t)a.n * (a.n - 1);
  double sq = 0.0;
  if (tile < a.ntiles) {
    const int64_t f = tile * 64 + lane;
    const bool valid = f < a.nf;
    int64_t g[7];
    face_neighbours(a.n, nv, valid ? f : 0, g);
    double xv[7][P];
#pragma unroll
    for (int s = 0; s < 7; ++s)
#pragma unroll
      for (int c = 0; c < P; ++c) xv[s][c] = (valid && g[s] >= 0) ? a.x[g[s] * P + c] : 0.0;
    double acc[P];
#pragma unroll
    for (int r = 0; r < P; ++r) acc[r] = 0.0;
    const dbl2* sp = reinterpret_cast<const dbl2*>(a.slab) + (tile * NQ) * 64 + lane;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const dbl2 w = __builtin_nontemporal_load(sp + q * 64);
      const int e0 = 2 * q, e1 = 2 * q + 1;
      acc[(e0 % P2) / P] += w.x * xv[e0 / P2][e0 % P];
      if (e1 < NE) acc[(e1 % P2) / P] += w.y * xv[e1 / P2][e1 % P];
    }
    if (valid) {
      if constexpr (MODE == TM_APPLY || MODE == TM_APPLY_DOT) {
#pragma unroll
        for (int r = 0; r < P; ++r) a.y[f * P + r] = acc[r];
        if constexpr (MODE == TM_APPLY_DOT) {
#pragma unroll
          for (int r = 0; r < P; ++r) sq += xv[0][r] * acc[r];
        }
      } else {
        double res[P];
#pragma unroll
        for (int r = 0; r < P; ++r) {
          res[r] = a.b[f * P + r] - acc[r];
          sq += res[r] * res[r];
        }
        if constexpr (MODE == TM_RESID) {
#pragma unroll
          for (int r = 0; r < P; ++r) a.y[f * P + r] = res[r];
        } else if constexpr (MODE == TM_FACE_SWEEP) {
          const dbl2* dp = reinterpret_cast<const dbl2*>(a.dinv) + (tile * NQD) * 64 + lane;
          double z[P];
#pragma unroll
          for (int r = 0; r < P; ++r) z[r] = 0.0;
#pragma unroll
          for (int q = 0; q < NQD; ++q) {
            const dbl2 w = dp[q * 64];
            const int e0 = 2 * q, e1 = 2 * q + 1;
            z[e0 / P] += w.x * res[e0 % P];
            if (e1 < P2) z[e1 / P] += w.y * res[e1 % P];
          }
#pragma unroll
          for (int r = 0; r < P; ++r) a.y[f * P + r] = xv[0][r] + a.omega * z[r];
        } else {  // TM_RESID_RESTRICT, P >= 2: y[f (P-1) + c] = sum_r Pp[r][c] res[r]
          if constexpr (P >= 2) {
#pragma unroll
            for (int c = 0; c < P - 1; ++c) {
              double s = 0.0;
#pragma unroll
              for (int r = 0; r < P; ++r) s += a.pmat[r * (P - 1) + c] * res[r];
              a.y[f * (P - 1) + c] = s;
            }
          }
        }
      }
    }
  }
  if (a.partial != nullptr) {  // per-wavefront partial, fixed shuffle tree, no barrier
    for (int off = 32; off >= 1; off >>= 1) sq += __shfl_xor(sq, off, 64);
    if (lane == 0) a.partial[(int64_t)blockIdx.x * (kWG / 64) + wave] = sq;
  }
}

template <int P>
static hipError_t launch_trace_p(int mode, const TraceArgs& a, hipStream_t s) {
  const dim3 grid(trace_grid(a.ntiles)), block(kWG);
  switch (mode) {
    case TM_APPLY: hipLaunchKernelGGL((k_trace<P, TM_APPLY>), grid, block, 0, s, a); break;
    case TM_APPLY_DOT: hipLaunchKernelGGL((k_trace<P, TM_APPLY_DOT>), grid, block, 0, s, a); break;
    case TM_RESID: hipLaunchKernelGGL((k_trace<P, TM_RESID>), grid, block, 0, s, a); break;
    case TM_FACE_SWEEP: hipLaunchKernelGGL((k_trace<P, TM_FACE_SWEEP>), grid, block, 0, s, a); break;
    case TM_RESID_RESTRICT:
      if (P < 2) return hipErrorInvalidValue;
      hipLaunchKernelGGL((k_trace<P, TM_RESID_RESTRICT>), grid, block, 0, s, a);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_trace(int P, int mode, const TraceArgs& a, hipStream_t s) {
  switch (P) {
    case 1: return launch_trace_p<1>(mode, a, s);
    case 2: return launch_trace_p<2>(mode, a, s);
    case 3: return launch_trace_p<3>(mode, a, s);
    case 4: return launch_trace_p<4>(mode, a, s);
    case 5: return launch_trace_p<5>(mode, a, s);
    case 6: return launch_trace_p<6>(mode, a, s);
    case 7: return launch_trace_p<7>(mode, a, s);
    case 8: return launch_trace_p<8>(mode, a, s);
    case 9: return launch_trace_p<9>(mode, a, s);
    default: return hipErrorInvalidValue;
  }
}

// ------------------------------------------------------------ face-local ops
template <int P>
__global__ __launch_bounds__(kWG) void k_dinv_apply(const double* dinv, const double* b, double omega,
                                                    double* x, int64_t nf) {
  constexpr int P2 = P * P, NQD = (P2 + 1) / 2;
  const int64_t f = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (f >= nf) return;
  const int64_t tile = f >> 6;
  const int lane = (int)(f & 63);
  double r[P], z[P];
#pragma unroll
  for (int c = 0; c < P; ++c) { r[c] = b[f * P + c]; z[c] = 0.0; }
  const dbl2* dp = reinterpret_cast<const dbl2*>(dinv) + (tile * NQD) * 64 + lane;
#pragma unroll
  for (int q = 0; q < NQD; ++q) {
    const dbl2 w = dp[q * 64];
    const int e0 = 2 * q, e1 = 2 * q + 1;
    z[e0 / P] += w.x * r[e0 % P];
    if (e1 < P2) z[e1 / P] += w.y * r[e1 % P];
  }
#pragma unroll
  for (int c = 0; c < P; ++c) x[f * P + c] = omega * z[c];
}

template <int P>
__global__ __launch_bounds__(kWG) void k_p_restrict(const double* pm, const double* rf, double* rc,
                                                    int64_t nf) {
  const int64_t f = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (f >= nf) return;
  double r[P];
#pragma unroll
  for (int a = 0; a < P; ++a) r[a] = rf[f * P + a];
#pragma unroll
  for (int c = 0; c < P - 1; ++c) {
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < P; ++a) s += pm[a * (P - 1) + c] * r[a];
    rc[f * (P - 1) + c] = s;
  }
}

template <int P>
__global__ __launch_bounds__(kWG) void k_p_prolong_add(const double* pm, const double* ec, double* xf,
                                                       int64_t nf) {
  const int64_t f = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (f >= nf) return;
  double e[P - 1];
#pragma unroll
  for (int c = 0; c < P - 1; ++c) e[c] = ec[f * (P - 1) + c];
#pragma unroll
  for (int a = 0; a < P; ++a) {
    double s = xf[f * P + a];
#pragma unroll
    for (int c = 0; c < P - 1; ++c) s += pm[a * (P - 1) + c] * e[c];
    xf[f * P + a] = s;
  }
}

static inline dim3 grid_for(int64_t n) { return dim3((unsigned)((n + kWG - 1) / kWG)); }

#define HDG_DISPATCH_P(P, CALL)                       \
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

hipError_t launch_dinv_apply(int P, const double* dinv, const double* b, double omega, double* x,
                             int64_t nf, hipStream_t s) {
  if (nf == 0) return hipSuccess;
  HDG_DISPATCH_P(P, hipLaunchKernelGGL((k_dinv_apply<PP>), grid_for(nf), dim3(kWG), 0, s, dinv, b,
                                       omega, x, nf));
  return hipGetLastError();
}

hipError_t launch_p_restrict(int P, const double* pm, const double* rf, double* rc, int64_t nf,
                             hipStream_t s) {
  if (P < 2) return hipErrorInvalidValue;
  if (nf == 0) return hipSuccess;
  HDG_DISPATCH_P(P, if constexpr (PP >= 2) hipLaunchKernelGGL((k_p_restrict<PP>), grid_for(nf),
                                                               dim3(kWG), 0, s, pm, rf, rc, nf));
  return hipGetLastError();
}

hipError_t launch_p_prolong_add(int P, const double* pm, const double* ec, double* xf, int64_t nf,
                                hipStream_t s) {
  if (P < 2) return hipErrorInvalidValue;
  if (nf == 0) return hipSuccess;
  HDG_DISPATCH_P(P, if constexpr (PP >= 2) hipLaunchKernelGGL((k_p_prolong_add<PP>), grid_for(nf),
                                                               dim3(kWG), 0, s, pm, ec, xf, nf));
  return hipGetLastError();
}

// ------------------------------------------------------------ chain Schwarz
// Exact solve with the block-tridiagonal matrix of every chain of faces (2n
// chains: vertical faces of element row c, then horizontal faces of element
// column c - n), by block cyclic reduction with factors precomputed at setup.
// One workgroup per chain; the right-hand side lives in LDS and is reduced in
// place.  Level l keeps the positions i = j 2^l with j even:
//   forward   r_j <- r_j - M-_j r_{j-1} - M+_j r_{j+1}           (j even)
//   last      x_0 = Dinv r_0
//   backward  x_j = Dinv_j r_j - W_j x_{j-1} - Z_j x_{j+1}        (j odd)
// with W = Dinv A, Z = Dinv C.  One thread per (position, row): it streams one
// row of the position's blocks, so registers stay at a few times P for every
// degree.  Factors of a level of size ml: the even records [M-, M+] as 2 P^2
// arrays over the ne = ceil(ml/2) even positions, then the odd records
// [Dinv, W, Z] as 3 P^2 arrays over the no = floor(ml/2) odd positions
// (entry-major, so a wavefront reads consecutive addresses); the last level
// stores Dinv of its single block.
template <int P>
__global__ __launch_bounds__(1024) void k_chain(ChainArgs a) {
  constexpr int P2 = P * P;
  extern __shared__ double R[];
  const int64_t c = blockIdx.x;
  const int m = a.n - 1;
  const int64_t nv = (int64_t)a.n * (a.n - 1);
  const bool vert = c < a.n;
  const int64_t base = vert ? c * (a.n - 1) : nv + (c - a.n);
  const int64_t stride = vert ? 1 : a.n;
  const double* F = a.factors + c * a.cstride;
  const int t = threadIdx.x;
  const int nt = blockDim.x;
  for (int idx = t; idx < m * P; idx += nt) {
    const int i = idx / P, r = idx - i * P;
    R[idx] = a.r[(base + stride * i) * P + r];
  }
  int ml = m, lev = 0;
  int64_t off = 0;
  // factor row of this thread's first item of the coming phase, loaded before the
  // barrier that precedes the phase (factors do not depend on the data)
  double pm[P], pp[P];
  auto prefetch_fwd = [&](int mlv, int64_t offv) {
    const int ne = (mlv + 1) >> 1;
    if (mlv > 1 && t < ne * P) {
      const int r = t / ne, tt = t - r * ne;
      const double* E = F + offv;
#pragma unroll
      for (int q = 0; q < P; ++q) {
        pm[q] = E[(int64_t)(r * P + q) * ne + tt];
        pp[q] = E[(int64_t)(P2 + r * P + q) * ne + tt];
      }
    }
  };
  prefetch_fwd(ml, off);
  __syncthreads();
  while (ml > 1) {
    const int ne = (ml + 1) >> 1;
    const double* E = F + off;
    for (int it = t; it < ne * P; it += nt) {
      const int r = it / ne, tt = it - r * ne;
      const int j = 2 * tt;
      const int i = j << lev;
      if (it != t) {
#pragma unroll
        for (int q = 0; q < P; ++q) {
          pm[q] = E[(int64_t)(r * P + q) * ne + tt];
          pp[q] = E[(int64_t)(P2 + r * P + q) * ne + tt];
        }
      }
      double v = R[i * P + r];
      if (j >= 1) {
        const int il = (j - 1) << lev;
#pragma unroll
        for (int q = 0; q < P; ++q) v -= pm[q] * R[il * P + q];
      }
      if (j + 1 < ml) {
        const int ir = (j + 1) << lev;
#pragma unroll
        for (int q = 0; q < P; ++q) v -= pp[q] * R[ir * P + q];
      }
      R[i * P + r] = v;
    }
    off += (int64_t)2 * P2 * ne + (int64_t)3 * P2 * (ml >> 1);
    ml = ne;
    ++lev;
    prefetch_fwd(ml, off);
    __syncthreads();
  }
  double xr = 0.0;
  if (t < P) {
#pragma unroll
    for (int q = 0; q < P; ++q) xr += F[off + t * P + q] * R[q];
  }
  __syncthreads();
  if (t < P) R[t] = xr;
  __syncthreads();
  while (lev > 0) {
    --lev;
    ml = (m + (1 << lev) - 1) >> lev;
    const int ne = (ml + 1) >> 1, no = ml >> 1;
    int64_t lo = 0;  // offset of level lev: record sizes of the levels below it
    for (int l = 0, s = m; l < lev; ++l, s = (s + 1) >> 1)
      lo += (int64_t)2 * P2 * ((s + 1) >> 1) + (int64_t)3 * P2 * (s >> 1);
    const double* O = F + lo + (int64_t)2 * P2 * ne;
    // one pass computes every (position, row) value into registers; a thread
    // handles at most ceil(no P / blockDim) of them, bounded below by kMaxItems
    constexpr int kMaxItems = 8;
    double res[kMaxItems];
    int cnt = 0;
    for (int it = t; it < no * P && cnt < kMaxItems; it += nt, ++cnt) {
      const int r = it / no, tt = it - r * no;
      const int j = 2 * tt + 1;
      const int i = j << lev;
      const int il = (j - 1) << lev;
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < P; ++q)
        s += O[(int64_t)(r * P + q) * no + tt] * R[i * P + q] - O[(int64_t)(P2 + r * P + q) * no + tt] * R[il * P + q];
      if (j + 1 < ml) {
        const int ir = (j + 1) << lev;
#pragma unroll
        for (int q = 0; q < P; ++q) s -= O[(int64_t)(2 * P2 + r * P + q) * no + tt] * R[ir * P + q];
      }
      res[cnt] = s;
    }
    __syncthreads();
    cnt = 0;
    for (int it = t; it < no * P && cnt < kMaxItems; it += nt, ++cnt) {
      const int r = it / no, tt = it - r * no;
      R[((2 * tt + 1) << lev) * P + r] = res[cnt];
    }
    __syncthreads();
  }
  for (int idx = t; idx < m * P; idx += nt) {
    const int i = idx / P, r = idx - i * P;
    const int64_t g = (base + stride * i) * P + r;
    a.out[g] = (a.x ? a.x[g] : 0.0) + a.omega * R[idx];
  }
}

hipError_t launch_chain_solve(int P, const ChainArgs& a, hipStream_t s) {
  const int64_t nch = 2LL * a.n;
  const size_t lds = (size_t)(a.n - 1) * P * sizeof(double);
  // the back-substitution keeps at most 8 (position, row) items per thread
  const int64_t items = (int64_t)((a.n - 1) / 2) * P;
  int threads = 256;
  while (threads < 1024 && items > (int64_t)threads * 8) threads *= 2;
  if (items > (int64_t)threads * 8) return hipErrorInvalidValue;
  HDG_DISPATCH_P(P, hipLaunchKernelGGL((k_chain<PP>), dim3((unsigned)nch), dim3(threads), lds, s, a));
  return hipGetLastError();
}

// ------------------------------------------------------------------ Q1 levels
__device__ __forceinline__ double q1_apply(const double* st, const double* x, int m, int64_t Nv,
                                           int i, int j, int64_t v) {
  double s = 0.0;
#pragma unroll
  for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
    for (int di = -1; di <= 1; ++di) {
      const int ii = i + di, jj = j + dj;
      if (ii >= 1 && jj >= 1 && ii <= m - 1 && jj <= m - 1)
        s += st[(int64_t)((di + 1) + 3 * (dj + 1)) * Nv + v] * x[(ii - 1) + (int64_t)(m - 1) * (jj - 1)];
    }
  return s;
}

__global__ __launch_bounds__(kWG) void k_q1_resid(const double* st, const double* b, const double* x,
                                                  double* r, int m) {
  const int64_t Nv = (int64_t)(m - 1) * (m - 1);
  const int64_t v = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (v >= Nv) return;
  const int i = (int)(v % (m - 1)) + 1, j = (int)(v / (m - 1)) + 1;
  r[v] = b[v] - q1_apply(st, x, m, Nv, i, j, v);
}

__global__ __launch_bounds__(kWG) void k_q1_cheb(const double* st, const double* dinv, const double* b,
                                                 const double* x, double* d, double* xo, double c1,
                                                 double c2, int m) {
  const int64_t Nv = (int64_t)(m - 1) * (m - 1);
  const int64_t v = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (v >= Nv) return;
  const int i = (int)(v % (m - 1)) + 1, j = (int)(v / (m - 1)) + 1;
  const double ax = x ? q1_apply(st, x, m, Nv, i, j, v) : 0.0;
  const double z = dinv[v] * (b[v] - ax);
  const double dn = (c1 != 0.0 ? c1 * d[v] : 0.0) + c2 * z;
  d[v] = dn;
  xo[v] = (x ? x[v] : 0.0) + dn;
}

// full weighting: coarse vertex (I, J) gathers fine (2I + di, 2J + dj), weight w(di) w(dj)
__global__ __launch_bounds__(kWG) void k_q1_restrict(const double* rf, double* rc, int mf) {
  const int mc = mf / 2;
  const int64_t Nc = (int64_t)(mc - 1) * (mc - 1);
  const int64_t v = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (v >= Nc) return;
  const int I = (int)(v % (mc - 1)) + 1, J = (int)(v / (mc - 1)) + 1;
  double s = 0.0;
#pragma unroll
  for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
    for (int di = -1; di <= 1; ++di) {
      const double w = (di == 0 ? 1.0 : 0.5) * (dj == 0 ? 1.0 : 0.5);
      const int fi = 2 * I + di, fj = 2 * J + dj;  // always interior of the fine mesh
      s += w * rf[(fi - 1) + (int64_t)(mf - 1) * (fj - 1)];
    }
  rc[v] = s;
}

__global__ __launch_bounds__(kWG) void k_q1_prolong_add(const double* ec, double* xf, int mf) {
  const int mc = mf / 2;
  const int64_t Nf = (int64_t)(mf - 1) * (mf - 1);
  const int64_t v = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (v >= Nf) return;
  const int I = (int)(v % (mf - 1)) + 1, J = (int)(v / (mf - 1)) + 1;
  int xi[2], yi[2];
  double wx[2], wy[2];
  int nx, ny;
  if ((I & 1) == 0) { xi[0] = I / 2; wx[0] = 1.0; nx = 1; } else { xi[0] = I / 2; xi[1] = I / 2 + 1; wx[0] = wx[1] = 0.5; nx = 2; }
  if ((J & 1) == 0) { yi[0] = J / 2; wy[0] = 1.0; ny = 1; } else { yi[0] = J / 2; yi[1] = J / 2 + 1; wy[0] = wy[1] = 0.5; ny = 2; }
  double s = 0.0;
  for (int b = 0; b < ny; ++b)
    for (int a = 0; a < nx; ++a) {
      const int ci = xi[a], cj = yi[b];
      if (ci >= 1 && cj >= 1 && ci <= mc - 1 && cj <= mc - 1)
        s += wx[a] * wy[b] * ec[(ci - 1) + (int64_t)(mc - 1) * (cj - 1)];
    }
  xf[v] += s;
}

// P_J^T: vertex (i, j) gathers its four incident interior faces, weight 1/2
__global__ __launch_bounds__(kWG) void k_pj_restrict(const double* rface, double* rv, int n) {
  const int64_t Nv = (int64_t)(n - 1) * (n - 1);
  const int64_t v = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (v >= Nv) return;
  const int i = (int)(v % (n - 1)) + 1, j = (int)(v / (n - 1)) + 1;
  const int64_t nv = (int64_t)n * (n - 1);
  const double s = rface[(i - 1) + (int64_t)(n - 1) * j] + rface[(i - 1) + (int64_t)(n - 1) * (j - 1)] +
                   rface[nv + i + (int64_t)n * (j - 1)] + rface[nv + (i - 1) + (int64_t)n * (j - 1)];
  rv[v] = 0.5 * s;
}

// P_J: face value += mean of its two end vertices (boundary vertices are 0)
__global__ __launch_bounds__(kWG) void k_pj_prolong_add(const double* ev, double* xface, int n) {
  const int64_t nf = 2LL * n * (n - 1), nv = (int64_t)n * (n - 1);
  const int64_t f = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (f >= nf) return;
  int ai, aj, bi, bj;
  if (f < nv) {
    const int j = (int)(f / (n - 1)), i = (int)(f % (n - 1)) + 1;
    ai = i; aj = j; bi = i; bj = j + 1;
  } else {
    const int64_t q = f - nv;
    const int j = (int)(q / n) + 1, i = (int)(q % n);
    ai = i; aj = j; bi = i + 1; bj = j;
  }
  double s = 0.0;
  if (ai >= 1 && aj >= 1 && ai <= n - 1 && aj <= n - 1) s += ev[(ai - 1) + (int64_t)(n - 1) * (aj - 1)];
  if (bi >= 1 && bj >= 1 && bi <= n - 1 && bj <= n - 1) s += ev[(bi - 1) + (int64_t)(n - 1) * (bj - 1)];
  xface[f] += 0.5 * s;
}

// one wavefront per row, lanes stride the columns, fixed shuffle-tree sum
__global__ __launch_bounds__(kWG) void k_dense_gemv(const double* A, const double* b, double* y, int m) {
  const int row = blockIdx.x * (kWG / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= m) return;
  double s = 0.0;
  for (int c = lane; c < m; c += 64) s += A[(int64_t)row * m + c] * b[c];
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) y[row] = s;
}

hipError_t launch_q1_resid(const double* st, const double* b, const double* x, double* r, int m,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_q1_resid, grid_for((int64_t)(m - 1) * (m - 1)), dim3(kWG), 0, s, st, b, x, r, m);
  return hipGetLastError();
}
hipError_t launch_q1_cheb(const double* st, const double* dinv, const double* b, const double* x,
                          double* d, double* xo, double c1, double c2, int m, hipStream_t s) {
  hipLaunchKernelGGL(k_q1_cheb, grid_for((int64_t)(m - 1) * (m - 1)), dim3(kWG), 0, s, st, dinv, b, x,
                     d, xo, c1, c2, m);
  return hipGetLastError();
}
hipError_t launch_q1_restrict(const double* rf, double* rc, int mf, hipStream_t s) {
  const int mc = mf / 2;
  hipLaunchKernelGGL(k_q1_restrict, grid_for((int64_t)(mc - 1) * (mc - 1)), dim3(kWG), 0, s, rf, rc, mf);
  return hipGetLastError();
}
hipError_t launch_q1_prolong_add(const double* ec, double* xf, int mf, hipStream_t s) {
  hipLaunchKernelGGL(k_q1_prolong_add, grid_for((int64_t)(mf - 1) * (mf - 1)), dim3(kWG), 0, s, ec, xf, mf);
  return hipGetLastError();
}
hipError_t launch_pj_restrict(const double* rface, double* rv, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_pj_restrict, grid_for((int64_t)(n - 1) * (n - 1)), dim3(kWG), 0, s, rface, rv, n);
  return hipGetLastError();
}
hipError_t launch_pj_prolong_add(const double* ev, double* xface, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_pj_prolong_add, grid_for(2LL * n * (n - 1)), dim3(kWG), 0, s, ev, xface, n);
  return hipGetLastError();
}
hipError_t launch_dense_gemv(const double* A, const double* b, double* y, int m, hipStream_t s) {
  hipLaunchKernelGGL(k_dense_gemv, dim3((m + 3) / 4), dim3(kWG), 0, s, A, b, y, m);
  return hipGetLastError();
}

// ---------------------------------------------------------------- reductions
int reduce_grid(int64_t n) {
  int64_t g = (n + kWG * 4 - 1) / (kWG * 4);
  if (g > 1024) g = 1024;
  if (g < 1) g = 1;
  return (int)g;
}

__global__ __launch_bounds__(kWG) void k_dot_partials(const double* a, const double* b, int64_t n,
                                                      double* partial) {
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kWG)
    s += a[i] * b[i];
  const double t = block_sum(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ __launch_bounds__(kWG) void k_sum_partials(const double* partial, int np, double* out) {
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += kWG) s += partial[i];
  const double t = block_sum(s);
  if (threadIdx.x == 0) *out = t;
}

__global__ __launch_bounds__(kWG) void k_axpy(double alpha, const double* x, double* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i < n) y[i] += alpha * x[i];
}
__global__ __launch_bounds__(kWG) void k_xpby(const double* x, double beta, double* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i < n) y[i] = x[i] + beta * y[i];
}
__global__ __launch_bounds__(kWG) void k_axpy_norm(double alpha, const double* q, double* r, int64_t n,
                                                   double* partial) {
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kWG) {
    const double v = r[i] - alpha * q[i];
    r[i] = v;
    s += v * v;
  }
  const double t = block_sum(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}
__global__ __launch_bounds__(kWG) void k_copy(const double* x, double* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i < n) y[i] = x[i];
}
__global__ __launch_bounds__(kWG) void k_fill(double v, double* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i < n) y[i] = v;
}

hipError_t launch_dot_partials(const double* a, const double* b, int64_t n, double* partial,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_dot_partials, dim3(reduce_grid(n)), dim3(kWG), 0, s, a, b, n, partial);
  return hipGetLastError();
}
hipError_t launch_sum_partials(const double* partial, int np, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kWG), 0, s, partial, np, out);
  return hipGetLastError();
}
hipError_t launch_axpy(double alpha, const double* x, double* y, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpy, grid_for(n), dim3(kWG), 0, s, alpha, x, y, n);
  return hipGetLastError();
}
hipError_t launch_xpby(const double* x, double beta, double* y, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_xpby, grid_for(n), dim3(kWG), 0, s, x, beta, y, n);
  return hipGetLastError();
}
hipError_t launch_axpy_norm(double alpha, const double* q, double* r, int64_t n, double* partial,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_norm, dim3(reduce_grid(n)), dim3(kWG), 0, s, alpha, q, r, n, partial);
  return hipGetLastError();
}
hipError_t launch_copy(const double* x, double* y, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, grid_for(n), dim3(kWG), 0, s, x, y, n);
  return hipGetLastError();
}
hipError_t launch_fill(double v, double* y, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, grid_for(n), dim3(kWG), 0, s, v, y, n);
  return hipGetLastError();
}

}  // namespace hdg
