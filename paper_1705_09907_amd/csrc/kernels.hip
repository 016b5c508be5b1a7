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
//
// Every kernel is instantiated for FP64 blocks and vectors, FP32 blocks and
// vectors, and BF16 blocks with FP32 vectors (FP32 accumulation).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <mutex>

#include "device.hpp"
#include "kernels.hpp"

namespace hdg {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t bf16_t;  // bfloat16 storage: the high half of an FP32 word

static constexpr int kWG = 256;

// ---------------------------------------------------------------- storage
// 16-byte load of V = 16 / sizeof(TM) consecutive matrix entries, widened to TV.
template <typename TM, typename TV>
struct Lanes16;
template <>
struct Lanes16<double, double> {
  static constexpr int V = 2;
  __device__ static void unpack(u32x4 r, double* w) { __builtin_memcpy(w, &r, 16); }
};
template <>
struct Lanes16<float, float> {
  static constexpr int V = 4;
  __device__ static void unpack(u32x4 r, float* w) { __builtin_memcpy(w, &r, 16); }
};
template <>
struct Lanes16<bf16_t, float> {
  static constexpr int V = 8;
  __device__ static void unpack(u32x4 r, float* w) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const unsigned int u = r[i];
      w[2 * i] = __uint_as_float(u << 16);
      w[2 * i + 1] = __uint_as_float(u & 0xffff0000u);
    }
  }
};

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

template <int P, int MODE, typename TM, typename TV>
__global__ __launch_bounds__(kWG) void k_trace(TraceArgs a) {
  using L16 = Lanes16<TM, TV>;
  constexpr int V = L16::V;
  constexpr int P2 = P * P;
  constexpr int NE = 7 * P2;
  constexpr int NQ = (NE + V - 1) / V;
  constexpr int NQD = (P2 + V - 1) / V;
  const TV* x = static_cast<const TV*>(a.x);
  const TV* b = static_cast<const TV*>(a.b);
  TV* y = static_cast<TV*>(a.y);
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
    // missing neighbours (and lanes past the last face) gather an existing row
    // and zero it: no load sits under a branch
    TV xv[7][P];
#pragma unroll
    for (int s = 0; s < 7; ++s) {
      const bool ok = valid && g[s] >= 0;
      const int64_t gs = ok ? g[s] : 0;
#pragma unroll
      for (int c = 0; c < P; ++c) {
        const TV v = x[gs * P + c];
        xv[s][c] = ok ? v : TV(0);
      }
    }
    TV acc[P];
#pragma unroll
    for (int r = 0; r < P; ++r) acc[r] = TV(0);
    const u32x4* sp = static_cast<const u32x4*>(a.slab) + (tile * NQ) * 64 + lane;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      TV w[V];
      L16::unpack(__builtin_nontemporal_load(sp + q * 64), w);
#pragma unroll
      for (int u = 0; u < V; ++u) {
        const int e = q * V + u;
        if constexpr (MODE == TM_ABS) {
          if (e < NE) acc[(e % P2) / P] += fabs(w[u]) * fabs(xv[e / P2][e % P]);
        } else {
          if (e < NE) acc[(e % P2) / P] += w[u] * xv[e / P2][e % P];
        }
      }
    }
    if (valid) {
      if constexpr (MODE == TM_UPDATE) {
#pragma unroll
        for (int r = 0; r < P; ++r) {
          const TV base = b != nullptr ? b[f * P + r] : TV(0);
          y[f * P + r] = base + TV(a.omega) * acc[r];
        }
      } else if constexpr (MODE == TM_APPLY || MODE == TM_APPLY_DOT || MODE == TM_ABS) {
#pragma unroll
        for (int r = 0; r < P; ++r) y[f * P + r] = acc[r];
        if constexpr (MODE == TM_APPLY_DOT) {
#pragma unroll
          for (int r = 0; r < P; ++r) sq += (double)xv[0][r] * (double)acc[r];
        }
      } else {
        TV res[P];
#pragma unroll
        for (int r = 0; r < P; ++r) {
          res[r] = b[f * P + r] - acc[r];
          sq += (double)res[r] * (double)res[r];
        }
        if constexpr (MODE == TM_RESID) {
#pragma unroll
          for (int r = 0; r < P; ++r) y[f * P + r] = res[r];
        } else if constexpr (MODE == TM_FACE_SWEEP) {
          const u32x4* dp = static_cast<const u32x4*>(a.dinv) + (tile * NQD) * 64 + lane;
          TV z[P];
#pragma unroll
          for (int r = 0; r < P; ++r) z[r] = TV(0);
#pragma unroll
          for (int q = 0; q < NQD; ++q) {
            TV w[V];
            L16::unpack(dp[q * 64], w);
#pragma unroll
            for (int u = 0; u < V; ++u) {
              const int e = q * V + u;
              if (e < P2) z[e / P] += w[u] * res[e % P];
            }
          }
#pragma unroll
          for (int r = 0; r < P; ++r) y[f * P + r] = xv[0][r] + TV(a.omega) * z[r];
        } else {  // TM_RESID_RESTRICT, P >= 2: y[f (P-1) + c] = sum_r Pp[r][c] res[r]
          if constexpr (P >= 2) {
            const TV* pm = static_cast<const TV*>(a.pmat);
#pragma unroll
            for (int c = 0; c < P - 1; ++c) {
              TV s = TV(0);
#pragma unroll
              for (int r = 0; r < P; ++r) s += pm[r * (P - 1) + c] * res[r];
              y[f * (P - 1) + c] = s;
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

// ------------------------------------------------ many meshes in one launch
// y = S x on one 64-face tile of one mesh, by one wavefront: the APPLY path of
// k_trace<P, TM_APPLY, TM, TV> with the same loads and the same order of
// operations (TM: stored block entries, TV: vectors and accumulation).
template <int P, typename TM, typename TV>
__device__ __forceinline__ void apply_tile(const BatchMesh& M, int64_t tile, int lane) {
  using L16 = Lanes16<TM, TV>;
  constexpr int V = L16::V;
  constexpr int P2 = P * P;
  constexpr int NE = 7 * P2;
  constexpr int NQ = (NE + V - 1) / V;
  const TV* x = static_cast<const TV*>(M.x);
  TV* y = static_cast<TV*>(M.y);
  const int64_t nv = (int64_t)M.n * (M.n - 1);
  const int64_t f = tile * 64 + lane;
  const bool valid = f < M.nf;
  int64_t g[7];
  face_neighbours(M.n, nv, valid ? f : 0, g);
  TV xv[7][P];
#pragma unroll
  for (int s = 0; s < 7; ++s)
#pragma unroll
    for (int c = 0; c < P; ++c) xv[s][c] = (valid && g[s] >= 0) ? x[g[s] * P + c] : TV(0);
  TV acc[P];
#pragma unroll
  for (int r = 0; r < P; ++r) acc[r] = TV(0);
  const u32x4* sp = static_cast<const u32x4*>(M.slab) + (tile * NQ) * 64 + lane;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    TV w[V];
    L16::unpack(__builtin_nontemporal_load(sp + q * 64), w);
#pragma unroll
    for (int u = 0; u < V; ++u) {
      const int e = q * V + u;
      if (e < NE) acc[(e % P2) / P] += w[u] * xv[e / P2][e % P];
    }
  }
  if (valid) {
#pragma unroll
    for (int r = 0; r < P; ++r) y[f * P + r] = acc[r];
  }
}

// One mesh's tile with the block storage its descriptor names (FP64 blocks and
// vectors, or FP32 / bfloat16 blocks with FP32 vectors).
template <int P, bool LP>
__device__ __forceinline__ void apply_tile_any(const BatchMesh& M, int64_t tile, int lane) {
  if constexpr (LP) {
    if (M.mp == (int)Prec::BF16) apply_tile<P, bf16_t, float>(M, tile, lane);
    else apply_tile<P, float, float>(M, tile, lane);
  } else {
    apply_tile<P, double, double>(M, tile, lane);
  }
}

// A fixed grid of workgroups walks the list of (mesh, tile) items with a static
// stride (deterministic); wavefront w of workgroup b takes items 4 b + w,
// 4 b + w + 4 G, ...  Meshes are found by a scan of the tile offsets.  PMAX is
// the largest P compiled in: registers are sized for it, so the launcher takes
// the smallest instance that covers the batch (P <= 5: about half the registers
// of P <= 9).  LP: the meshes' cycle-precision operators (FP32 vectors).
template <int PMAX, bool LP>
__global__ __launch_bounds__(kWG) void k_trace_batch(const BatchMesh* meshes, int nmesh, int64_t total) {
  const int lane = threadIdx.x & 63;
  const int64_t nwaves = (int64_t)gridDim.x * (kWG / 64);
  for (int64_t item = (int64_t)blockIdx.x * (kWG / 64) + (threadIdx.x >> 6); item < total; item += nwaves) {
    int m = 0;
    while (m + 1 < nmesh && meshes[m + 1].tile0 <= item) ++m;
    const BatchMesh& M = meshes[m];
    const int64_t tile = item - M.tile0;
    switch (M.P) {
      case 1: apply_tile_any<1, LP>(M, tile, lane); break;
      case 2: apply_tile_any<2, LP>(M, tile, lane); break;
      case 3: apply_tile_any<3, LP>(M, tile, lane); break;
      case 4: apply_tile_any<4, LP>(M, tile, lane); break;
      case 5: apply_tile_any<5, LP>(M, tile, lane); break;
      default:
        if constexpr (PMAX > 5) {
          switch (M.P) {
            case 6: apply_tile_any<6, LP>(M, tile, lane); break;
            case 7: apply_tile_any<7, LP>(M, tile, lane); break;
            case 8: apply_tile_any<8, LP>(M, tile, lane); break;
            default: apply_tile_any<9, LP>(M, tile, lane); break;
          }
        }
        break;
    }
  }
}

hipError_t launch_trace_batch(const BatchMesh* meshes_dev, int nmesh, int64_t total_tiles, int grid, int pmax,
                              hipStream_t s, bool lp) {
  if (total_tiles == 0) return hipSuccess;
  if (lp) {
    if (pmax <= 5)
      hipLaunchKernelGGL((k_trace_batch<5, true>), dim3((unsigned)grid), dim3(kWG), 0, s, meshes_dev, nmesh,
                         total_tiles);
    else
      hipLaunchKernelGGL((k_trace_batch<9, true>), dim3((unsigned)grid), dim3(kWG), 0, s, meshes_dev, nmesh,
                         total_tiles);
  } else if (pmax <= 5) {
    hipLaunchKernelGGL((k_trace_batch<5, false>), dim3((unsigned)grid), dim3(kWG), 0, s, meshes_dev, nmesh,
                       total_tiles);
  } else {
    hipLaunchKernelGGL((k_trace_batch<9, false>), dim3((unsigned)grid), dim3(kWG), 0, s, meshes_dev, nmesh,
                       total_tiles);
  }
  return hipGetLastError();
}

// Descriptor table of the allocation-free many-mesh apply: a file-scope device
// array, one copy per GPU at its own address, held until the process ends.
// Host code never uses this name as an address: batch_scratch_address() looks
// the device address up once per device and every later use goes through it.
static __device__ __align__(256) BatchMesh scratch[kBatchNoallocMax];

hipError_t batch_scratch_address(void** out) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = p;
  }
  *out = addr[dev];
  return hipSuccess;
}

template <int P, typename TM, typename TV>
static hipError_t launch_trace_t(int mode, const TraceArgs& a, hipStream_t s) {
  const dim3 grid(trace_grid(a.ntiles)), block(kWG);
  switch (mode) {
    case TM_APPLY:
      if (a.ev_start)  // events recorded at the kernel's own start and end
        hipExtLaunchKernelGGL((k_trace<P, TM_APPLY, TM, TV>), grid, block, 0, s, (hipEvent_t)a.ev_start,
                              (hipEvent_t)a.ev_stop, 0, a);
      else
        hipLaunchKernelGGL((k_trace<P, TM_APPLY, TM, TV>), grid, block, 0, s, a);
      break;
    case TM_APPLY_DOT: hipLaunchKernelGGL((k_trace<P, TM_APPLY_DOT, TM, TV>), grid, block, 0, s, a); break;
    case TM_UPDATE: hipLaunchKernelGGL((k_trace<P, TM_UPDATE, TM, TV>), grid, block, 0, s, a); break;
    case TM_ABS:
      if constexpr (sizeof(TV) == 8) {
        hipLaunchKernelGGL((k_trace<P, TM_ABS, TM, TV>), grid, block, 0, s, a);
        break;
      } else {
        return hipErrorInvalidValue;
      }
    case TM_RESID: hipLaunchKernelGGL((k_trace<P, TM_RESID, TM, TV>), grid, block, 0, s, a); break;
    case TM_FACE_SWEEP: hipLaunchKernelGGL((k_trace<P, TM_FACE_SWEEP, TM, TV>), grid, block, 0, s, a); break;
    case TM_RESID_RESTRICT:
      if (P < 2) return hipErrorInvalidValue;
      hipLaunchKernelGGL((k_trace<P, TM_RESID_RESTRICT, TM, TV>), grid, block, 0, s, a);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int P>
static hipError_t launch_trace_p(Prec pr, int mode, const TraceArgs& a, hipStream_t s) {
  switch (pr) {
    case Prec::F64: return launch_trace_t<P, double, double>(mode, a, s);
    case Prec::F32: return launch_trace_t<P, float, float>(mode, a, s);
    case Prec::BF16: return launch_trace_t<P, bf16_t, float>(mode, a, s);
  }
  return hipErrorInvalidValue;
}

// ------------------------------------------------- many right-hand sides
// One workgroup per group of FW consecutive faces (FW divides 64, so a group
// lies in one tile): the group's 7 P^2 blocks are read once from the
// interleaved slab (runs of FW 16-byte words) into LDS, then threads take
// (face, right-hand side) pairs; with 64 or more right-hand sides a wavefront
// works on one face with its lanes over right-hand sides, so every x gather and
// y store is a contiguous 64-lane access and the block entries are LDS
// broadcasts.  LDS holds each block transposed with its columns padded to PQ
// (a multiple of 16 bytes), so the P entries that multiply one gathered x value
// come in a few 16-byte LDS reads.
template <int P, typename TV>
struct MultiGroup {
  static constexpr int FW = P <= 6 ? 16 : 8;
  static constexpr int PQ = sizeof(TV) == 8 ? (P + 1) / 2 * 2 : (P + 3) / 4 * 4;
};

template <int P, int MODE, typename TM, typename TV>
__global__ __launch_bounds__(256) void k_trace_multi(MultiArgs a) {
  using L16 = Lanes16<TM, TV>;
  constexpr int V = L16::V;
  constexpr int P2 = P * P;
  constexpr int NE = 7 * P2;
  constexpr int NQ = (NE + V - 1) / V;
  constexpr int FW = MultiGroup<P, TV>::FW;
  constexpr int PQ = MultiGroup<P, TV>::PQ;
  __shared__ __align__(16) TV blk[FW][7 * P * PQ];
  // a.remap: workgroups are dealt round-robin to the 8 XCDs; giving XCD x the
  // contiguous range of groups [x G/8, (x+1) G/8) lets its L2 serve the x rows
  // that neighbouring groups share
  const int64_t G = (a.nf + FW - 1) / FW;
  int64_t grp = blockIdx.x;
  if (a.remap && G % 8 == 0) grp = (int64_t)(blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
  const int64_t f0 = grp * FW;
  const int64_t tile = f0 >> 6;
  const int l0 = (int)(f0 & 63);
  const u32x4* sp = static_cast<const u32x4*>(a.slab) + tile * NQ * 64 + l0;
  for (int i = threadIdx.x; i < NQ * FW; i += blockDim.x) {
    const int q = i / FW, fl = i - q * FW;
    TV w[V];
    L16::unpack(__builtin_nontemporal_load(sp + q * 64 + fl), w);
#pragma unroll
    for (int u = 0; u < V; ++u) {
      const int e = q * V + u;  // slot s, row r, column c  ->  blk[s][c][r]
      if (e < NE) {
        const int s = e / P2, rc = e - s * P2, r = rc / P, c = rc - r * P;
        blk[fl][(s * P + c) * PQ + r] = w[u];
      }
    }
  }
  __syncthreads();
  const TV* X = static_cast<const TV*>(a.X);
  TV* Y = static_cast<TV*>(a.Y);
  const int R = a.nrhs;
  const int64_t nv = (int64_t)a.n * (a.n - 1);
  for (int pair = threadIdx.x; pair < FW * R; pair += blockDim.x) {
    const int fl = pair / R, r = pair - fl * R;
    const int64_t f = f0 + fl;
    if (f >= a.nf) continue;
    int64_t g[7];
    face_neighbours(a.n, nv, f, g);
    TV acc[P];
#pragma unroll
    for (int q = 0; q < P; ++q) acc[q] = TV(0);
    // missing (boundary) neighbours: the gather reads the face's own row and is
    // zeroed, so the 7 P steps form one branch-free block the compiler can pipeline
#pragma unroll
    for (int s = 0; s < 7; ++s) {
      const bool ok = g[s] >= 0;
      const int64_t gs = ok ? g[s] : f;
#pragma unroll
      for (int c = 0; c < P; ++c) {
        const TV xl = X[(gs * P + c) * R + r];
        const TV xv = ok ? xl : TV(0);
        const TV* col = &blk[fl][(s * P + c) * PQ];
#pragma unroll
        for (int q = 0; q < P; ++q) acc[q] += col[q] * xv;
      }
    }
    if constexpr (MODE == TM_APPLY) {
#pragma unroll
      for (int q = 0; q < P; ++q) Y[(f * P + q) * R + r] = acc[q];
    } else {
      const TV* B = static_cast<const TV*>(a.B);
#pragma unroll
      for (int q = 0; q < P; ++q) acc[q] = B[(f * P + q) * R + r] - acc[q];
      if constexpr (MODE == TM_RESID) {
#pragma unroll
        for (int q = 0; q < P; ++q) Y[(f * P + q) * R + r] = acc[q];
      } else if constexpr (P >= 2) {  // TM_RESID_RESTRICT: Y (coarse) = P_p^T (B - S X)
        const TV* pm = static_cast<const TV*>(a.pmat);
#pragma unroll
        for (int c = 0; c < P - 1; ++c) {
          TV s = TV(0);
#pragma unroll
          for (int q = 0; q < P; ++q) s += pm[q * (P - 1) + c] * acc[q];
          Y[(f * (P - 1) + c) * R + r] = s;
        }
      }
    }
  }
}

// ------------------------------- many right-hand sides on the matrix cores
// FP32 vectors (blocks FP32, or bfloat16 widened to FP32).  The per-face
// product Y_f [P x R] = B_f [P x 7P] X_f [7P x R] (X_f the gathered neighbour
// rows) runs on v_mfma_f32_4x4x1_16b_f32: sixteen independent 4 x 4 outer-product
// blocks per instruction, block b taking the right-hand sides 4b .. 4b+3 of a
// 64-column chunk and one group of 4 output rows (rows padded to a multiple of
// 4 with zero rows).  Lane l = 4b + j supplies x[k][column l] (the B operand,
// one coalesced 64-lane load per k) and row 4 rg + j of B_f at k (the A operand,
// the same for every block); it receives rows 4 rg .. 4 rg + 3 of column l.  So
// a lane owns one right-hand side of the face: 4 multiply-adds per instruction
// per lane instead of 1, and one 16-byte LDS read of A per 4 k values.
//
// Each wavefront walks L consecutive faces of one chain (the vertical faces of
// an element row, or the horizontal faces of an element column).  Consecutive
// faces of a chain share an element, so 4 of the 7 gathered rows of the next
// face are already in registers (the next face itself, the shared element's
// other faces, and the current face): each step loads only the 3 rows of the
// new element, 3P values per column instead of 7P.  A workgroup takes 4
// neighbouring chains (one per wavefront) over the same L positions, and stages
// their 4 L blocks in LDS (rows x k, zero padded) with coalesced slab reads.
// Summation over k is sequential within each parity of k; the even and odd
// partial sums are added at the end.
typedef float v4f __attribute__((ext_vector_type(4)));

template <int P>
struct WalkShape {
  static constexpr int NRG = (P + 3) / 4;       // groups of 4 output rows
  static constexpr int K = 7 * P;               // gathered rows per face
  static constexpr int KP = (K + 3) / 4 * 4;    // k padded to whole 16-byte LDS reads
#ifdef HDG_WALK_L
  static constexpr int L = HDG_WALK_L;
#else
  static constexpr int L = P <= 4 ? 16 : 8;     // faces per wavefront along its chain
#endif
  static_assert(L % 4 == 0, "a region holds L/4 tiles of each face type");
};

// Workgroups of a walk launch.  The mesh is cut into regions of L x L elements;
// a region holds L/4 vertical tiles (4 element rows, L faces along each) and L/4
// horizontal tiles (4 element columns, L faces along each), L/2 workgroups that
// read overlapping rows of X.
template <int P>
__host__ __device__ inline int64_t walk_blocks(int n) {
  constexpr int L = WalkShape<P>::L;
  const int64_t nr = (n + L - 1) / L;
  return nr * nr * (L / 2);
}

template <int P, int MODE, typename TM>
__global__ __launch_bounds__(256) void k_trace_multi_walk(MultiArgs a) {
  using L16 = Lanes16<TM, float>;
  using WS = WalkShape<P>;
  constexpr int V = L16::V, P2 = P * P, NE = 7 * P2, NQ = (NE + V - 1) / V;
  constexpr int NRG = WS::NRG, K = WS::K, KP = WS::KP, L = WS::L;
  __shared__ __align__(16) float blk[4][L][NRG * 4][KP];
  const int n = a.n, m = n - 1;
  const int64_t nv = (int64_t)n * m;
  // Workgroups are dealt round-robin to the 8 XCDs: XCD x takes the contiguous
  // run of regions [x R/8, (x+1) R/8) in row-major order, and a region's L/2
  // tiles run back to back on it, so the X rows they share meet in its L2.
  const int64_t total = walk_blocks<P>(n);
  const int64_t q = (total % 8 == 0) ? (int64_t)(blockIdx.x & 7) * (total >> 3) + (blockIdx.x >> 3)
                                     : (int64_t)blockIdx.x;
  const int nr = (n + L - 1) / L;
  const int64_t region = q / (L / 2);
  const int tr = (int)(q - region * (L / 2));
  const int rr = (int)(region / nr), rc = (int)(region - (int64_t)rr * nr);
  const bool vert = tr < L / 4;
  // chain group (4 chains) and the first position along them
  const int cg = vert ? rr * (L / 4) + tr : rc * (L / 4) + (tr - L / 4);
  const int pos0 = vert ? rc * L : rr * L;
  if (pos0 >= m || 4 * cg >= n) return;  // uniform over the workgroup, before any barrier
  // face at chain c, position pos (0 .. m-1)
  auto face_at = [&](int c, int pos) -> int64_t {
    return vert ? (int64_t)pos + (int64_t)m * c : nv + c + (int64_t)n * pos;
  };
  float* bl = &blk[0][0][0][0];
  for (int i = threadIdx.x; i < 4 * L * NRG * 4 * KP; i += blockDim.x) bl[i] = 0.f;
  __syncthreads();
  const u32x4* sp = static_cast<const u32x4*>(a.slab);
  // consecutive threads read consecutive faces: along the chain for vertical
  // faces (consecutive face numbers), across the 4 chains for horizontal ones
  for (int i = threadIdx.x; i < 4 * L * NQ; i += blockDim.x) {
    int w, t, q;
    if (vert) {
      t = i % L;
      q = (i / L) % NQ;
      w = i / (L * NQ);
    } else {
      w = i & 3;
      q = (i >> 2) % NQ;
      t = (i >> 2) / NQ;
    }
    const int c = 4 * cg + w, pos = pos0 + t;
    if (c >= n || pos >= m) continue;
    const int64_t f = face_at(c, pos);
    float wv[V];
    L16::unpack(__builtin_nontemporal_load(sp + ((f >> 6) * NQ + q) * 64 + (f & 63)), wv);
#pragma unroll
    for (int u = 0; u < V; ++u) {
      const int e = q * V + u;  // slot sl, row r, column cc  ->  blk[w][t][r][sl P + cc]
      if (e < NE) {
        const int sl = e / P2, rc = e - sl * P2, r = rc / P, cc = rc - r * P;
        blk[w][t][r][sl * P + cc] = wv[u];
      }
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, j = lane & 3;
  const int c = 4 * cg + wave;
  if (c >= n) return;  // uniform over the wavefront; no barrier follows
  const int steps = min(L, m - pos0);
  float* Y = static_cast<float*>(a.Y);
  const float* B = static_cast<const float*>(a.B);
  const int R = a.nrhs;
  // X by buffer loads: one 32-bit lane offset per gathered row, the column
  // offset c R of the row as a wave-uniform offset (the launcher keeps X below
  // 2 GiB)
  const __amdgpu_buffer_rsrc_t xr = buffer_rsrc(a.X, (int)((int64_t)a.nf * P * R * 4));
  for (int r0 = 0; r0 < R; r0 += 64) {
    const int col = r0 + lane;
    const bool cok = col < R;
    const int cl = cok ? col : R - 1;
    // a missing (boundary) neighbour reads the face's own row, zeroed
    auto load_row = [&](int64_t gs, int64_t fself, float* dst) __attribute__((always_inline)) {
      const bool ok = gs >= 0 && cok;
      const int xo = (int)(((gs >= 0 ? gs : fself) * P * R + cl) * 4);
#pragma unroll
      for (int cc = 0; cc < P; ++cc) {
        const float v = buffer_load<float>(xr, xo, cc * R * 4);
        dst[cc] = ok ? v : 0.f;
      }
    };
    float xw[7][P];
    {
      const int64_t f = face_at(c, pos0);
      int64_t g[7];
      face_neighbours(n, nv, f, g);
#pragma unroll
      for (int sl = 0; sl < 7; ++sl) load_row(g[sl], f, xw[sl]);
    }
    for (int t = 0; t < steps; ++t) {
      const int64_t f = face_at(c, pos0 + t);
      // the next face's 3 new rows (the other faces of its new element), in flight
      // while this face is computed
      float nx[3][P];
      const bool more = t + 1 < steps;
      if (more) {
        // the other faces of the next face's hi element (slots 4-6), or -1
        const int pn = pos0 + t + 1;
        const int64_t fn = face_at(c, pn);
        int64_t g4, g5, g6;
        if (vert) {  // row c, hi element (pn + 1, c): right, bottom, top
          g4 = pn <= m - 2 ? fn + 1 : -1;
          g5 = c >= 1 ? nv + (pn + 1) + (int64_t)n * (c - 1) : -1;
          g6 = c <= n - 2 ? nv + (pn + 1) + (int64_t)n * c : -1;
        } else {     // column c, hi element (c, pn + 1): left, right, top
          g4 = c >= 1 ? (int64_t)(c - 1) + (int64_t)m * (pn + 1) : -1;
          g5 = c <= n - 2 ? (int64_t)c + (int64_t)m * (pn + 1) : -1;
          g6 = pn <= m - 2 ? fn + n : -1;
        }
        load_row(g4, fn, nx[0]);
        load_row(g5, fn, nx[1]);
        load_row(g6, fn, nx[2]);
      }
      v4f acc[2][NRG];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int rg = 0; rg < NRG; ++rg) acc[h][rg] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kq = 0; kq < KP / 4; ++kq) {
        v4f av[NRG];
#pragma unroll
        for (int rg = 0; rg < NRG; ++rg) av[rg] = *reinterpret_cast<const v4f*>(&blk[wave][t][4 * rg + j][4 * kq]);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = 4 * kq + u;
          if (k < K) {  // resolved at compile time
            const float xv = xw[k / P][k % P];
#pragma unroll
            for (int rg = 0; rg < NRG; ++rg)
              acc[u & 1][rg] = __builtin_amdgcn_mfma_f32_4x4x1f32(av[rg][u], xv, acc[u & 1][rg], 0, 0, 0);
          }
        }
      }
      if (cok) {
        float res[NRG * 4];
#pragma unroll
        for (int rg = 0; rg < NRG; ++rg) {
          const v4f sacc = acc[0][rg] + acc[1][rg];
#pragma unroll
          for (int i = 0; i < 4; ++i) res[4 * rg + i] = sacc[i];
        }
        if constexpr (MODE == TM_APPLY) {
#pragma unroll
          for (int q = 0; q < P; ++q) Y[(f * P + q) * R + col] = res[q];
        } else {
#pragma unroll
          for (int q = 0; q < P; ++q) res[q] = B[(f * P + q) * R + col] - res[q];
          if constexpr (MODE == TM_RESID) {
#pragma unroll
            for (int q = 0; q < P; ++q) Y[(f * P + q) * R + col] = res[q];
          } else if constexpr (P >= 2) {  // TM_RESID_RESTRICT
            const float* pm = static_cast<const float*>(a.pmat);
#pragma unroll
            for (int cc = 0; cc < P - 1; ++cc) {
              float sacc = 0.f;
#pragma unroll
              for (int q = 0; q < P; ++q) sacc += pm[q * (P - 1) + cc] * res[q];
              Y[(f * (P - 1) + cc) * R + col] = sacc;
            }
          }
        }
      }
      if (more) {
        // slot order (face_neighbours): 0 self, 1-3 the lo element's other faces,
        // 4-6 the hi element's; the next face's lo element is this face's hi one
        float o[7][P];
#pragma unroll
        for (int sl = 0; sl < 7; ++sl)
#pragma unroll
          for (int cc = 0; cc < P; ++cc) o[sl][cc] = xw[sl][cc];
        // vertical (lo: L B T, hi: R B T): self' = R, L' = self, B' T' = hi's B T
        // horizontal (lo: L R B, hi: L R T): self' = T, L' R' = hi's L R, B' = self
#pragma unroll
        for (int cc = 0; cc < P; ++cc) {
          xw[0][cc] = vert ? o[4][cc] : o[6][cc];
          xw[1][cc] = vert ? o[0][cc] : o[4][cc];
          xw[2][cc] = o[5][cc];
          xw[3][cc] = vert ? o[6][cc] : o[0][cc];
#pragma unroll
          for (int u = 0; u < 3; ++u) xw[4 + u][cc] = nx[u][cc];
        }
      }
    }
  }
}

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

// right-hand sides from which the FP32 / bfloat16 product runs on the matrix cores
template <int P, int MODE>
static hipError_t launch_trace_multi_pm(Prec pr, const MultiArgs& a, hipStream_t s) {
  if (pr != Prec::F64 && a.kernel == 1 && a.nf * P * (int64_t)a.nrhs * 4 < ((int64_t)1 << 31)) {
    const dim3 grid((unsigned)walk_blocks<P>(a.n)), block(256);
    if (pr == Prec::F32) hipLaunchKernelGGL((k_trace_multi_walk<P, MODE, float>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_trace_multi_walk<P, MODE, bf16_t>), grid, block, 0, s, a);
    return hipGetLastError();
  }
  constexpr int FW = MultiGroup<P, double>::FW;
  const dim3 grid((unsigned)((a.nf + FW - 1) / FW));
  const int64_t pairs = (int64_t)FW * a.nrhs;
  const dim3 block((unsigned)(pairs >= 256 ? 256 : (pairs + 63) / 64 * 64));
  switch (pr) {
    case Prec::F64: hipLaunchKernelGGL((k_trace_multi<P, MODE, double, double>), grid, block, 0, s, a); break;
    case Prec::F32: hipLaunchKernelGGL((k_trace_multi<P, MODE, float, float>), grid, block, 0, s, a); break;
    case Prec::BF16: hipLaunchKernelGGL((k_trace_multi<P, MODE, bf16_t, float>), grid, block, 0, s, a); break;
  }
  return hipGetLastError();
}

template <int P>
static hipError_t launch_trace_multi_p(Prec pr, int mode, const MultiArgs& a, hipStream_t s) {
  switch (mode) {
    case TM_APPLY: return launch_trace_multi_pm<P, TM_APPLY>(pr, a, s);
    case TM_RESID: return launch_trace_multi_pm<P, TM_RESID>(pr, a, s);
    case TM_RESID_RESTRICT:
      if (P < 2) return hipErrorInvalidValue;
      return launch_trace_multi_pm<P, TM_RESID_RESTRICT>(pr, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_trace_multi(Prec pr, int P, const MultiArgs& a, hipStream_t s, int mode) {
  if (a.nrhs < 1) return hipErrorInvalidValue;
  if (a.nf == 0) return hipSuccess;
  HDG_DISPATCH_P(P, return launch_trace_multi_p<PP>(pr, mode, a, s));
}

hipError_t launch_trace(Prec pr, int P, int mode, const TraceArgs& a, hipStream_t s) {
  HDG_DISPATCH_P(P, return launch_trace_p<PP>(pr, mode, a, s));
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------ face-local ops
static inline dim3 grid_for(int64_t n) { return dim3((unsigned)((n + kWG - 1) / kWG)); }

template <int P, typename TM, typename TV>
__global__ __launch_bounds__(kWG) void k_dinv_apply(const void* dinv, const TV* b, double omega, TV* x,
                                                    int64_t nf) {
  using L16 = Lanes16<TM, TV>;
  constexpr int V = L16::V, P2 = P * P, NQD = (P2 + V - 1) / V;
  const int64_t f = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (f >= nf) return;
  const int64_t tile = f >> 6;
  const int lane = (int)(f & 63);
  TV r[P], z[P];
#pragma unroll
  for (int c = 0; c < P; ++c) { r[c] = b[f * P + c]; z[c] = TV(0); }
  const u32x4* dp = static_cast<const u32x4*>(dinv) + (tile * NQD) * 64 + lane;
#pragma unroll
  for (int q = 0; q < NQD; ++q) {
    TV w[V];
    L16::unpack(dp[q * 64], w);
#pragma unroll
    for (int u = 0; u < V; ++u) {
      const int e = q * V + u;
      if (e < P2) z[e / P] += w[u] * r[e % P];
    }
  }
#pragma unroll
  for (int c = 0; c < P; ++c) x[f * P + c] = TV(omega) * z[c];
}

template <int P, typename T>
__global__ __launch_bounds__(kWG) void k_p_restrict(const T* pm, const T* rf, T* rc, int64_t nf) {
  const int64_t f = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (f >= nf) return;
  T r[P];
#pragma unroll
  for (int a = 0; a < P; ++a) r[a] = rf[f * P + a];
#pragma unroll
  for (int c = 0; c < P - 1; ++c) {
    T s = T(0);
#pragma unroll
    for (int a = 0; a < P; ++a) s += pm[a * (P - 1) + c] * r[a];
    rc[f * (P - 1) + c] = s;
  }
}

template <int P, typename T>
__global__ __launch_bounds__(kWG) void k_p_prolong_add(const T* pm, const T* ec, T* xf, int64_t nf) {
  const int64_t f = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (f >= nf) return;
  T e[P - 1];
#pragma unroll
  for (int c = 0; c < P - 1; ++c) e[c] = ec[f * (P - 1) + c];
#pragma unroll
  for (int a = 0; a < P; ++a) {
    T s = xf[f * P + a];
#pragma unroll
    for (int c = 0; c < P - 1; ++c) s += pm[a * (P - 1) + c] * e[c];
    xf[f * P + a] = s;
  }
}

hipError_t launch_dinv_apply(Prec pr, int P, const void* dinv, const void* b, double omega, void* x,
                             int64_t nf, hipStream_t s) {
  if (nf == 0) return hipSuccess;
  switch (pr) {
    case Prec::F64:
      HDG_DISPATCH_P(P, hipLaunchKernelGGL((k_dinv_apply<PP, double, double>), grid_for(nf), dim3(kWG), 0, s,
                                           dinv, (const double*)b, omega, (double*)x, nf));
      break;
    case Prec::F32:
      HDG_DISPATCH_P(P, hipLaunchKernelGGL((k_dinv_apply<PP, float, float>), grid_for(nf), dim3(kWG), 0, s,
                                           dinv, (const float*)b, omega, (float*)x, nf));
      break;
    case Prec::BF16:
      HDG_DISPATCH_P(P, hipLaunchKernelGGL((k_dinv_apply<PP, bf16_t, float>), grid_for(nf), dim3(kWG), 0, s,
                                           dinv, (const float*)b, omega, (float*)x, nf));
      break;
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t p_restrict_t(int P, const void* pm, const void* rf, void* rc, int64_t nf, hipStream_t s) {
  HDG_DISPATCH_P(P, if constexpr (PP >= 2) hipLaunchKernelGGL((k_p_restrict<PP, T>), grid_for(nf), dim3(kWG), 0,
                                                               s, (const T*)pm, (const T*)rf, (T*)rc, nf));
  return hipGetLastError();
}
template <typename T>
static hipError_t p_prolong_t(int P, const void* pm, const void* ec, void* xf, int64_t nf, hipStream_t s) {
  HDG_DISPATCH_P(P, if constexpr (PP >= 2) hipLaunchKernelGGL((k_p_prolong_add<PP, T>), grid_for(nf),
                                                               dim3(kWG), 0, s, (const T*)pm, (const T*)ec,
                                                               (T*)xf, nf));
  return hipGetLastError();
}

hipError_t launch_p_restrict(Prec pr, int P, const void* pm, const void* rf, void* rc, int64_t nf,
                             hipStream_t s) {
  if (P < 2) return hipErrorInvalidValue;
  if (nf == 0) return hipSuccess;
  return pr == Prec::F64 ? p_restrict_t<double>(P, pm, rf, rc, nf, s) : p_restrict_t<float>(P, pm, rf, rc, nf, s);
}

hipError_t launch_p_prolong_add(Prec pr, int P, const void* pm, const void* ec, void* xf, int64_t nf,
                                hipStream_t s) {
  if (P < 2) return hipErrorInvalidValue;
  if (nf == 0) return hipSuccess;
  return pr == Prec::F64 ? p_prolong_t<double>(P, pm, ec, xf, nf, s) : p_prolong_t<float>(P, pm, ec, xf, nf, s);
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
// with W = Dinv A, Z = Dinv C.  Every reduced matrix is symmetric, so the
// even positions' multipliers need no storage of their own: M-_j = Z_{j-1}^T
// and M+_j = W_{j+1}^T.  Work item = (position, row): it streams one row of
// its blocks (a column of W or Z for the forward reduction).  Factors of a
// level of size ml: the odd records [Dinv, W, Z] as 3 P^2 arrays over the
// no = floor(ml/2) odd positions (entry-major, so a wavefront reads
// consecutive addresses); the last level stores Dinv of its single block.
// The right-hand side in LDS is ordered by level too: a position whose odd
// index at level l is o (position (2o+1) 2^l) sits in level l's array
// [row][o] of floor(ml_l/2) columns, at word P (m - ml_l) + o + row floor(ml_l/2)
// (the arrays of the levels before l hold m - ml_l positions); position 0
// takes the last P words.  Every phase then reads and writes its operands at
// unit stride across a wavefront, where the position-major order had lanes
// 2^(l+1) P words apart and serialised the LDS banks.
// The reduction has 2 log2(n) dependent phases, one barrier each (a level of
// the back substitution writes only its own odd positions, which no other
// thread reads in that phase).  Work item = (position, block of RB rows): a
// thread loads the item's factor rows once, reads the position's neighbours
// from LDS once and updates RB rows, so the index arithmetic of an item is
// shared by its P RB multiply-adds.  The factors of the small levels
// l >= a.lds_level are copied to LDS together with the right-hand side, so only
// the first lds_level levels of each sweep wait on HBM; there a thread issues
// the loads of a batch of KB positions before using any of them, and loads the
// next batch (or the next level's first) once the current one is used, before
// the barrier.  Level 0's first batch is requested before the staging copies,
// the backward sweep's first HBM batch before the top solve (few registers) or
// at the end of the last staged level.  A second kernel, k_chain_flat, requests
// every factor of a sweep at once where the registers allow it.
// The multiply-adds of the chain solve, written out as fused operations in a
// fixed order: every launch schedule then rounds alike, so their results are
// bit-identical (left to itself the compiler may contract a*b + c*d either way).
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
// forward: v - (z l + w r)
template <typename T>
__device__ __forceinline__ T chain_fwd_step(T v, T z, T l, T w, T r) {
  return fma_t(-w, r, fma_t(-z, l, v));
}
// backward: s + d o - w l - z r
template <typename T>
__device__ __forceinline__ T chain_bwd_step(T s, T d, T o, T w, T l, T z, T r) {
  return fma_t(-z, r, fma_t(-w, l, fma_t(d, o, s)));
}

template <int P, bool WIDE>
struct ChainShape {
  // Rows per item (RBF forward, RBB backward) and positions whose loads are in
  // flight together (KBF, KBB): a batch holds KBF RBF 2P forward or KBB RBB 3P
  // backward factor entries.  The lean shape keeps a thread within 128
  // registers (4 waves per SIMD, for meshes with many chains per CU); the wide
  // shape (P = 3 ... 5) loads every row of a position in one batch, so a level
  // whose positions fit the workgroup costs one load round trip, at up to 256
  // registers (for meshes with few chains per CU).
  static constexpr bool W = WIDE && P >= 3 && P <= 5;
  static constexpr int RBF = W ? P : (P <= 4 ? P : (P <= 5 ? 3 : (P <= 8 ? 2 : 1)));
  static constexpr int RBB = W ? P : (P <= 2 ? P : (P <= 4 ? 2 : 1));
  static constexpr int NRBF = (P + RBF - 1) / RBF;
  static constexpr int NRBB = (P + RBB - 1) / RBB;
  static constexpr int KBF = P <= 1 ? 8 : (P <= 2 ? 2 : 1);
  static constexpr int KBB = P <= 1 ? 4 : (P <= 2 ? 2 : 1);
  // the first backward batch is requested before the top solve when its
  // registers are few, else at the end of the last level staged in LDS
  static constexpr bool EARLYB = 3 * KBB * RBB * P + 3 * P * P <= 40;
  static constexpr int MAXT = W ? 512 : (P <= 4 ? 1024 : 512);  // workgroup size bound (registers)
};

template <int P, typename T, bool WIDE>
__global__ __launch_bounds__((ChainShape<P, WIDE>::MAXT)) void k_chain(ChainArgs a) {
  constexpr int P2 = P * P;
  using CS = ChainShape<P, WIDE>;
  extern __shared__ unsigned char lds_raw[];
  T* R = reinterpret_cast<T*>(lds_raw);
  const T* rin = static_cast<const T*>(a.r);
  const T* xin = static_cast<const T*>(a.x);
  T* out = static_cast<T*>(a.out);
  // Neighbouring horizontal chains read neighbouring faces: the values of one
  // position of 8 consecutive chains share cache lines.  Workgroups are dealt
  // round-robin to the 8 XCDs, so chain c is given to workgroup
  // (c mod (2n/8)) * 8 + c / (2n/8): consecutive chains then run on the same
  // XCD at about the same time and share its L2.
  const int64_t nch = 2LL * a.n;
  const int64_t c = (a.remap && nch % 8 == 0) ? (int64_t)(blockIdx.x & 7) * (nch >> 3) + (blockIdx.x >> 3)
                                                : (int64_t)blockIdx.x;
  const int m = a.n - 1;
  const int64_t nv = (int64_t)a.n * (a.n - 1);
  const bool vert = c < a.n;
  const int64_t base = vert ? c * (a.n - 1) : nv + (c - a.n);
  const int64_t stride = vert ? 1 : a.n;
  const T* F = static_cast<const T*>(a.factors) + c * a.cstride;
  const int t = threadIdx.x;
  const int nt = blockDim.x;
  // LDS word of row 0 of position pos of level l, and the row stride
  auto slot = [m](int l, int pos, int& rs) -> int {
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
  auto level_offset = [&](int l) {
    int64_t lo = 0;
    for (int q = 0, s = m; q < l; ++q, s = (s + 1) >> 1)
      lo += (int64_t)3 * P2 * (s >> 1);
    return lo;
  };
  int Lf = 0;  // index of the last level (a single block)
  for (int s = m; s > 1; s = (s + 1) >> 1) ++Lf;
  const int Ls = a.lds_level < Lf ? a.lds_level : Lf;  // the last level is always staged
  const int64_t tail_off = level_offset(Ls);
  T* TL = R + m * P;  // LDS copy of the factors of levels >= Ls
  // Factors of level l come from HBM (l < Ls: loaded in register batches, the
  // first batch of a level before the barrier that ends the previous one) or
  // from LDS (l >= Ls: read where they are used).  The two never share a
  // pointer, so the compiler emits global or LDS loads rather than flat ones.
  // ---- forward reduction.  Rows r of M-_j and M+_j (j = 2 tt): column r of Z
  // at odd index tt - 1 and of W at odd index tt.
  constexpr int KB = CS::KBF, RB = CS::RBF, NRB = CS::NRBF;
  T zm[KB][RB][P], wp[KB][RB][P];
  // Loads are unconditional, at indices clamped into the level's arrays (whose
  // entries are all finite), and the operand they multiply is masked where the
  // product is used: a load under a branch makes the compiler wait for it before
  // the branch joins, and so does a select on the loaded value placed next to
  // the load, which would turn every prefetch into a synchronous load.
  constexpr int S = (int)sizeof(T);
  // HBM factors by buffer loads: one register offset per lane, a wave-uniform
  // byte offset per entry
  const __amdgpu_buffer_rsrc_t fr = buffer_rsrc(F, (int)(a.cstride * S));
  // an empty range: loads through it return 0 and touch no memory, so a
  // pipelined load with nothing left to fetch needs no branch around it
  const __amdgpu_buffer_rsrc_t fr0 = buffer_rsrc(F, 0);
  auto load_fwd = [&](__amdgpu_buffer_rsrc_t rs, int64_t off_l, int ml_, int rb, int c0) __attribute__((always_inline)) {
    const int ne_ = (ml_ + 1) >> 1, no_ = ml_ >> 1;  // no_ >= 1
    const int o8 = (int)off_l * S;
#pragma unroll
    for (int kk = 0; kk < KB; ++kk) {
      const int tt = c0 + kk * nt;
      const unsigned zi = (unsigned)min(max(tt - 1, 0), no_ - 1), wi = (unsigned)min(tt, no_ - 1);
#pragma unroll
      for (int rr = 0; rr < RB; ++rr) {
        const int r = rb * RB + rr;
#pragma unroll
        for (int q = 0; q < P; ++q) {
          if (r < P) {  // resolved at compile time; the missing neighbours' values are masked in fwd_compute
            zm[kk][rr][q] = buffer_load<T>(rs, (int)zi * S, o8 + (2 * P2 + q * P + r) * no_ * S);
            wp[kk][rr][q] = buffer_load<T>(rs, (int)wi * S, o8 + (P2 + q * P + r) * no_ * S);
          } else {
            zm[kk][rr][q] = wp[kk][rr][q] = T(0);
          }
        }
      }
    }
  };
  auto fwd_compute = [&](int ml_, int lev_, int rb, int c0) __attribute__((always_inline)) {
    const int ne_ = (ml_ + 1) >> 1, no_ = ml_ >> 1;
    const int ob = P * (m - ml_);  // level lev_'s odd positions: [row][o]
#pragma unroll
    for (int kk = 0; kk < KB; ++kk) {
      const int tt = c0 + kk * nt;
      if (tt < ne_) {
        T lv[P], rv[P];
        const int li = max(tt - 1, 0), ri = min(tt, no_ - 1);
#pragma unroll
        for (int q = 0; q < P; ++q) {
          const T x = R[ob + q * no_ + li], y = R[ob + q * no_ + ri];
          lv[q] = tt >= 1 ? x : T(0);
          rv[q] = tt < no_ ? y : T(0);
        }
        int rs;
        const int w = slot(lev_ + 1, tt, rs);
#pragma unroll
        for (int rr = 0; rr < RB; ++rr) {
          const int r = rb * RB + rr;
          if (r < P) {
            T v = R[w + r * rs];
#pragma unroll
            for (int q = 0; q < P; ++q) v = chain_fwd_step(v, zm[kk][rr][q], lv[q], wp[kk][rr][q], rv[q]);
            R[w + r * rs] = v;
          }
        }
      }
    }
  };
  int ml = m, lev = 0;
  int64_t off = 0;
  // forward level with factors in LDS: one position (all rows) per item
  auto fwd_level_lds = [&](const T* O) __attribute__((always_inline)) {
    const int ne_ = (ml + 1) >> 1, no_ = ml >> 1;
    const int ob = P * (m - ml);
    for (int tt = t; tt < ne_; tt += nt) {
      T lv[P], rv[P];
      const int li = max(tt - 1, 0), ri = min(tt, no_ - 1);
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const T x = R[ob + q * no_ + li], y = R[ob + q * no_ + ri];
        lv[q] = tt >= 1 ? x : T(0);  // a missing neighbour contributes 0 times a finite factor
        rv[q] = tt < no_ ? y : T(0);
      }
      int rs;
      const int w = slot(lev + 1, tt, rs);
#pragma unroll
      for (int r = 0; r < P; ++r) {
        T v = R[w + r * rs];
#pragma unroll
        for (int q = 0; q < P; ++q)
          v = chain_fwd_step(v, O[(2 * P2 + q * P + r) * no_ + li], lv[q], O[(P2 + q * P + r) * no_ + ri], rv[q]);
        R[w + r * rs] = v;
      }
    }
  };
  // The first batch of level 0's factors and this thread's first values of x
  // (read again only by the final update) are requested before the staging
  // copies, so their latency overlaps the staging's.
  if (ml > 1 && Ls > 0) load_fwd(fr, 0, ml, 0, t);
  constexpr int CBP = P >= 8 ? 1 : 8 / P;
  constexpr bool XPRE = P <= 1;  // registers held across the whole kernel
  T xpre[CBP][P];
#pragma unroll
  for (int u = 0; u < CBP; ++u)
#pragma unroll
    for (int r = 0; r < P; ++r) xpre[u][r] = T(0);
  if (XPRE && xin) {
#pragma unroll
    for (int u = 0; u < CBP; ++u) {
      const int i = t + u * nt;
#pragma unroll
      for (int r = 0; r < P; ++r) xpre[u][r] = xin[(base + stride * min(i, m - 1)) * P + r];  // used for i < m only
    }
  }
  // copies to LDS keep about 8 loads per thread in flight (a load-store loop
  // would wait for every load before the next one is issued)
  for (int i0 = t; i0 < m; i0 += nt * CBP) {
    T v[CBP][P];
#pragma unroll
    for (int u = 0; u < CBP; ++u) {
      const int i = i0 + u * nt;
      if (i < m) {
        const T* src = rin + (base + stride * i) * P;
#pragma unroll
        for (int r = 0; r < P; ++r) v[u][r] = src[r];
      }
    }
#pragma unroll
    for (int u = 0; u < CBP; ++u) {
      const int i = i0 + u * nt;
      if (i < m) {
        int rs;
        const int w = slot(0, i, rs);
#pragma unroll
        for (int r = 0; r < P; ++r) R[w + r * rs] = v[u][r];
      }
    }
  }
  constexpr int CB = 8;
  const int64_t tail_len = a.cstride - tail_off;
  for (int64_t b0 = t; b0 < tail_len; b0 += (int64_t)nt * CB) {
    T v[CB];
#pragma unroll
    for (int u = 0; u < CB; ++u)
      if (b0 + u * nt < tail_len) v[u] = F[tail_off + b0 + u * nt];
#pragma unroll
    for (int u = 0; u < CB; ++u)
      if (b0 + u * nt < tail_len) TL[b0 + u * nt] = v[u];
  }
  lds_barrier();
  // levels in HBM, then levels in LDS
  // Software pipeline: a batch's registers hold its factors on entry; once used
  // they receive the next batch of the level, or after the level the first
  // batch of the next one.  The batch loop runs the same number of times in
  // every lane (items past the level are masked), so the loads sit under
  // uniform branches only, and the scheduling barriers keep them after the
  // use: the registers are reused rather than doubled.
  while (ml > 1 && lev < Ls) {
    const int ne = (ml + 1) >> 1;
    const int64_t off_next = off + (int64_t)3 * P2 * (ml >> 1);
    for (int cb = 0; cb < ne; cb += nt * KB) {
      const int c0 = cb + t;
#pragma unroll
      for (int rb = 0; rb < NRB; ++rb) {
        if (rb > 0) {
          __builtin_amdgcn_sched_barrier(0);
          load_fwd(fr, off, ml, rb, c0);
        }
        fwd_compute(ml, lev, rb, c0);
      }
      // the next batch of this level, else the first of the next level in HBM
      const bool more = cb + nt * KB < ne, next = ne > 1 && lev + 1 < Ls;
      __builtin_amdgcn_sched_barrier(0);
      load_fwd(more || next ? fr : fr0, more ? off : off_next, more ? ml : max(ne, 2), 0, more ? c0 + nt * KB : t);
    }
    off = off_next;
    ml = ne;
    ++lev;
    lds_barrier();
  }
  while (ml > 1) {
    fwd_level_lds(TL + (off - tail_off));
    off += (int64_t)3 * P2 * (ml >> 1);
    ml = (ml + 1) >> 1;
    ++lev;
    lds_barrier();
  }
  // ---- back substitution.  Level l writes the solution of its odd positions,
  // which no other thread reads in that phase (their neighbours are even
  // positions, solved at deeper levels), so a thread computes all rows of its
  // positions, writes them, and one barrier ends the level.
  constexpr int KBB = CS::KBB, RBB = CS::RBB, NRBB = CS::NRBB;
  T od[KBB][RBB][P], ow[KBB][RBB][P], oz[KBB][RBB][P];
  auto load_bwd_from = [&](__amdgpu_buffer_rsrc_t rs, int64_t lo, int mlv, int rb, int c0) __attribute__((always_inline)) {
    (void)mlv;
    const int no_ = mlv >> 1;
    const int o8 = (int)lo * S;
#pragma unroll
    for (int kk = 0; kk < KBB; ++kk) {
      const int tt = c0 + kk * nt;
      const unsigned ti = (unsigned)min(tt, no_ - 1);
#pragma unroll
      for (int rr = 0; rr < RBB; ++rr) {
        const int r = rb * RBB + rr;
#pragma unroll
        for (int q = 0; q < P; ++q) {
          if (r < P) {  // resolved at compile time; a missing right neighbour's value is masked at use
            od[kk][rr][q] = buffer_load<T>(rs, (int)ti * S, o8 + (r * P + q) * no_ * S);
            ow[kk][rr][q] = buffer_load<T>(rs, (int)ti * S, o8 + (P2 + r * P + q) * no_ * S);
            oz[kk][rr][q] = buffer_load<T>(rs, (int)ti * S, o8 + (2 * P2 + r * P + q) * no_ * S);
          } else {
            od[kk][rr][q] = ow[kk][rr][q] = oz[kk][rr][q] = T(0);
          }
        }
      }
    }
  };
  auto load_bwd = [&](__amdgpu_buffer_rsrc_t rs, int l, int rb, int c0) __attribute__((always_inline)) {
    load_bwd_from(rs, level_offset(l), (m + (1 << l) - 1) >> l, rb, c0);
  };
  // The first batch of the first level whose factors are in HBM is requested
  // now (the top solve and the levels staged in LDS do not use these registers,
  // and hide the load's latency), or before the barrier of the last staged level.
  const bool staged_bwd = Lf - 1 >= Ls;
  if (CS::EARLYB && Ls > 0) load_bwd(fr, Ls - 1, 0, t);
  T xr = T(0);
  const int top = P * (m - 1);
  if (t < P) {  // the last level is always staged (Ls <= Lf = lev)
    const T* D = TL + (off - tail_off);
#pragma unroll
    for (int q = 0; q < P; ++q) xr = fma_t(D[t * P + q], R[top + q], xr);
  }
  lds_barrier();
  if (t < P) R[top + t] = xr;
  lds_barrier();
  // back substitution of a level with factors in LDS: one position per item
  auto bwd_level_lds = [&](const T* O, int no, int ob0, bool pre) __attribute__((always_inline)) {
    for (int tt = t; tt < no; tt += nt) {
      {
        T own[P], xl[P], xrt[P], res[P];
        int rl, rr2;
        const int wl = slot(lev + 1, tt, rl);
        const bool right = 2 * tt + 2 < ml;
        const int wr = right ? slot(lev + 1, tt + 1, rr2) : (rr2 = rl, wl);
#pragma unroll
        for (int q = 0; q < P; ++q) {
          own[q] = R[ob0 + tt + q * no];
          xl[q] = R[wl + q * rl];
          const T x = R[wr + q * rr2];
          xrt[q] = right ? x : T(0);  // Z is finite, so a missing neighbour contributes 0
        }
#pragma unroll
        for (int r = 0; r < P; ++r) {
          T s = T(0);
#pragma unroll
          for (int q = 0; q < P; ++q)
            s = chain_bwd_step(s, O[(r * P + q) * no + tt], own[q], O[(P2 + r * P + q) * no + tt], xl[q],
                               O[(2 * P2 + r * P + q) * no + tt], xrt[q]);
          res[r] = s;
        }
#pragma unroll
        for (int r = 0; r < P; ++r) R[ob0 + tt + r * no] = res[r];
      }
    }
    if (pre) {
      __builtin_amdgcn_sched_barrier(0);
      load_bwd(fr, Ls - 1, 0, t);
    }
    lds_barrier();
  };
  // levels in LDS, then levels in HBM.  The last staged level is peeled off,
  // so the prefetch it issues keeps its registers out of the other staged levels.
  while (lev > 0 && lev - 1 > Ls) {
    --lev;
    ml = (m + (1 << lev) - 1) >> lev;
    bwd_level_lds(TL + (level_offset(lev) - tail_off), ml >> 1, P * (m - ml), false);
  }
  if (lev > 0 && lev - 1 == Ls) {
    --lev;
    ml = (m + (1 << lev) - 1) >> lev;
    bwd_level_lds(TL + (level_offset(lev) - tail_off), ml >> 1, P * (m - ml), !CS::EARLYB && Ls > 0);
  }
  if (!CS::EARLYB && Ls > 0 && !staged_bwd) load_bwd(fr, Ls - 1, 0, t);  // no staged level to hide it
  while (lev > 0) {
    --lev;
    ml = (m + (1 << lev) - 1) >> lev;
    const int no = ml >> 1;
    const int ob0 = P * (m - ml);
    for (int cb = 0; cb < no; cb += nt * KBB) {
      const int c0 = cb + t;
      // a position's right-hand side and neighbours are read once, before any
      // of its rows is written
      T own[KBB][P], xl[KBB][P], xrt[KBB][P];
#pragma unroll
      for (int kk = 0; kk < KBB; ++kk) {
        const int tt = min(c0 + kk * nt, no - 1);
        int rl, rr2;
        const int wl = slot(lev + 1, tt, rl);
        const bool right = 2 * tt + 2 < ml;
        const int wr = right ? slot(lev + 1, tt + 1, rr2) : (rr2 = rl, wl);
#pragma unroll
        for (int q = 0; q < P; ++q) {
          own[kk][q] = R[ob0 + tt + q * no];
          xl[kk][q] = R[wl + q * rl];
          const T x = R[wr + q * rr2];
          xrt[kk][q] = right ? x : T(0);  // Z is finite, so a missing neighbour contributes 0
        }
      }
#pragma unroll
      for (int rb = 0; rb < NRBB; ++rb) {
        if (rb > 0) {
          __builtin_amdgcn_sched_barrier(0);
          load_bwd(fr, lev, rb, c0);
        }
#pragma unroll
        for (int kk = 0; kk < KBB; ++kk) {
          const int tt = c0 + kk * nt;
          if (tt < no) {
#pragma unroll
            for (int rr = 0; rr < RBB; ++rr) {
              const int r = rb * RBB + rr;
              if (r < P) {
                T s = T(0);
#pragma unroll
                for (int q = 0; q < P; ++q)
                  s = chain_bwd_step(s, od[kk][rr][q], own[kk][q], ow[kk][rr][q], xl[kk][q], oz[kk][rr][q], xrt[kk][q]);
                R[ob0 + tt + r * no] = s;
              }
            }
          }
        }
      }
      // as in the forward sweep: the next batch of this level, else the first of the next
      const bool more = cb + nt * KBB < no;
      __builtin_amdgcn_sched_barrier(0);
      load_bwd(more || lev > 0 ? fr : fr0, more ? lev : max(lev - 1, 0), 0, more ? c0 + nt * KBB : t);
    }
    lds_barrier();
  }
  for (int i0 = t; i0 < m; i0 += nt * CBP) {
    T v[CBP][P];
#pragma unroll
    for (int u = 0; u < CBP; ++u) {
      const int i = i0 + u * nt;
      if (i < m) {
#pragma unroll
        for (int r = 0; r < P; ++r) v[u][r] = XPRE && i0 == t ? xpre[u][r] : (xin ? xin[(base + stride * i) * P + r] : T(0));
      }
    }
#pragma unroll
    for (int u = 0; u < CBP; ++u) {
      const int i = i0 + u * nt;
      if (i < m) {
        int rs;
        const int w = slot(0, i, rs);
        T* dst = out + (base + stride * i) * P;
#pragma unroll
        for (int r = 0; r < P; ++r) dst[r] = v[u][r] + T(a.omega) * R[w + r * rs];
      }
    }
  }
}

// Chain solve with every factor load of a sweep requested at once (the flat
// schedule), for chains whose factors fit the workgroup's registers.  The items
// of all levels of a sweep are numbered consecutively (forward: the ne_l even
// positions of level l, level 0 first; backward: the no_l odd positions, the
// deepest level first, so the first slots' loads are the first ones waited
// for), and item g is held by thread g mod nt in slot g / nt (K slots).  Before
// a sweep a thread requests the factors of all its slots, so each sweep waits
// on memory about once instead of once per level; the levels then run from
// registers and the LDS copy of the right-hand side, one barrier each.  Each
// item computes exactly the expressions of k_chain, so the results are the
// same.  Registers: 2 K P^2 factor entries in the forward sweep, 3 K P^2 in the
// backward one.
template <int P, int K>
struct ChainFlat {
  static constexpr int MAXT = 3 * K * P * P <= 24 ? 1024 : 512;  // also chain_flat_maxt
};

template <int P, typename T, int K>
__global__ __launch_bounds__((ChainFlat<P, K>::MAXT)) void k_chain_flat(ChainArgs a) {
  constexpr int P2 = P * P;
  constexpr int S = (int)sizeof(T);
  extern __shared__ unsigned char lds_raw[];
  T* R = reinterpret_cast<T*>(lds_raw);
  const T* rin = static_cast<const T*>(a.r);
  const T* xin = static_cast<const T*>(a.x);
  T* out = static_cast<T*>(a.out);
  const int64_t nch = 2LL * a.n;  // chain order as in k_chain
  const int64_t c = (a.remap && nch % 8 == 0) ? (int64_t)(blockIdx.x & 7) * (nch >> 3) + (blockIdx.x >> 3)
                                                : (int64_t)blockIdx.x;
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
  auto level_size = [m](int l) { return (m + (1 << l) - 1) >> l; };
  int Lf = 0;
  for (int q = m; q > 1; q = (q + 1) >> 1) ++Lf;
  // The first chunk of the right-hand side is requested first, then the
  // factors (and, when registers allow, the backward sweep's factors and x),
  // so the chunk can be stored to LDS while the rest is in flight.
  constexpr int CBP = P >= 8 ? 1 : 8 / P;
  T v0[CBP][P];
#pragma unroll
  for (int u = 0; u < CBP; ++u) {
    const T* src = rin + (base + stride * min(t + u * nt, m - 1)) * P;
#pragma unroll
    for (int r = 0; r < P; ++r) v0[u][r] = src[r];
  }
  // ---- forward items: level and even index of each slot, and their factors
  int fl[K], ft[K];
  T zm[K][P][P], wp[K][P][P];
  {
    int ntot = 0;  // sum over levels of ne_l = m (m >= 1)
    for (int l = 0; l < Lf; ++l) ntot += (level_size(l) + 1) >> 1;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int g0 = t + k * nt;
      const int g = min(g0, max(ntot - 1, 0));  // past the last item: a copy of it, masked below
      int l = 0, acc = 0;
      int64_t lo = 0;
      while (l < Lf - 1 && g >= acc + ((level_size(l) + 1) >> 1)) {
        acc += (level_size(l) + 1) >> 1;
        lo += (int64_t)3 * P2 * (level_size(l) >> 1);
        ++l;
      }
      fl[k] = (g0 < ntot && Lf > 0) ? l : -1;
      ft[k] = g - acc;
      const int no_ = max(level_size(l) >> 1, 1);
      const int zi = min(max(ft[k] - 1, 0), no_ - 1), wi = min(ft[k], no_ - 1);
      const int zb = (int)lo + zi, wb = (int)lo + wi;
#pragma unroll
      for (int r = 0; r < P; ++r)
#pragma unroll
        for (int q = 0; q < P; ++q) {
          zm[k][r][q] = buffer_load<T>(fr, (zb + (2 * P2 + q * P + r) * no_) * S, 0);
          wp[k][r][q] = buffer_load<T>(fr, (wb + (P2 + q * P + r) * no_) * S, 0);
        }
    }
  }
  // the last level's single block, for the threads that solve it
  T dtop[P];
  {
    int64_t lo = 0;
    for (int l = 0; l < Lf; ++l) lo += (int64_t)3 * P2 * (level_size(l) >> 1);
    const int tr = min(t, P - 1);
#pragma unroll
    for (int q = 0; q < P; ++q) dtop[q] = buffer_load<T>(fr, ((int)lo + tr * P + q) * S, 0);
  }
  // ---- backward items (deepest level first) and their factors
  int bl[K], bt[K];
  T od[K][P][P], ow[K][P][P], oz[K][P][P];
  auto load_bwd_all = [&]() __attribute__((always_inline)) {
    int ntot = 0;
    for (int l = 0; l < Lf; ++l) ntot += level_size(l) >> 1;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int g0 = t + k * nt;
      const int g = min(g0, max(ntot - 1, 0));
      int l = Lf - 1, acc = 0;
      while (l > 0 && g >= acc + (level_size(l) >> 1)) {
        acc += level_size(l) >> 1;
        --l;
      }
      int64_t lo = 0;
      for (int q = 0; q < l; ++q) lo += (int64_t)3 * P2 * (level_size(q) >> 1);
      bl[k] = (g0 < ntot && Lf > 0) ? l : -1;
      bt[k] = g - acc;
      const int no_ = max(level_size(l) >> 1, 1);
      const int tb = (int)lo + min(bt[k], no_ - 1);
#pragma unroll
      for (int r = 0; r < P; ++r)
#pragma unroll
        for (int q = 0; q < P; ++q) {
          od[k][r][q] = buffer_load<T>(fr, (tb + (r * P + q) * no_) * S, 0);
          ow[k][r][q] = buffer_load<T>(fr, (tb + (P2 + r * P + q) * no_) * S, 0);
          oz[k][r][q] = buffer_load<T>(fr, (tb + (2 * P2 + r * P + q) * no_) * S, 0);
        }
    }
  };
  // with few factor entries per thread the backward sweep's are requested at
  // once too: the forward levels then run while they arrive
  constexpr bool EARLY = 5 * K * P * P <= 20;
  if constexpr (EARLY) load_bwd_all();
  // ---- the right-hand side into LDS, in k_chain's level order
#pragma unroll
  for (int u = 0; u < CBP; ++u) {
    const int i = t + u * nt;
    if (i < m) {
      int rs;
      const int w = slot(0, i, rs);
#pragma unroll
      for (int r = 0; r < P; ++r) R[w + r * rs] = v0[u][r];
    }
  }
  for (int i0 = t + nt * CBP; i0 < m; i0 += nt * CBP) {
    T v[CBP][P];
#pragma unroll
    for (int u = 0; u < CBP; ++u) {
      const int i = i0 + u * nt;
      if (i < m) {
        const T* src = rin + (base + stride * i) * P;
#pragma unroll
        for (int r = 0; r < P; ++r) v[u][r] = src[r];
      }
    }
#pragma unroll
    for (int u = 0; u < CBP; ++u) {
      const int i = i0 + u * nt;
      if (i < m) {
        int rs;
        const int w = slot(0, i, rs);
#pragma unroll
        for (int r = 0; r < P; ++r) R[w + r * rs] = v[u][r];
      }
    }
  }
  lds_barrier();
  // ---- forward reduction, level by level
  for (int l = 0; l < Lf; ++l) {
    const int ml = level_size(l);
    const int ne_ = (ml + 1) >> 1, no_ = ml >> 1;
    const int ob = P * (m - ml);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (fl[k] == l) {
        const int tt = ft[k];
        T lv[P], rv[P];
        const int li = max(tt - 1, 0), ri = min(tt, no_ - 1);
#pragma unroll
        for (int q = 0; q < P; ++q) {
          const T x = R[ob + q * no_ + li], y = R[ob + q * no_ + ri];
          lv[q] = tt >= 1 ? x : T(0);
          rv[q] = tt < no_ ? y : T(0);
        }
        int rs;
        const int w = slot(l + 1, tt, rs);
#pragma unroll
        for (int r = 0; r < P; ++r) {
          T v = R[w + r * rs];
#pragma unroll
          for (int q = 0; q < P; ++q) v = chain_fwd_step(v, zm[k][r][q], lv[q], wp[k][r][q], rv[q]);
          R[w + r * rs] = v;
        }
      }
    }
    (void)ne_;
    lds_barrier();
  }
  if constexpr (!EARLY) load_bwd_all();  // registers are free now; the top solve hides part of the wait
  T xr = T(0);
  const int top = P * (m - 1);
  if (t < P) {
#pragma unroll
    for (int q = 0; q < P; ++q) xr = fma_t(dtop[q], R[top + q], xr);
  }
  lds_barrier();
  if (t < P) R[top + t] = xr;
  lds_barrier();
  // ---- back substitution, level by level
  for (int l = Lf - 1; l >= 0; --l) {
    const int ml = level_size(l);
    const int no = ml >> 1;
    const int ob0 = P * (m - ml);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (bl[k] == l) {
        const int tt = bt[k];
        T own[P], xl[P], xrt[P];
        int rl, rr2;
        const int wl = slot(l + 1, tt, rl);
        const bool right = 2 * tt + 2 < ml;
        const int wr = right ? slot(l + 1, tt + 1, rr2) : (rr2 = rl, wl);
#pragma unroll
        for (int q = 0; q < P; ++q) {
          own[q] = R[ob0 + tt + q * no];
          xl[q] = R[wl + q * rl];
          const T x = R[wr + q * rr2];
          xrt[q] = right ? x : T(0);
        }
#pragma unroll
        for (int r = 0; r < P; ++r) {
          T s = T(0);
#pragma unroll
          for (int q = 0; q < P; ++q) s = chain_bwd_step(s, od[k][r][q], own[q], ow[k][r][q], xl[q], oz[k][r][q], xrt[q]);
          R[ob0 + tt + r * no] = s;
        }
      }
    }
    lds_barrier();
  }
  for (int i0 = t; i0 < m; i0 += nt * CBP) {
    T v[CBP][P];
#pragma unroll
    for (int u = 0; u < CBP; ++u) {
      const int i = i0 + u * nt;
      if (i < m) {
#pragma unroll
        for (int r = 0; r < P; ++r) v[u][r] = xin ? xin[(base + stride * i) * P + r] : T(0);
      }
    }
#pragma unroll
    for (int u = 0; u < CBP; ++u) {
      const int i = i0 + u * nt;
      if (i < m) {
        int rs;
        const int w = slot(0, i, rs);
        T* dst = out + (base + stride * i) * P;
#pragma unroll
        for (int r = 0; r < P; ++r) dst[r] = v[u][r] + T(a.omega) * R[w + r * rs];
      }
    }
  }
}

// Bytes of the factors of the levels >= l of one chain (element size es); the
// last level's record (one block) is always included, as the kernel stages it.
static int64_t chain_tail_bytes(int P, int n, int l, size_t es) {
  int64_t tot = 0;
  int q = 0;
  for (int s = n - 1;; s = (s + 1) >> 1, ++q) {
    const int64_t rec = s == 1 ? (int64_t)P * P : (int64_t)3 * P * P * (s >> 1);
    if (q >= l || s == 1) tot += rec;
    if (s == 1) break;
  }
  return tot * (int64_t)es;
}

int chain_lds_level(int P, int n, size_t es, int64_t budget) {
  if (budget < 0) budget = 0;
  int l = 0;
  while (l < 64 && chain_tail_bytes(P, n, l, es) > budget) ++l;
  return l;
}

size_t chain_lds_bytes(int P, int n, size_t es, int lds_level) {
  return (size_t)(n - 1) * P * es + (size_t)chain_tail_bytes(P, n, lds_level, es);
}

int chain_max_threads(int P, bool wide) {
  static constexpr int t[] = {0, ChainShape<1, false>::MAXT, ChainShape<2, false>::MAXT, ChainShape<3, false>::MAXT,
                              ChainShape<4, false>::MAXT, ChainShape<5, false>::MAXT, ChainShape<6, false>::MAXT,
                              ChainShape<7, false>::MAXT, ChainShape<8, false>::MAXT, ChainShape<9, false>::MAXT};
  static constexpr int w[] = {0, ChainShape<1, true>::MAXT, ChainShape<2, true>::MAXT, ChainShape<3, true>::MAXT,
                              ChainShape<4, true>::MAXT, ChainShape<5, true>::MAXT, ChainShape<6, true>::MAXT,
                              ChainShape<7, true>::MAXT, ChainShape<8, true>::MAXT, ChainShape<9, true>::MAXT};
  return P >= 1 && P <= 9 ? (wide ? w[P] : t[P]) : 0;
}

// Workgroup size: 128 threads for P <= 2 and 256 for larger P (more threads
// per chain lengthen every phase).
int chain_threads(int P, int n) {
  (void)n;
  return P <= 2 ? 128 : 256;
}

// XCD-aware chain order pays where the strided right-hand side of horizontal
// chains dominates (small P); measured neutral to slightly negative for P >= 4.
int chain_remap(int P) { return P <= 3 ? 1 : 0; }

// Slots per thread of the flat schedule's instances at P (0: none).
static int chain_flat_k(int P, int need) {
  static constexpr int ks[6][3] = {{0, 0, 0}, {4, 8, 16}, {2, 4, 0}, {1, 2, 0}, {1, 0, 0}, {1, 0, 0}};
  if (P < 1 || P > 5) return 0;
  for (int k : ks[P])
    if (k >= need) return k;
  return 0;
}

static int chain_flat_maxt(int P, int K) { return 3 * K * P * P <= 24 ? 1024 : 512; }  // ChainFlat<P, K>::MAXT

// Workgroup size of the flat schedule (0: none fits): the fewest slots per
// thread whose workgroup has at most 256 threads, else at most its launch bound.
int chain_flat_threads(int P, int n) {
  static constexpr int ks[6][3] = {{0, 0, 0}, {4, 8, 16}, {2, 4, 0}, {1, 2, 0}, {1, 0, 0}, {1, 0, 0}};
  if (P < 1 || P > 5) return 0;
  const int m = n - 1;
  int fallback = 0;
  for (int k : ks[P]) {
    if (k == 0) continue;
    const int th = std::max(64, ((m + k - 1) / k + 63) / 64 * 64);
    if (th <= 256) return th;
    if (!fallback && th <= chain_flat_maxt(P, k)) fallback = th;
  }
  return fallback;
}

// Launch shape (ChainArgs::shape): 0 chooses, 1 lean, 2 wide (P = 3 ... 5,
// else lean), 3 flat (P <= 5, when the chain's factors fit the registers of at
// most 1024 threads; else chosen).  The choice: flat for meshes with at most 4
// chains per CU (2n <= 1024) and for P = 2; else wide for P = 3, 4 (within 128
// registers either way), lean otherwise (measured on MI355X at n = 256, k = 4
// and n = 1024, k = 3).
int chain_shape_kind(int P, int n, int shape) {
  const int th = chain_flat_threads(P, n);
  const bool flat_ok = th > 0;
  const bool tri_ok = P == 1 && chain_tri_lmax(n) > 0;
  if ((shape == 4 || shape == 0) && tri_ok) return 4;  // P = 1: the partitioned solve by default
  if (shape == 3 && flat_ok) return 3;  // else as chosen below
  if (shape == 2) return P >= 3 && P <= 5 ? 2 : 1;
  if (shape == 1) return 1;
  if (flat_ok && (P == 2 || 2LL * n <= 1024)) return 3;
  return P >= 3 && P <= 4 ? 2 : 1;
}

template <int P, typename T, int K>
static hipError_t launch_chain_flat_t(const ChainArgs& a, int64_t nch, int threads, size_t lds, hipStream_t s) {
  if (threads > ChainFlat<P, K>::MAXT) return hipErrorInvalidValue;
  if (lds > 65536 && hipFuncSetAttribute(reinterpret_cast<const void*>(&k_chain_flat<P, T, K>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_chain_flat<P, T, K>), dim3((unsigned)nch), dim3(threads), lds, s, a);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_chain_flat(int P, const ChainArgs& a, int64_t nch, int threads, hipStream_t s) {
  const int m = a.n - 1;
  const int K = chain_flat_k(P, (m + threads - 1) / threads);
  const size_t lds = (size_t)m * P * sizeof(T);  // the right-hand side only
  if ((int64_t)lds > (a.lds_cap > 0 ? a.lds_cap : 65536)) return hipErrorInvalidValue;
  switch (P * 32 + K) {
    case 1 * 32 + 4: return launch_chain_flat_t<1, T, 4>(a, nch, threads, lds, s);
    case 1 * 32 + 8: return launch_chain_flat_t<1, T, 8>(a, nch, threads, lds, s);
    case 1 * 32 + 16: return launch_chain_flat_t<1, T, 16>(a, nch, threads, lds, s);
    case 2 * 32 + 2: return launch_chain_flat_t<2, T, 2>(a, nch, threads, lds, s);
    case 2 * 32 + 4: return launch_chain_flat_t<2, T, 4>(a, nch, threads, lds, s);
    case 3 * 32 + 1: return launch_chain_flat_t<3, T, 1>(a, nch, threads, lds, s);
    case 3 * 32 + 2: return launch_chain_flat_t<3, T, 2>(a, nch, threads, lds, s);
    case 4 * 32 + 1: return launch_chain_flat_t<4, T, 1>(a, nch, threads, lds, s);
    case 5 * 32 + 1: return launch_chain_flat_t<5, T, 1>(a, nch, threads, lds, s);
    default: return hipErrorInvalidValue;
  }
}

template <int P, typename T, bool WIDE>
static hipError_t launch_chain_t(const ChainArgs& a, int64_t nch, int threads, size_t lds, hipStream_t s) {
  constexpr bool W = ChainShape<P, WIDE>::W;  // other P have one shape
  // beyond 64 KiB a kernel's dynamic LDS is raised explicitly
  if (lds > 65536 && hipFuncSetAttribute(reinterpret_cast<const void*>(&k_chain<P, T, W>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_chain<P, T, W>), dim3((unsigned)nch), dim3(threads), lds, s, a);
  return hipGetLastError();
}

// ------------------------------------------ partitioned chain solve (P = 1)
// One wavefront per chain; lane k owns segment k (positions o .. o + L - 1, L
// >= 2) of the scalar tridiagonal chain matrix and keeps it in registers:
//  1. the segment interior is solved for the right-hand side with the stored
//     elimination (ch, ip): its end values y_1, y_{L-2} give the right-hand
//     sides gF, gL of the segment's first and last rows in the tridiagonal
//     system that remains on the segment ends;
//  2. eliminating the first ends (one shuffle) leaves one row per lane, solved
//     by parallel cyclic reduction across the lanes (6 levels of shuffles with
//     stored multipliers): the last ends x_l, then the first ends x_o;
//  3. the interior is solved again with x_o and x_l moved to its right-hand side.
// No barrier inside the solve; a workgroup of G wavefronts (G chains) stages the
// right-hand sides and the results in LDS so that global memory is accessed
// along the faces' storage order: a vertical chain's faces are consecutive, a
// horizontal chain's are n apart and G adjacent chains share each 8 G-byte run.
__device__ __forceinline__ int tri_pad(int i) { return i + (i >> 4); }

// RES: the right-hand side is the residual b - S x of the chain's faces,
// gathered from the face slab as the trace kernel does (7 entries per face at
// P = 1), instead of a residual vector computed by a launch of its own; x is
// staged in LDS beside it for the final update.
template <typename T, int LMAX, bool RES>
__global__ __launch_bounds__(512) void k_chain_tri(ChainArgs a) {
  extern __shared__ unsigned char lds_raw[];
  const int n = a.n, m = n - 1;
  const int G = (int)(blockDim.x >> 6);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nvw = (n + G - 1) / G;
  const bool vert = (int)blockIdx.x < nvw;
  const int c0 = vert ? G * (int)blockIdx.x : n + G * ((int)blockIdx.x - nvw);
  const int cend = vert ? n : 2 * n;
  const int c = c0 + w;
  const bool act = c < cend;
  const int ld = m + (m >> 4) + 1;
  T* buf = reinterpret_cast<T*>(lds_raw);
  T* mine = buf + w * ld;
  const T* r = static_cast<const T*>(a.r);
  const T* xin = static_cast<const T*>(a.x);
  T* out = static_cast<T*>(a.out);
  const int64_t nv = (int64_t)n * m;
  const T* rec = static_cast<const T*>(a.tri) + (int64_t)(act ? c : c0) * ((2 * LMAX + kTriScalars) * 64);
  const int nseg = min(64, m / 2), base = m / nseg, extra = m % nseg;
  const int L = lane < nseg ? base + (lane < extra ? 1 : 0) : 0;
  const int o = lane * base + min(lane, extra);
  // the lane's factors first, then the right-hand sides into LDS
  T ch[LMAX], ip[LMAX], sc[kTriScalars];
  ch[0] = ip[0] = ch[LMAX - 1] = ip[LMAX - 1] = T(0);
#pragma unroll
  for (int j = 1; j < LMAX - 1; ++j) {
    ch[j] = rec[j * 64 + lane];
    ip[j] = rec[(LMAX + j) * 64 + lane];
  }
#pragma unroll
  for (int q = 0; q < kTriScalars; ++q) sc[q] = rec[(2 * LMAX + q) * 64 + lane];
  // The faces this thread stages and writes: positions pos0 + 64 t (t < LMAX,
  // which covers m <= 64 LMAX) of one chain; vertical: the wavefront's own chain
  // (pos0 = lane), horizontal: chain tid mod G of the G (pos0 = tid / G), so that
  // G consecutive threads touch G adjacent faces.  Position pos0 + 64 t is face
  // f0 + df t and LDS slot s0 + 68 t (tri_pad adds one slot per 16 positions).
  const int w2 = vert ? w : (int)threadIdx.x % G;
  const int pos0 = vert ? lane : (int)threadIdx.x / G;
  const bool own = vert ? act : c0 + w2 < cend;
  const int64_t f0 = vert ? (int64_t)m * c + lane : nv + (c0 - n + w2) + (int64_t)n * pos0;
  const int64_t df = vert ? 64 : 64 * (int64_t)n;
  const int s0 = w2 * ld + pos0 + (pos0 >> 4);
  // the iterate is requested first, so that its round trip overlaps the
  // right-hand side's and the factors' (while the registers allow)
  constexpr bool XPRE = !RES && LMAX * sizeof(T) <= 128;
  T* xbuf = buf + G * ld;  // RES: the iterate of every staged face
  T xr[LMAX];
  if (XPRE && xin) {
#pragma unroll
    for (int t = 0; t < LMAX; ++t) xr[t] = own && pos0 + 64 * t < m ? xin[f0 + df * t] : T(0);
  }
  if constexpr (RES) {
    // two faces per round: slab words, the 7 gathered x values and b of both
    // are requested before either is summed (missing neighbours and slots past
    // the chain read face 0 and are zeroed or not stored)
    using L16 = Lanes16<T, T>;
    constexpr int V = L16::V, NQ = (7 + V - 1) / V;
    const u32x4* sp = static_cast<const u32x4*>(a.slab);
    const T* bvec = static_cast<const T*>(a.b);
#pragma unroll
    for (int t0 = 0; t0 < LMAX; t0 += 2) {
      T wv[2][NQ * V], xv[2][7], bb[2];
      unsigned okm[2];
      bool okf[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int t = t0 + u;
        okf[u] = own && pos0 + 64 * t < m;
        const int64_t f = okf[u] ? f0 + df * t : 0;
        int64_t g[7];
        face_neighbours(n, nv, f, g);
#pragma unroll
        for (int q = 0; q < NQ; ++q) L16::unpack(sp[((f >> 6) * NQ + q) * 64 + (f & 63)], &wv[u][q * V]);
        okm[u] = 0;
#pragma unroll
        for (int s = 0; s < 7; ++s) {
          okm[u] |= (g[s] >= 0 ? 1u : 0u) << s;
          xv[u][s] = xin[g[s] >= 0 ? g[s] : f];
        }
        bb[u] = bvec[f];
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        T acc = T(0);
#pragma unroll
        for (int e = 0; e < 7; ++e) acc = fma_t(wv[u][e], (okm[u] >> e) & 1u ? xv[u][e] : T(0), acc);
        if (okf[u]) {
          buf[s0 + 68 * (t0 + u)] = bb[u] - acc;
          xbuf[s0 + 68 * (t0 + u)] = xv[u][0];
        }
      }
    }
  } else {
#pragma unroll
    for (int t = 0; t < LMAX; ++t)
      if (own && pos0 + 64 * t < m) buf[s0 + 68 * t] = r[f0 + df * t];
  }
  __syncthreads();
  // 1. interior solve (slots outside the interior hold ch = ip = 0); only the
  //    end values of the backward sweep are kept
  const T r0 = L > 0 ? mine[tri_pad(o)] : T(0);
  T u[LMAX], rl = r0;
  u[0] = T(0);
#pragma unroll
  for (int j = 1; j < LMAX; ++j) {
    const T rj = j < L ? mine[tri_pad(o + j)] : T(0);
    u[j] = fma_t(-ch[j - 1], u[j - 1], rj);
    rl = j == L - 1 ? rj : rl;
  }
  T yn = T(0), y1 = T(0), yl = T(0);
#pragma unroll
  for (int j = LMAX - 2; j >= 1; --j) {
    yn = fma_t(-ch[j], yn, u[j] * ip[j]);
    yl = j == L - 2 ? yn : yl;
    y1 = yn;
  }
  // 2. the segment ends
  const T gF = fma_t(-sc[0], y1, r0);
  const T gL = fma_t(-sc[1], yl, rl);
  const T gF1 = __shfl_down(gF, 1, 64);
  T g = fma_t(-sc[3], gF1, fma_t(-sc[2], gF, gL));
#pragma unroll
  for (int h = 0; h < 6; ++h) {
    const T gm = __shfl_up(g, 1 << h, 64), gp = __shfl_down(g, 1 << h, 64);
    g = fma_t(-sc[8 + 2 * h], gp, fma_t(-sc[7 + 2 * h], gm, g));
  }
  const T xL = g * sc[19];
  const T xLm = __shfl_up(xL, 1, 64);
  const T xF = fma_t(-sc[6], xL, fma_t(-sc[5], xLm, gF)) * sc[4];
  // 3. interior with the ends known: the forward sweep is linear, so x_o enters
  //    as x_o phi_j (phi_1 = -E_o, phi_{j+1} = -ch_j phi_j) and x_l at the last
  //    interior position; then the backward sweep in place
  T phi = -sc[0];
#pragma unroll
  for (int j = 1; j < LMAX; ++j) {
    u[j] = fma_t(xF, phi, u[j]);
    u[j] = j == L - 2 ? fma_t(-sc[1], xL, u[j]) : u[j];
    phi = -ch[j] * phi;
  }
  u[LMAX - 1] = T(0);
#pragma unroll
  for (int j = LMAX - 2; j >= 1; --j) u[j] = fma_t(-ch[j], u[j + 1], u[j] * ip[j]);
#pragma unroll
  for (int j = 0; j < LMAX; ++j)
    if (j < L) mine[tri_pad(o + j)] = j == 0 ? xF : (j == L - 1 ? xL : u[j]);
  __syncthreads();
  const T om = T(a.omega);
#pragma unroll
  for (int t = 0; t < LMAX; ++t)
    if (own && pos0 + 64 * t < m)
      out[f0 + df * t] = (xin ? (RES ? xbuf[s0 + 68 * t] : (XPRE ? xr[t] : xin[f0 + df * t])) : T(0)) +
                         om * buf[s0 + 68 * t];
}

int chain_tri_lmax(int n) {
  const int m = n - 1;
  if (m < 4) return 0;
  const int nseg = std::min(64, m / 2);
  const int lmax = (m + nseg - 1) / nseg;
  for (int b : {4, 8, 16, 32})
    if (lmax <= b) return b;
  return 0;
}
int64_t chain_tri_stride(int n) { return (int64_t)(2 * chain_tri_lmax(n) + kTriScalars) * 64; }
size_t chain_tri_lds_bytes(int n, int G, size_t es) {
  const int m = n - 1;
  return (size_t)G * (m + (m >> 4) + 1) * es;
}

template <typename T, int LMAX, bool RES>
static hipError_t launch_chain_tri_t(const ChainArgs& a, int G, hipStream_t s) {
  const size_t lds = chain_tri_lds_bytes(a.n, G, sizeof(T)) * (RES ? 2 : 1);
  if ((int64_t)lds > (a.lds_cap > 0 ? a.lds_cap : 65536)) return hipErrorInvalidValue;
  if (lds > 65536 && hipFuncSetAttribute(reinterpret_cast<const void*>(&k_chain_tri<T, LMAX, RES>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return hipErrorInvalidValue;
  const int nvw = (a.n + G - 1) / G;
  hipLaunchKernelGGL((k_chain_tri<T, LMAX, RES>), dim3((unsigned)(2 * nvw)), dim3(64 * G), lds, s, a);
  return hipGetLastError();
}
template <typename T, int LMAX>
static hipError_t launch_chain_tri_r(const ChainArgs& a, int G, hipStream_t s) {
  // the residual in the launch needs x, b and the slab, and no residual vector
  const bool res = a.r == nullptr && a.b != nullptr && a.slab != nullptr && a.x != nullptr;
  if (!res && a.r == nullptr) return hipErrorInvalidValue;
  if (!res) return launch_chain_tri_t<T, LMAX, false>(a, G, s);
  // the staged iterate doubles the LDS: fewer chains per workgroup where it
  // does not fit (each chain's arithmetic does not depend on it)
  const int64_t cap = a.lds_cap > 0 ? a.lds_cap : 65536;
  while (G > 1 && (int64_t)(2 * chain_tri_lds_bytes(a.n, G, sizeof(T))) > cap) G /= 2;
  return launch_chain_tri_t<T, LMAX, true>(a, G, s);
}

template <typename T>
static hipError_t launch_chain_tri(const ChainArgs& a, hipStream_t s) {
  const int G = a.threads > 0 ? a.threads / 64 : 4;
  if (a.threads % 64 || G < 1 || G > 8 || !a.tri) return hipErrorInvalidValue;
  switch (chain_tri_lmax(a.n)) {
    case 4: return launch_chain_tri_r<T, 4>(a, G, s);
    case 8: return launch_chain_tri_r<T, 8>(a, G, s);
    case 16: return launch_chain_tri_r<T, 16>(a, G, s);
    case 32: return launch_chain_tri_r<T, 32>(a, G, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_chain_solve(Prec pr, int P, const ChainArgs& a, hipStream_t s) {
  const int64_t nch = 2LL * a.n;
  const int kind = chain_shape_kind(P, a.n, a.shape);
  if (kind == 0) return hipErrorInvalidValue;
  if (kind == 4) {
    // the residual in the launch reads the slab as vector-precision words: a
    // bfloat16 slab has another word layout
    if (pr == Prec::BF16 && a.r == nullptr) return hipErrorInvalidValue;
    return pr == Prec::F64 ? launch_chain_tri<double>(a, s) : launch_chain_tri<float>(a, s);
  }
  if (kind == 3) {
    const int threads = a.threads > 0 ? a.threads : chain_flat_threads(P, a.n);
    if (threads % 64 || threads > 1024) return hipErrorInvalidValue;
    return pr == Prec::F64 ? launch_chain_flat<double>(P, a, nch, threads, s)
                           : launch_chain_flat<float>(P, a, nch, threads, s);
  }
  const int threads = a.threads > 0 ? a.threads : chain_threads(P, a.n);
  const size_t lds = chain_lds_bytes(P, a.n, vec_bytes(pr), a.lds_level);
  if ((int64_t)lds > (a.lds_cap > 0 ? a.lds_cap : 65536)) return hipErrorInvalidValue;
  const bool wide = kind == 2;
  if (chain_max_threads(P, wide) == 0 || threads > chain_max_threads(P, wide) || threads % 64)
    return hipErrorInvalidValue;
  if (pr == Prec::F64) {
    HDG_DISPATCH_P(P, return wide ? (launch_chain_t<PP, double, true>)(a, nch, threads, lds, s)
                                  : (launch_chain_t<PP, double, false>)(a, nch, threads, lds, s));
  } else {
    HDG_DISPATCH_P(P, return wide ? (launch_chain_t<PP, float, true>)(a, nch, threads, lds, s)
                                  : (launch_chain_t<PP, float, false>)(a, nch, threads, lds, s));
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ Q1 levels
// The per-vertex arithmetic of the Q1 levels is written once, with fused
// multiply-adds in a fixed order, and shared by the one-operation kernels and
// the fused level kernels below, whose results are therefore bit-identical.
//
// 9-point stencil sum at interior vertex (i, j): dj outer, di inner; sat(d)
// returns the vertex's stencil entry for direction d = (di + 1) + 3 (dj + 1),
// xat(ic, jc) x at a clamped (existing) vertex, zeroed here for neighbours
// outside the interior, so no load sits under a branch (the stencil entries
// are finite).
template <typename T, typename SAt, typename XAt>
__device__ __forceinline__ T q1_stencil_sum(int m, int i, int j, SAt sat, XAt xat) {
  T s = T(0);
#pragma unroll
  for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
    for (int di = -1; di <= 1; ++di) {
      const int ii = i + di, jj = j + dj;
      const bool ok = ii >= 1 && jj >= 1 && ii <= m - 1 && jj <= m - 1;
      const int ic = min(max(ii, 1), m - 1), jc = min(max(jj, 1), m - 1);
      const T xv = xat(ic, jc);
      s = fma_t(sat((di + 1) + 3 * (dj + 1)), ok ? xv : T(0), s);
    }
  return s;
}

// The cycle's Q1 operators are symmetric (Galerkin products R A P with R =
// P^T), and their stencils are kept by five entries per vertex: directions 4
// ... 8 (centre, east, north-west, north, north-east) at st[(d - 4) Nv + v].  The
// other four are the mirrored entries of the neighbour, A[v, v + e] =
// A[v + e, v], read at a clamped vertex where the neighbour is outside the
// interior (the caller masks that term).  HBM traffic per stencil sweep: 5
// entries per vertex instead of 9.
template <typename T>
__device__ __forceinline__ T q1_sym_entry(const T* st, int64_t Nv, int m, int i, int j, int64_t v, int d) {
  if (d >= 4) return st[(int64_t)(d - 4) * Nv + v];
  const int di = d % 3 - 1, dj = d / 3 - 1;
  const int ic = min(max(i + di, 1), m - 1), jc = min(max(j + dj, 1), m - 1);
  return st[(int64_t)(4 - d) * Nv + (ic - 1) + (int64_t)(m - 1) * (jc - 1)];
}

template <typename T>
__device__ __forceinline__ T q1_apply(const T* st, const T* x, int m, int64_t Nv, int i, int j, int64_t v) {
  return q1_stencil_sum<T>(
      m, i, j, [&](int d) { return q1_sym_entry(st, Nv, m, i, j, v, d); },
      [&](int ic, int jc) { return x[(ic - 1) + (int64_t)(m - 1) * (jc - 1)]; });
}

// r = b - A x with the full 9-entry FP64 stencil st[9][Nv] of the set-up (the
// Lanczos estimate of lambda_max runs before the cycle copy exists).
__global__ __launch_bounds__(kWG) void k_q1_resid9(const double* st, const double* b, const double* x, double* r,
                                                   int m) {
  const int64_t Nv = (int64_t)(m - 1) * (m - 1);
  const int64_t v = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (v >= Nv) return;
  const int i = (int)(v % (m - 1)) + 1, j = (int)(v / (m - 1)) + 1;
  r[v] = b[v] - q1_stencil_sum<double>(
                    m, i, j, [&](int d) { return st[(int64_t)d * Nv + v]; },
                    [&](int ic, int jc) { return x[(ic - 1) + (int64_t)(m - 1) * (jc - 1)]; });
}

// One Chebyshev step at a vertex: z = Dinv (b - A x), d' = c1 d + c2 z (c1 = 0
// on the first step: d is not read), x' = x + d'.
template <typename T>
__device__ __forceinline__ T q1_cheb_dir(T dinv, T b, T ax, T d, double c1, double c2) {
#pragma clang fp contract(off)
  const T z = dinv * (b - ax);
  const T cz = T(c2) * z;
  return c1 != 0.0 ? fma_t(T(c1), d, cz) : cz;
}

// Full weighting at coarse vertex (I, J): fine (2I + di, 2J + dj), weight
// w(di) w(dj), dj outer, di inner (the fine vertices are always interior).
template <typename T, typename RAt>
__device__ __forceinline__ T q1_restrict_sum(int I, int J, RAt rat) {
  T s = T(0);
#pragma unroll
  for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
    for (int di = -1; di <= 1; ++di) {
      const T w = T((di == 0 ? 1.0 : 0.5) * (dj == 0 ? 1.0 : 0.5));
      s = fma_t(w, rat(2 * I + di, 2 * J + dj), s);
    }
  return s;
}

// Bilinear interpolation at fine vertex (I, J) from the 2 x 2 coarse vertices
// around it: an even index has one parent (the second weight is 0); parents
// outside the interior read a clamped vertex and are zeroed.
template <typename T>
__device__ __forceinline__ T q1_prolong_sum(const T* ec, int mc, int I, int J) {
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
      const T e = ec[((cic - 1) + (int64_t)(mc - 1) * (cjc - 1))];
      s = fma_t(wx[aa] * wy[bb], ok ? e : T(0), s);
    }
  return s;
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_q1_resid(const T* st, const T* b, const T* x, T* r, int m) {
  const int64_t Nv = (int64_t)(m - 1) * (m - 1);
  const int64_t v = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (v >= Nv) return;
  const int i = (int)(v % (m - 1)) + 1, j = (int)(v / (m - 1)) + 1;
  r[v] = b[v] - q1_apply(st, x, m, Nv, i, j, v);
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_q1_cheb(const T* st, const T* dinv, const T* b, const T* x, T* d, T* xo,
                                                 double c1, double c2, int m) {
#pragma clang fp contract(off)
  const int64_t Nv = (int64_t)(m - 1) * (m - 1);
  const int64_t v = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (v >= Nv) return;
  const int i = (int)(v % (m - 1)) + 1, j = (int)(v / (m - 1)) + 1;
  const T ax = x ? q1_apply(st, x, m, Nv, i, j, v) : T(0);
  const T dn = q1_cheb_dir(dinv[v], b[v], ax, c1 != 0.0 ? d[v] : T(0), c1, c2);
  d[v] = dn;
  xo[v] = (x ? x[v] : T(0)) + dn;
}

// full weighting: coarse vertex (I, J) gathers fine (2I + di, 2J + dj), weight w(di) w(dj)
template <typename T>
__global__ __launch_bounds__(kWG) void k_q1_restrict(const T* rf, T* rc, int mf) {
  const int mc = mf / 2;
  const int64_t Nc = (int64_t)(mc - 1) * (mc - 1);
  const int64_t v = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (v >= Nc) return;
  const int I = (int)(v % (mc - 1)) + 1, J = (int)(v / (mc - 1)) + 1;
  rc[v] = q1_restrict_sum<T>(I, J, [&](int fi, int fj) { return rf[(fi - 1) + (int64_t)(mf - 1) * (fj - 1)]; });
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_q1_prolong_add(const T* ec, T* xf, int mf) {
  const int mc = mf / 2;
  const int64_t Nf = (int64_t)(mf - 1) * (mf - 1);
  const int64_t v = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (v >= Nf) return;
  const int I = (int)(v % (mf - 1)) + 1, J = (int)(v / (mf - 1)) + 1;
  xf[v] += q1_prolong_sum(ec, mc, I, J);
}

// Fused level visits of the Q1 hierarchy (Sec. 7: Chebyshev smoothing on the
// Q1 levels).  One launch does the pre-smoothing steps, the residual and the
// full-weighting restriction of a level; a second the bilinear prolongation of
// the coarse correction and the post-smoothing steps.  Each workgroup owns a
// TS x TS tile of interior vertices and works on the tile grown by a halo
// (redundantly with its neighbours): a step on the tile grown by h needs the
// previous iterate on the tile grown by h + 1, so the halo shrinks by one
// vertex per step and no workgroup waits for another.  The iterates, the
// Chebyshev directions and the residual live in LDS; only the level's inputs,
// its new iterate and the restricted residual touch global memory.
//
// Region R_h: the tile's vertices [t0 + 1, t0 + TS] in each direction grown by
// h and clipped to the interior [1, m - 1].  LDS arrays cover the tile grown by
// the kernel's full halo H, with origin t0 + 1 - H.
struct Q1Tile {
  int m;
  int ti0, tj0;  // first vertex of the tile in each direction
  int i0, j0;    // origin of the LDS region
  int RW;        // LDS region width
  int TS;
};

// Workgroup -> tile: the tiles of one contiguous band go to one XCD (dispatch
// deals workgroups to the XCDs round robin), so the halo rows that adjacent
// tiles share are read through the same L2.
__device__ __forceinline__ bool q1_tile(int m, int TS, int H, Q1Tile& t) {
  const int nt = (m - 1 + TS - 1) / TS;
  const int ntot = nt * nt, per = (ntot + 7) / 8;
  const int tile = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (tile >= ntot) return false;
  t.m = m;
  t.TS = TS;
  t.ti0 = (tile % nt) * TS + 1;
  t.tj0 = (tile / nt) * TS + 1;
  t.i0 = t.ti0 - H;
  t.j0 = t.tj0 - H;
  t.RW = TS + 2 * H;
  return true;
}

// f(i, j, v, l) for every vertex of R_h: (i, j) the vertex, v its global index,
// l its LDS index.
template <typename F>
__device__ __forceinline__ void q1_for_region(const Q1Tile& t, int h, F f) {
  const int lo_i = max(1, t.ti0 - h), hi_i = min(t.m - 1, t.ti0 + t.TS - 1 + h);
  const int lo_j = max(1, t.tj0 - h), hi_j = min(t.m - 1, t.tj0 + t.TS - 1 + h);
  const int w = hi_i - lo_i + 1, cnt = w * (hi_j - lo_j + 1);
  for (int q = threadIdx.x; q < cnt; q += kQ1Threads) {
    const int i = lo_i + q % w, j = lo_j + q / w;
    f(i, j, (int64_t)(i - 1) + (int64_t)(t.m - 1) * (j - 1), (i - t.i0) + t.RW * (j - t.j0));
  }
}

// Batched walk of R_h: each round takes vertices q0 + b kQ1Threads (b < B) and
// issues the global loads of all B (load(b, i, j, v)) before using any of them
// (use(b, i, j, v, l, ok)), so that a workgroup waits on memory once per round,
// not once per vertex.  A slot past the region takes the region's last vertex
// (valid indices, finite values) with ok = false: it must store nothing.
template <int B, typename Load, typename Use>
__device__ __forceinline__ void q1_for_region_b(const Q1Tile& t, int h, Load load, Use use) {
  const int lo_i = max(1, t.ti0 - h), hi_i = min(t.m - 1, t.ti0 + t.TS - 1 + h);
  const int lo_j = max(1, t.tj0 - h), hi_j = min(t.m - 1, t.tj0 + t.TS - 1 + h);
  const int w = hi_i - lo_i + 1, cnt = w * (hi_j - lo_j + 1);
  for (int q0 = threadIdx.x; q0 < cnt; q0 += B * kQ1Threads) {
    int ii[B], jj[B];
    bool ok[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int q = q0 + b * kQ1Threads;
      ok[b] = q < cnt;
      const int qc = ok[b] ? q : cnt - 1;
      ii[b] = lo_i + qc % w;
      jj[b] = lo_j + qc / w;
      load(b, ii[b], jj[b], (int64_t)(ii[b] - 1) + (int64_t)(t.m - 1) * (jj[b] - 1));
    }
#pragma unroll
    for (int b = 0; b < B; ++b)
      use(b, ii[b], jj[b], (int64_t)(ii[b] - 1) + (int64_t)(t.m - 1) * (jj[b] - 1),
          (ii[b] - t.i0) + t.RW * (jj[b] - t.j0), ok[b]);
  }
}

// nu Chebyshev steps in LDS, the last on R_hend (step s on R_{hend + nu - 1 - s});
// xa holds the iterate on R_{hend + nu} on entry (unread when zero) and the
// result on exit; xb and dd are work arrays.
template <typename T, int B>
__device__ __forceinline__ void q1_cheb_steps(const Q1Tile& t, const T* st, const T* dinv, const T* b, int nu,
                                              int hend, bool zero, const Q1FusedArgs& a, T*& xa, T*& xb, T* dd) {
#pragma clang fp contract(off)
  const int64_t Nv = (int64_t)(t.m - 1) * (t.m - 1);
  for (int s = 0; s < nu; ++s) {
    const bool z0 = zero && s == 0;
    const double c1 = a.c1[s], c2 = a.c2[s];
    const T* xr = xa;
    T* xw = xb;
    T stv[B][9], dv[B], bv[B];
    q1_for_region_b<B>(
        t, hend + nu - 1 - s,
        [&](int q, int i, int j, int64_t v) {
          if (!z0) {
#pragma unroll
            for (int d = 0; d < 9; ++d) stv[q][d] = q1_sym_entry(st, Nv, t.m, i, j, v, d);
          }
          dv[q] = dinv[v];
          bv[q] = b[v];
        },
        [&](int q, int i, int j, int64_t, int l, bool ok) {
          const T ax = z0 ? T(0)
                          : q1_stencil_sum<T>(
                                t.m, i, j, [&](int d) { return stv[q][d]; },
                                [&](int ic, int jc) { return xr[(ic - t.i0) + t.RW * (jc - t.j0)]; });
          const T dn = q1_cheb_dir(dv[q], bv[q], ax, c1 != 0.0 ? dd[l] : T(0), c1, c2);
          if (ok) {
            dd[l] = dn;
            xw[l] = (z0 ? T(0) : xr[l]) + dn;
          }
        });
    __syncthreads();
    xa = xw;
    xb = const_cast<T*>(xr);
  }
}

// Pre-smoothing visit: nu1 steps from x_in (zero when null), x_out = the new
// iterate, bc = full-weighting restriction of b - A x_out to the coarse level.
template <typename T, int B>
__global__ __launch_bounds__(kQ1Threads) void k_q1_pre(Q1FusedArgs a) {
  extern __shared__ unsigned char lds_raw[];
  const int m = a.m, nu = a.nu, H = nu + 2;
  Q1Tile t;
  if (!q1_tile(m, a.tile, H, t)) return;
  T* xa = reinterpret_cast<T*>(lds_raw);
  T* xb = xa + t.RW * t.RW;
  T* dd = xb + t.RW * t.RW;
  const T* st = static_cast<const T*>(a.st);
  const T* dinv = static_cast<const T*>(a.dinv);
  const T* b = static_cast<const T*>(a.b);
  const T* xin = static_cast<const T*>(a.x_in);
  T* xout = static_cast<T*>(a.x_out);
  const bool zero = xin == nullptr;
  if (!zero) {
    T xv[B];
    q1_for_region_b<B>(
        t, H, [&](int q, int, int, int64_t v) { xv[q] = xin[v]; },
        [&](int q, int, int, int64_t, int l, bool ok) {
          if (ok) xa[l] = xv[q];
        });
    __syncthreads();
  }
  q1_cheb_steps<T, B>(t, st, dinv, b, nu, 2, zero, a, xa, xb, dd);
  const int64_t Nv = (int64_t)(m - 1) * (m - 1);
  q1_for_region(t, 0, [&](int, int, int64_t v, int l) { xout[v] = xa[l]; });
  {
    T stv[B][9], bv[B];
    q1_for_region_b<B>(
        t, 1,
        [&](int q, int i, int j, int64_t v) {
#pragma unroll
          for (int d = 0; d < 9; ++d) stv[q][d] = q1_sym_entry(st, Nv, m, i, j, v, d);
          bv[q] = b[v];
        },
        [&](int q, int i, int j, int64_t, int l, bool ok) {
          const T r = bv[q] - q1_stencil_sum<T>(
                                  m, i, j, [&](int d) { return stv[q][d]; },
                                  [&](int ic, int jc) { return xa[(ic - t.i0) + t.RW * (jc - t.j0)]; });
          if (ok) xb[l] = r;
        });
  }
  __syncthreads();
  // coarse vertices (I, J) whose fine vertex (2I, 2J) lies in the tile; their
  // fine neighbours lie in R_1
  const int mc = m / 2, hs = t.TS / 2;
  const int I0 = (t.ti0 + 1) / 2, J0 = (t.tj0 + 1) / 2;
  const int nI = min(hs, mc - I0), nJ = min(hs, mc - J0);
  T* bc = static_cast<T*>(a.bc);
  for (int q = threadIdx.x; q < nI * nJ; q += kQ1Threads) {
    const int I = I0 + q % nI, J = J0 + q / nI;
    bc[(I - 1) + (int64_t)(mc - 1) * (J - 1)] =
        q1_restrict_sum<T>(I, J, [&](int fi, int fj) { return xb[(fi - t.i0) + t.RW * (fj - t.j0)]; });
  }
}

// Post-smoothing visit: x = x_in + P e (e the coarse correction in a.ec), then
// nu2 steps; x_out = the result (x_out != x_in: neighbouring tiles read x_in).
template <typename T, int B>
__global__ __launch_bounds__(kQ1Threads) void k_q1_post(Q1FusedArgs a) {
  extern __shared__ unsigned char lds_raw[];
  const int m = a.m, nu = a.nu, H = nu;
  Q1Tile t;
  if (!q1_tile(m, a.tile, H, t)) return;
  T* xa = reinterpret_cast<T*>(lds_raw);
  T* xb = xa + t.RW * t.RW;
  T* dd = xb + t.RW * t.RW;
  const T* xin = static_cast<const T*>(a.x_in);
  const T* ec = static_cast<const T*>(a.ec);
  const int mc = m / 2;
  {
    T xv[B];
    q1_for_region_b<B>(
        t, H, [&](int q, int i, int j, int64_t v) { xv[q] = xin[v] + q1_prolong_sum(ec, mc, i, j); },
        [&](int q, int, int, int64_t, int l, bool ok) {
          if (ok) xa[l] = xv[q];
        });
  }
  __syncthreads();
  q1_cheb_steps<T, B>(t, static_cast<const T*>(a.st), static_cast<const T*>(a.dinv), static_cast<const T*>(a.b), nu,
                      0, false, a, xa, xb, dd);
  T* xout = static_cast<T*>(a.x_out);
  q1_for_region(t, 0, [&](int, int, int64_t v, int l) { xout[v] = xa[l]; });
}

// P_J^T: vertex (i, j) gathers its four incident interior faces, weight 1/2
template <typename T>
__global__ __launch_bounds__(kWG) void k_pj_restrict(const T* rface, T* rv, int n) {
  const int64_t Nv = (int64_t)(n - 1) * (n - 1);
  const int64_t v = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (v >= Nv) return;
  const int i = (int)(v % (n - 1)) + 1, j = (int)(v / (n - 1)) + 1;
  const int64_t nv = (int64_t)n * (n - 1);
  const T s = rface[(i - 1) + (int64_t)(n - 1) * j] + rface[(i - 1) + (int64_t)(n - 1) * (j - 1)] +
              rface[nv + i + (int64_t)n * (j - 1)] + rface[nv + (i - 1) + (int64_t)n * (j - 1)];
  rv[v] = T(0.5) * s;
}

// P_J: face value += mean of its two end vertices (boundary vertices are 0)
template <typename T>
__global__ __launch_bounds__(kWG) void k_pj_prolong_add(const T* ev, T* xface, int n) {
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
  T s = T(0);
  {  // end vertices on the boundary read a clamped vertex and are zeroed
    const bool oa = ai >= 1 && aj >= 1 && ai <= n - 1 && aj <= n - 1;
    const bool ob = bi >= 1 && bj >= 1 && bi <= n - 1 && bj <= n - 1;
    const T ea = ev[(min(max(ai, 1), n - 1) - 1) + (int64_t)(n - 1) * (min(max(aj, 1), n - 1) - 1)];
    const T eb = ev[(min(max(bi, 1), n - 1) - 1) + (int64_t)(n - 1) * (min(max(bj, 1), n - 1) - 1)];
    s += oa ? ea : T(0);
    s += ob ? eb : T(0);
  }
  xface[f] += T(0.5) * s;
}

// one wavefront per row, lanes stride the columns with four independent
// partial sums (four loads in flight per lane), fixed shuffle-tree sum (FP64)
template <typename T>
__global__ __launch_bounds__(kWG) void k_dense_gemv(const double* A, const T* b, T* y, int m) {
  const int row = blockIdx.x * (kWG / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= m) return;
  const double* Ar = A + (int64_t)row * m;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int c = lane;
  for (; c + 192 < m; c += 256) {
    s0 = fma(Ar[c], (double)b[c], s0);
    s1 = fma(Ar[c + 64], (double)b[c + 64], s1);
    s2 = fma(Ar[c + 128], (double)b[c + 128], s2);
    s3 = fma(Ar[c + 192], (double)b[c + 192], s3);
  }
  for (; c < m; c += 64) s0 = fma(Ar[c], (double)b[c], s0);
  double s = (s0 + s1) + (s2 + s3);
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) y[row] = T(s);
}

#define HDG_DISPATCH_T(pr, CALL)                      \
  if ((pr) == Prec::F64) { using TT = double; CALL; } \
  else { using TT = float; CALL; }

hipError_t launch_q1_resid(Prec pr, const void* st, const void* b, const void* x, void* r, int m, hipStream_t s) {
  HDG_DISPATCH_T(pr, hipLaunchKernelGGL(k_q1_resid<TT>, grid_for((int64_t)(m - 1) * (m - 1)), dim3(kWG), 0, s,
                                        (const TT*)st, (const TT*)b, (const TT*)x, (TT*)r, m));
  return hipGetLastError();
}
hipError_t launch_q1_resid9(const double* st, const double* b, const double* x, double* r, int m, hipStream_t s) {
  hipLaunchKernelGGL(k_q1_resid9, grid_for((int64_t)(m - 1) * (m - 1)), dim3(kWG), 0, s, st, b, x, r, m);
  return hipGetLastError();
}
hipError_t launch_q1_cheb(Prec pr, const void* st, const void* dinv, const void* b, const void* x, void* d,
                          void* xo, double c1, double c2, int m, hipStream_t s) {
  HDG_DISPATCH_T(pr, hipLaunchKernelGGL(k_q1_cheb<TT>, grid_for((int64_t)(m - 1) * (m - 1)), dim3(kWG), 0, s,
                                        (const TT*)st, (const TT*)dinv, (const TT*)b, (const TT*)x, (TT*)d,
                                        (TT*)xo, c1, c2, m));
  return hipGetLastError();
}
hipError_t launch_q1_restrict(Prec pr, const void* rf, void* rc, int mf, hipStream_t s) {
  const int mc = mf / 2;
  HDG_DISPATCH_T(pr, hipLaunchKernelGGL(k_q1_restrict<TT>, grid_for((int64_t)(mc - 1) * (mc - 1)), dim3(kWG), 0,
                                        s, (const TT*)rf, (TT*)rc, mf));
  return hipGetLastError();
}
hipError_t launch_q1_prolong_add(Prec pr, const void* ec, void* xf, int mf, hipStream_t s) {
  HDG_DISPATCH_T(pr, hipLaunchKernelGGL(k_q1_prolong_add<TT>, grid_for((int64_t)(mf - 1) * (mf - 1)), dim3(kWG),
                                        0, s, (const TT*)ec, (TT*)xf, mf));
  return hipGetLastError();
}
// The largest tile that still gives at least 32 x 32 tiles (four workgroups
// per CU: a workgroup's phases are a chain of memory round trips, which other
// resident workgroups hide); below that 8 x 8.
int q1_fused_tile(int m) {
  if (m - 1 > 31 * 32) return 32;
  if (m - 1 > 31 * 16) return 16;
  return 8;
}
static hipError_t launch_q1_fused(Prec pr, bool pre, const Q1FusedArgs& a, hipStream_t s) {
  if (a.nu < 1 || a.nu > kQ1MaxNu || (a.m % 2) != 0 || a.m < 4 || (a.tile != 8 && a.tile != 16 && a.tile != 32) ||
      a.c1[0] != 0.0 || !a.st || !a.dinv || !a.b || !a.x_out || (pre ? !a.bc : (!a.x_in || !a.ec)) ||
      a.x_in == a.x_out)
    return hipErrorInvalidValue;
  const int H = pre ? a.nu + 2 : a.nu, RW = a.tile + 2 * H;
  const int nt = (a.m - 1 + a.tile - 1) / a.tile, per = (nt * nt + 7) / 8;
  const size_t lds = (size_t)3 * RW * RW * (pr == Prec::F64 ? sizeof(double) : sizeof(float));
  // vertices per thread and round (measured at n = 1024: two for the
  // pre-smoothing visit on 32 x 32 and 16 x 16 tiles, 37.0 -> 34.7 and 14.6 ->
  // 13.1 us; four, or two in the post-smoothing visit, were slower: registers)
  if (pre && a.tile >= 16) {
    HDG_DISPATCH_T(pr, hipLaunchKernelGGL((k_q1_pre<TT, 2>), dim3(8 * per), dim3(kQ1Threads), lds, s, a));
  } else if (pre) {
    HDG_DISPATCH_T(pr, hipLaunchKernelGGL((k_q1_pre<TT, 1>), dim3(8 * per), dim3(kQ1Threads), lds, s, a));
  } else {
    HDG_DISPATCH_T(pr, hipLaunchKernelGGL((k_q1_post<TT, 1>), dim3(8 * per), dim3(kQ1Threads), lds, s, a));
  }
  return hipGetLastError();
}
hipError_t launch_q1_pre(Prec pr, const Q1FusedArgs& a, hipStream_t s) { return launch_q1_fused(pr, true, a, s); }
hipError_t launch_q1_post(Prec pr, const Q1FusedArgs& a, hipStream_t s) { return launch_q1_fused(pr, false, a, s); }
hipError_t launch_pj_restrict(Prec pr, const void* rface, void* rv, int n, hipStream_t s) {
  HDG_DISPATCH_T(pr, hipLaunchKernelGGL(k_pj_restrict<TT>, grid_for((int64_t)(n - 1) * (n - 1)), dim3(kWG), 0, s,
                                        (const TT*)rface, (TT*)rv, n));
  return hipGetLastError();
}
hipError_t launch_pj_prolong_add(Prec pr, const void* ev, void* xface, int n, hipStream_t s) {
  HDG_DISPATCH_T(pr, hipLaunchKernelGGL(k_pj_prolong_add<TT>, grid_for(2LL * n * (n - 1)), dim3(kWG), 0, s,
                                        (const TT*)ev, (TT*)xface, n));
  return hipGetLastError();
}
hipError_t launch_dense_gemv(Prec pr, const double* A, const void* b, void* y, int m, hipStream_t s) {
  HDG_DISPATCH_T(pr, hipLaunchKernelGGL(k_dense_gemv<TT>, dim3((m + 3) / 4), dim3(kWG), 0, s, A, (const TT*)b,
                                        (TT*)y, m));
  return hipGetLastError();
}

// ---------------------------------------------------------------- reductions
// ----------------------------------------------------- element-local kernels
// Misfit gradient with respect to theta_K = log K_K (adjoint method on eqs.
// shur0 / shur1; A_K = exp(-theta_K) A0).  One 64-lane workgroup per element;
// lanes take the rows of each small dense product, vectors live in LDS, the
// reference matrices (a few KiB) stay in L1 / L2.
template <int P>
struct ElemRef {
  static constexpr int P2 = P * P, F4 = 4 * P;
  const double *V, *delta, *mu, *E, *H, *C, *Bt, *Mvinv;
  __device__ explicit ElemRef(const double* r) {
    V = r;
    delta = V + P2 * P2;
    mu = delta + P2;
    E = mu + P2;
    H = E + P2 * F4;
    C = H + P2 * F4;
    Bt = C + 2 * P2 * F4;
    Mvinv = Bt + 2 * P2 * P2;
  }
};

// the element's 4P trace values: interior faces from lam, boundary faces from
// lam_bd (or 0 when lam_bd is null)
template <int P>
__device__ void elem_trace(const double* lam, const double* lam_bd, int n, int i, int j, double* out) {
  const int64_t nv = (int64_t)n * (n - 1);
  for (int idx = threadIdx.x; idx < 4 * P; idx += 64) {
    const int lf = idx / P, c = idx - lf * P;
    int64_t f = -1, nb = -1;
    switch (lf) {
      case 0: if (i >= 1) f = (i - 1) + (int64_t)(n - 1) * j; else nb = 3LL * n + j; break;
      case 1: if (i <= n - 2) f = i + (int64_t)(n - 1) * j; else nb = (int64_t)n + j; break;
      case 2: if (j >= 1) f = nv + i + (int64_t)n * (j - 1); else nb = i; break;
      default: if (j <= n - 2) f = nv + i + (int64_t)n * j; else nb = 2LL * n + i; break;
    }
    out[idx] = f >= 0 ? lam[f * P + c] : (lam_bd ? lam_bd[nb * P + c] : 0.0);
  }
}

// out = (D + K G)^{-1} in (both [P2] in LDS; tmp [P2] LDS scratch)
template <int P>
__device__ void elem_zsolve(const ElemRef<P>& R, double kap, const double* in, double* tmp, double* out) {
  constexpr int P2 = P * P;
  for (int q = threadIdx.x; q < P2; q += 64) {
    double s = 0.0;
    for (int I = 0; I < P2; ++I) s += R.V[I * P2 + q] * in[I];
    tmp[q] = s / (R.delta[q] + kap * R.mu[q]);
  }
  __syncthreads();
  for (int I = threadIdx.x; I < P2; I += 64) {
    double s = 0.0;
    for (int q = 0; q < P2; ++q) s += R.V[I * P2 + q] * tmp[q];
    out[I] = s;
  }
  __syncthreads();
}

// out[I] = in0[I] - sum_c (E - K H)[I][c] lam[c]
template <int P>
__device__ void elem_rhs(const ElemRef<P>& R, double kap, const double* in0, const double* lam, double* out) {
  constexpr int P2 = P * P, F4 = 4 * P;
  for (int I = threadIdx.x; I < P2; I += 64) {
    double s = in0[I];
    for (int c = 0; c < F4; ++c) s -= (R.E[I * F4 + c] - kap * R.H[I * F4 + c]) * lam[c];
    out[I] = s;
  }
  __syncthreads();
}

template <int P>
__global__ __launch_bounds__(64) void k_elem_reconstruct(ElemArgs a) {
  constexpr int P2 = P * P, F4 = 4 * P;
  __shared__ double lam[F4], F[P2], t[P2], tmp[P2], U[P2], s[2 * P2];
  const ElemRef<P> R(a.ref);
  const int64_t e = blockIdx.x;
  const int i = (int)(e % a.n), j = (int)(e / a.n);
  const double kap = a.kappa[e];
  elem_trace<P>(a.lam, a.lam_bd, a.n, i, j, lam);
  for (int I = threadIdx.x; I < P2; I += 64) F[I] = a.F[e * P2 + I];
  __syncthreads();
  elem_rhs<P>(R, kap, F, lam, t);
  elem_zsolve<P>(R, kap, t, tmp, U);
  for (int I = threadIdx.x; I < P2; I += 64) a.Uout[e * P2 + I] = U[I];
  if (a.Qout) {
    for (int r = threadIdx.x; r < 2 * P2; r += 64) {
      double v = 0.0;
      for (int J = 0; J < P2; ++J) v += R.Bt[r * P2 + J] * U[J];
      for (int c = 0; c < F4; ++c) v -= R.C[r * F4 + c] * lam[c];
      s[r] = v;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < 2 * P2; r += 64) {
      const int half = r / P2, I = r - half * P2;
      double v = 0.0;
      for (int J = 0; J < P2; ++J) v += R.Mvinv[I * P2 + J] * s[half * P2 + J];
      a.Qout[e * 2 * P2 + r] = kap * v;
    }
  }
}

template <int P>
__global__ __launch_bounds__(64) void k_elem_adjoint(ElemArgs a) {
  constexpr int P2 = P * P, F4 = 4 * P;
  __shared__ double r[P2], tmp[P2], z[P2];
  const ElemRef<P> R(a.ref);
  const int64_t e = blockIdx.x;
  const double kap = a.kappa[e];
  double sq = 0.0;
  for (int I = threadIdx.x; I < P2; I += 64) {
    const double v = a.U[e * P2 + I] - a.Uobs[e * P2 + I];
    r[I] = v;
    sq += v * v;
  }
  for (int off = 32; off >= 1; off >>= 1) sq += __shfl_xor(sq, off, 64);
  if (threadIdx.x == 0) a.misfit[e] = 0.5 * sq;
  __syncthreads();
  elem_zsolve<P>(R, kap, r, tmp, z);
  for (int c = threadIdx.x; c < F4; c += 64) {
    double v = 0.0;
    for (int I = 0; I < P2; ++I) v += (R.E[I * F4 + c] - kap * R.H[I * F4 + c]) * z[I];
    a.tout[e * F4 + c] = -v;
  }
}

template <int P>
__global__ __launch_bounds__(64) void k_elem_gradient(ElemArgs a) {
  constexpr int P2 = P * P, F4 = 4 * P;
  __shared__ double lam[F4], mu[F4], r[P2], q1[P2], tmp[P2], w[P2], U[P2], s[2 * P2], v[2 * P2];
  const ElemRef<P> R(a.ref);
  const int64_t e = blockIdx.x;
  const int i = (int)(e % a.n), j = (int)(e / a.n);
  const double kap = a.kappa[e];
  elem_trace<P>(a.lam, a.lam_bd, a.n, i, j, lam);
  elem_trace<P>(a.mu, nullptr, a.n, i, j, mu);  // boundary traces are data: no adjoint there
  for (int I = threadIdx.x; I < P2; I += 64) {
    U[I] = a.U[e * P2 + I];
    r[I] = U[I] - a.Uobs[e * P2 + I];
  }
  __syncthreads();
  elem_rhs<P>(R, kap, r, mu, q1);
  elem_zsolve<P>(R, kap, q1, tmp, w);
  for (int row = threadIdx.x; row < 2 * P2; row += 64) {
    double cv = 0.0, cs = 0.0;
    for (int c = 0; c < F4; ++c) {
      cv += R.C[row * F4 + c] * mu[c];
      cs -= R.C[row * F4 + c] * lam[c];
    }
    for (int J = 0; J < P2; ++J) {
      cv -= R.Bt[row * P2 + J] * w[J];
      cs += R.Bt[row * P2 + J] * U[J];
    }
    v[row] = cv;
    s[row] = cs;
  }
  __syncthreads();
  double g = 0.0;
  for (int row = threadIdx.x; row < 2 * P2; row += 64) {
    const int half = row / P2, I = row - half * P2;
    double m = 0.0;
    for (int J = 0; J < P2; ++J) m += R.Mvinv[I * P2 + J] * s[half * P2 + J];
    g += v[row] * m;
  }
  for (int off = 32; off >= 1; off >>= 1) g += __shfl_xor(g, off, 64);
  if (threadIdx.x == 0) a.grad[e] = kap * g;
}

__global__ __launch_bounds__(kWG) void k_face_gather(const double* t, double* c, int n, int P) {
  const int64_t nv = (int64_t)n * (n - 1), nf = 2 * nv;
  const int64_t idx = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (idx >= nf * P) return;
  const int64_t f = idx / P;
  const int a = (int)(idx - f * P);
  int64_t lo, hi;
  int llo, lhi;
  if (f < nv) {
    const int64_t j = f / (n - 1), i = f - j * (n - 1) + 1;
    lo = (i - 1) + (int64_t)n * j;
    hi = i + (int64_t)n * j;
    llo = 1;
    lhi = 0;
  } else {
    const int64_t g = f - nv, j = g / n + 1, i = g - (j - 1) * n;
    lo = i + (int64_t)n * (j - 1);
    hi = i + (int64_t)n * j;
    llo = 3;
    lhi = 2;
  }
  c[idx] = t[lo * 4 * P + llo * P + a] + t[hi * 4 * P + lhi * P + a];
}

hipError_t launch_elem_reconstruct(int P, const ElemArgs& a, hipStream_t s) {
  HDG_DISPATCH_P(P, hipLaunchKernelGGL(k_elem_reconstruct<PP>, dim3((unsigned)((int64_t)a.n * a.n)), dim3(64), 0,
                                       s, a));
  return hipGetLastError();
}
hipError_t launch_elem_adjoint(int P, const ElemArgs& a, hipStream_t s) {
  HDG_DISPATCH_P(P, hipLaunchKernelGGL(k_elem_adjoint<PP>, dim3((unsigned)((int64_t)a.n * a.n)), dim3(64), 0, s,
                                       a));
  return hipGetLastError();
}
hipError_t launch_elem_gradient(int P, const ElemArgs& a, hipStream_t s) {
  HDG_DISPATCH_P(P, hipLaunchKernelGGL(k_elem_gradient<PP>, dim3((unsigned)((int64_t)a.n * a.n)), dim3(64), 0, s,
                                       a));
  return hipGetLastError();
}
hipError_t launch_face_gather(int P, const double* t, double* c, int n, hipStream_t s) {
  const int64_t tot = 2LL * n * (n - 1) * P;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_face_gather, grid_for(tot), dim3(kWG), 0, s, t, c, n, P);
  return hipGetLastError();
}

int reduce_grid(int64_t n) {
  int64_t g = (n + kWG * 4 - 1) / (kWG * 4);
  if (g > 1024) g = 1024;
  if (g < 1) g = 1;
  return (int)g;
}

// The dot-product kernels walk the vector with a grid stride; each round loads
// kDotRounds strides before adding any, so a thread has that many round trips in
// flight instead of one.  The additions keep index order, so the partials are the
// same as those of a one-stride loop.
constexpr int kDotRounds = 4;
__global__ __launch_bounds__(kWG) void k_dot_partials(const double* a, const double* b, int64_t n,
                                                      double* partial) {
  double s = 0.0;
  const int64_t st = (int64_t)gridDim.x * kWG;
  int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  for (; i + (kDotRounds - 1) * st < n; i += kDotRounds * st) {
    double av[kDotRounds], bv[kDotRounds];
#pragma unroll
    for (int u = 0; u < kDotRounds; ++u) {
      av[u] = a[i + u * st];
      bv[u] = b[i + u * st];
    }
#pragma unroll
    for (int u = 0; u < kDotRounds; ++u) s += av[u] * bv[u];
  }
  for (; i < n; i += st) s += a[i] * b[i];
  const double t = block_sum(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// Sums of np values by one workgroup in a fixed order: each thread keeps 8 loads
// in flight (8 running sums, added in order at the end), then a fixed tree.
// The summing kernels run one workgroup of kSumT threads (a fixed order again):
// a sum of 32K partials is then 4 rounds of 8 loads per thread instead of 16.
constexpr int kSumT = 1024;
__device__ __forceinline__ double thread_sum8_wide(const double* v, int np) {
  double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int i = threadIdx.x;
  for (; i + 7 * kSumT < np; i += 8 * kSumT) {
#pragma unroll
    for (int u = 0; u < 8; ++u) s[u] += v[i + u * kSumT];
  }
  for (; i < np; i += kSumT) s[0] += v[i];
  double t = 0.0;
#pragma unroll
  for (int u = 0; u < 8; ++u) t += s[u];
  return t;
}
// Deterministic sum over the kSumT threads (fixed shuffle tree, then the wave
// sums in order); valid in thread 0.  ws: kSumT / 64 shared slots.
__device__ __forceinline__ double block_sum_wide(double v, double* ws) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kSumT / 64; ++w) s += ws[w];
  return s;
}

__global__ __launch_bounds__(kSumT) void k_sum_partials(const double* partial, int np, double* out) {
  __shared__ double ws[kSumT / 64];
  const double t = block_sum_wide(thread_sum8_wide(partial, np), ws);
  if (threadIdx.x == 0) *out = t;
}

// Up to three dot products x_j . y_j in one pass (FP64 accumulation), partials
// of dot j at partial[j * gridDim.x + block].  Workgroup j of the summing
// kernel adds the partials of dot j.
template <typename T>
__global__ __launch_bounds__(kWG) void k_dots_partials(DotArgs a, int64_t n, double* partial) {
  double s[3] = {0.0, 0.0, 0.0};
  const int64_t st = (int64_t)gridDim.x * kWG;
  int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  for (; i + (kDotRounds - 1) * st < n; i += kDotRounds * st) {
    double xv[3][kDotRounds], yv[3][kDotRounds];
#pragma unroll
    for (int j = 0; j < 3; ++j)
      if (j < a.ndots)
#pragma unroll
        for (int u = 0; u < kDotRounds; ++u) {
          xv[j][u] = (double)static_cast<const T*>(a.x[j])[i + u * st];
          yv[j][u] = (double)static_cast<const T*>(a.y[j])[i + u * st];
        }
#pragma unroll
    for (int u = 0; u < kDotRounds; ++u)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        if (j < a.ndots) s[j] += xv[j][u] * yv[j][u];
  }
  for (; i < n; i += st)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      if (j < a.ndots) s[j] += (double)static_cast<const T*>(a.x[j])[i] * (double)static_cast<const T*>(a.y[j])[i];
  for (int j = 0; j < a.ndots; ++j) {
    const double t = block_sum(s[j]);
    if (threadIdx.x == 0) partial[(int64_t)j * gridDim.x + blockIdx.x] = t;
    __syncthreads();  // block_sum's shared slots are reused by the next dot
  }
}
__global__ __launch_bounds__(kSumT) void k_sum_partials_multi(const double* partial, int np, double* out) {
  __shared__ double ws[kSumT / 64];
  const double t = block_sum_wide(thread_sum8_wide(partial + (int64_t)blockIdx.x * np, np), ws);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_axpy(double alpha, const T* x, T* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i < n) y[i] += T(alpha) * x[i];
}
template <typename T>
__global__ __launch_bounds__(kWG) void k_xpby(const T* x, double beta, T* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i < n) y[i] = x[i] + T(beta) * y[i];
}
template <typename T>
__global__ __launch_bounds__(kWG) void k_fill_t(T v, T* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i < n) y[i] = v;
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
template <typename T>
__global__ __launch_bounds__(kWG) void k_copy(const T* x, T* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i < n) y[i] = x[i];
}
__global__ __launch_bounds__(kWG) void k_fill(double v, double* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i < n) y[i] = v;
}
__global__ __launch_bounds__(kWG) void k_to_f32(const double* x, float* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i < n) y[i] = (float)x[i];
}
__global__ __launch_bounds__(kWG) void k_to_f64(const float* x, double* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i < n) y[i] = (double)x[i];
}

hipError_t launch_dot_partials(const double* a, const double* b, int64_t n, double* partial, hipStream_t s) {
  hipLaunchKernelGGL(k_dot_partials, dim3(reduce_grid(n)), dim3(kWG), 0, s, a, b, n, partial);
  return hipGetLastError();
}
hipError_t launch_sum_partials(const double* partial, int np, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kSumT), 0, s, partial, np, out);
  return hipGetLastError();
}
hipError_t launch_dots(Prec pr, const DotArgs& a, int64_t n, double* partial, hipStream_t s) {
  if (a.ndots < 1 || a.ndots > 3) return hipErrorInvalidValue;
  HDG_DISPATCH_T(pr, hipLaunchKernelGGL(k_dots_partials<TT>, dim3(reduce_grid(n)), dim3(kWG), 0, s, a, n,
                                        partial));
  return hipGetLastError();
}
hipError_t launch_sum_partials_multi(const double* partial, int np, int ndots, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_partials_multi, dim3(ndots), dim3(kSumT), 0, s, partial, np, out);
  return hipGetLastError();
}
hipError_t launch_axpy(double alpha, const double* x, double* y, int64_t n, hipStream_t s) {
  return launch_axpy(Prec::F64, alpha, x, y, n, s);
}
hipError_t launch_xpby(const double* x, double beta, double* y, int64_t n, hipStream_t s) {
  return launch_xpby(Prec::F64, x, beta, y, n, s);
}
hipError_t launch_axpy(Prec pr, double alpha, const void* x, void* y, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  HDG_DISPATCH_T(pr, hipLaunchKernelGGL(k_axpy<TT>, grid_for(n), dim3(kWG), 0, s, alpha, (const TT*)x, (TT*)y, n));
  return hipGetLastError();
}
hipError_t launch_xpby(Prec pr, const void* x, double beta, void* y, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  HDG_DISPATCH_T(pr, hipLaunchKernelGGL(k_xpby<TT>, grid_for(n), dim3(kWG), 0, s, (const TT*)x, beta, (TT*)y, n));
  return hipGetLastError();
}
__device__ __forceinline__ double ratio_or_zero(double a, double b) {
  const double r = a / b;
  return (b > 0.0 && isfinite(r)) ? r : 0.0;
}
template <typename T>
__global__ __launch_bounds__(kWG) void k_axpy_dev(const double* sc, int num, int den, double sign, const T* x,
                                                  T* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i < n) y[i] += T(sign * ratio_or_zero(sc[num], sc[den])) * x[i];
}
// The end of a flexible CG step: e += alpha d and (r != null) r -= alpha q,
// alpha = sc[0] / sc[1], in one pass (the same operations as two k_axpy_dev).
template <typename T>
__global__ __launch_bounds__(kWG) void k_fcg_update(const double* sc, const T* d, T* e, const T* q, T* r, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i >= n) return;
  const double al = ratio_or_zero(sc[0], sc[1]);
  e[i] += T(1.0 * al) * d[i];
  if (r) r[i] += T(-1.0 * al) * q[i];
}
template <typename T>
__global__ __launch_bounds__(kWG) void k_xpby_dev(const T* x, const double* sc, int num, int den, double sign,
                                                  T* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i < n) y[i] = x[i] + T(sign * ratio_or_zero(sc[num], sc[den])) * y[i];
}
__global__ void k_fcg_scalars(double* sc) {
  if (threadIdx.x == 0) sc[0] = sc[3] - ratio_or_zero(sc[2], sc[1]) * sc[4];
}
// The three dot products of a flexible CG step (partials of dot j at
// partial[j np ...]) summed by one workgroup into sc[2], sc[3], sc[4], and then
// sc[0] = sc[3] - (sc[2] / sc[1]) sc[4] as k_fcg_scalars: one launch for both.
__global__ __launch_bounds__(kSumT) void k_sum_partials_fcg(const double* partial, int np, double* sc) {
  __shared__ double ws[kSumT / 64];
  double t[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    t[j] = block_sum_wide(thread_sum8_wide(partial + (int64_t)j * np, np), ws);
    __syncthreads();  // the shared slots are reused by the next dot
  }
  if (threadIdx.x == 0) {
    sc[2] = t[0];
    sc[3] = t[1];
    sc[4] = t[2];
    sc[0] = t[1] - ratio_or_zero(t[0], sc[1]) * t[2];
  }
}
hipError_t launch_axpy_dev(Prec pr, const double* sc, int num, int den, double sign, const void* x, void* y,
                           int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  HDG_DISPATCH_T(pr, hipLaunchKernelGGL(k_axpy_dev<TT>, grid_for(n), dim3(kWG), 0, s, sc, num, den, sign,
                                        (const TT*)x, (TT*)y, n));
  return hipGetLastError();
}
hipError_t launch_xpby_dev(Prec pr, const void* x, const double* sc, int num, int den, double sign, void* y,
                           int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  HDG_DISPATCH_T(pr, hipLaunchKernelGGL(k_xpby_dev<TT>, grid_for(n), dim3(kWG), 0, s, (const TT*)x, sc, num, den,
                                        sign, (TT*)y, n));
  return hipGetLastError();
}
hipError_t launch_fcg_update(Prec pr, const double* sc, const void* d, void* e, const void* q, void* r, int64_t n,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  HDG_DISPATCH_T(pr, hipLaunchKernelGGL(k_fcg_update<TT>, grid_for(n), dim3(kWG), 0, s, sc, (const TT*)d, (TT*)e,
                                        (const TT*)q, (TT*)r, n));
  return hipGetLastError();
}
hipError_t launch_fcg_scalars(double* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_fcg_scalars, dim3(1), dim3(64), 0, s, sc);
  return hipGetLastError();
}
hipError_t launch_sum_partials_fcg(const double* partial, int np, double* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_partials_fcg, dim3(1), dim3(kSumT), 0, s, partial, np, sc);
  return hipGetLastError();
}

hipError_t launch_zero(Prec pr, void* y, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  HDG_DISPATCH_T(pr, hipLaunchKernelGGL(k_fill_t<TT>, grid_for(n), dim3(kWG), 0, s, TT(0), (TT*)y, n));
  return hipGetLastError();
}
hipError_t launch_axpy_norm(double alpha, const double* q, double* r, int64_t n, double* partial,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_norm, dim3(reduce_grid(n)), dim3(kWG), 0, s, alpha, q, r, n, partial);
  return hipGetLastError();
}
hipError_t launch_copy(Prec pr, const void* x, void* y, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  HDG_DISPATCH_T(pr, hipLaunchKernelGGL(k_copy<TT>, grid_for(n), dim3(kWG), 0, s, (const TT*)x, (TT*)y, n));
  return hipGetLastError();
}
hipError_t launch_fill(double v, double* y, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, grid_for(n), dim3(kWG), 0, s, v, y, n);
  return hipGetLastError();
}
hipError_t launch_to_f32(const double* x, float* y, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_f32, grid_for(n), dim3(kWG), 0, s, x, y, n);
  return hipGetLastError();
}
hipError_t launch_to_f64(const float* x, double* y, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_f64, grid_for(n), dim3(kWG), 0, s, x, y, n);
  return hipGetLastError();
}

}  // namespace hdg
