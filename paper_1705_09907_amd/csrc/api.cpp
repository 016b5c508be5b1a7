// C ABI of the HDG trace-operator library: setup, operator, smoothers,
// transfers, V-cycle and solvers (Secs. 3, 6-8 of arXiv:1705.09907).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/hdggmg.h"
#include "kernels.hpp"
#include "setup.hpp"

using hdg::Vec;

namespace {

// Device data of a p-level.  `slab`, `dinv` (matrix precision `mp`), `chain`,
// `pmat` and the work vectors (vector precision) belong to the cycle; `slab64`
// holds FP64 blocks where the FP64 operator is kept (every level in FP64 mode,
// the finest level otherwise; it aliases `slab` in FP64 mode).
struct PLevel {
  int p = 0, P = 1;
  int64_t N = 0;
  hdg::Prec mp = hdg::Prec::F64;  // storage precision of slab / dinv in the cycle
  void* slab = nullptr;
  double* slab64 = nullptr;
  void* dinv = nullptr;                                           // facet Schwarz
  void* chain = nullptr;                                          // chain Schwarz factors
  void* tri = nullptr;                                            // P = 1: partitioned chain solve factors
  void* pslab = nullptr;                                          // element-patch Schwarz inverses (slab layout)
  int64_t cstride = 0;
  void* pmat = nullptr;                                           // P_p (p >= 1)
  double* pmat64 = nullptr;
  double omega = 0.8;
  void *x = nullptr, *b = nullptr, *r = nullptr, *t = nullptr;
  int chain_lds_level = 64;                           // chain factors of levels >= this are staged in LDS
  int chain_threads = 0;                              // chain launch shape (0: chain_threads default)
  int chain_remap = -1;                               // -1: chain_remap default
  int chain_shape = 0;                                // launch shape (ChainArgs::shape; 0: by the mesh)
  int inner = 0;                                      // K-cycle: FCG steps of this level's correction
  void *kz = nullptr, *kd = nullptr, *kq = nullptr;   // K-cycle work vectors
};

struct QLevel {
  int m = 0;
  int64_t Nv = 0;
  bool coarsest = false;
  void* st = nullptr;
  void* dinv = nullptr;
  double* inv = nullptr;   // coarsest level: FP64 dense inverse
  double lmax = 0.0;
  void *x = nullptr, *b = nullptr, *r = nullptr, *d = nullptr, *t = nullptr;
};

// Work vectors of the solve for many right-hand sides, [rows][R]: per p-level
// x, b, r in the cycle precision; per Q1 level x, b, r, d, t; FP64 outer
// vectors; per-column device scalars.  Allocated for one R at a time.
struct MultiWork {
  int R = 0;
  std::vector<void*> px, pb, pr;
  std::vector<void*> qx, qb, qr, qd, qt;
  double *vr = nullptr, *vz = nullptr, *vd = nullptr, *vq = nullptr;
  void *cva = nullptr, *cvb = nullptr;
  double *sc = nullptr, *nrm = nullptr, *nb = nullptr, *act = nullptr, *partial = nullptr;
  std::vector<int> rc;   // chain solve: columns per workgroup, per p-level (autotuned)
  std::vector<int> mk;   // multi apply kernel per p-level (MultiArgs::kernel), cycle precision
  std::vector<void*> allocs;
  ~MultiWork() {
    for (void* q : allocs) (void)hipFree(q);
  }
};

}  // namespace

struct hdg_ctx {
  hdg_config_t cfg{};
  hipStream_t stream = nullptr;
  std::string err;
  int n = 0, k = 0;
  int64_t nf = 0, ntiles = 0;
  std::vector<double> kappa;
  std::vector<PLevel> pl;      // index = p
  std::vector<QLevel> ql;
  std::vector<void*> allocs;
  double* partial = nullptr;
  int npartial = 0;
  double* scal = nullptr;      // device scalars [4]
  double* scal_h = nullptr;    // pinned host scalars [4]
  double *vr = nullptr, *vz = nullptr, *vd = nullptr, *vq = nullptr;  // solver vectors (FP64)
  void *cva = nullptr, *cvb = nullptr;  // cycle-precision copies of FP64 vectors (size N(k))
  hipEvent_t ev0 = nullptr, ev1 = nullptr;  // timed apply
  double* dsc = nullptr;                    // device scalars of the K-cycle (8 per p-level)
  hipStream_t cap_stream = nullptr;         // capture of the preconditioner as a HIP graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hdg::BatchMesh* batch_dev = nullptr;      // descriptor table of hdg_apply_trace_operator_batch
  int batch_cap = 0;
  std::vector<hdg::BatchMesh> batch_host;
  void* batch_scratch = nullptr;            // device address of the allocation-free descriptor table
  // misfit gradient: degree-k reference pack, coefficients, and the source state
  // of the last hdg_assemble_rhs (load vectors, boundary traces)
  double *ref_dev = nullptr, *kappa_dev = nullptr, *F_dev = nullptr, *lambd_dev = nullptr;
  double *elem_t = nullptr, *elem_m = nullptr;
  bool have_source = false;
  hdg::Prec prec = hdg::Prec::F64;      // precision of the multigrid cycle
  int nq = 0;
  int64_t lds_cap = 65536;              // LDS bytes per workgroup on this device
  std::unique_ptr<MultiWork> mw;        // solve for many right-hand sides
  std::map<int64_t, int> multi_pick;    // multi apply kernel per (level, columns), cycle precision

  hdg_ctx() = default;
  hdg_ctx(const hdg_ctx&) = delete;
  hdg_ctx& operator=(const hdg_ctx&) = delete;
  // Releases every resource, also after a failed hdg_create: work still queued
  // on the stream finishes first.
  ~hdg_ctx() {
    const bool on_device = !allocs.empty() || mw || graph_exec || cap_stream || ev0 || scal_h;
    if (on_device) (void)hipStreamSynchronize(stream);  // a rejected config made no device call
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    mw.reset();
    for (void* q : allocs) (void)hipFree(q);
    if (scal_h) (void)hipHostFree(scal_h);
  }
};

namespace {

struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct ArgError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

inline void hipchk(hipError_t e, const char* what) {
  if (e != hipSuccess) throw HipError(std::string(what) + ": " + hipGetErrorString(e));
}

void* balloc(hdg_ctx* h, size_t bytes) {
  void* p = nullptr;
  if (bytes == 0) bytes = 16;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    throw std::bad_alloc();
  }
  h->allocs.push_back(p);
  return p;
}
double* dalloc(hdg_ctx* h, int64_t n) { return (double*)balloc(h, (size_t)std::max<int64_t>(n, 1) * 8); }
void* valloc(hdg_ctx* h, int64_t n) { return balloc(h, (size_t)std::max<int64_t>(n, 1) * hdg::vec_bytes(h->prec)); }

double* upload(hdg_ctx* h, const Vec& v) {
  double* d = dalloc(h, (int64_t)v.size());
  hipchk(hipMemcpy(d, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice), "upload");
  return d;
}

// bfloat16 of x: round to nearest even on the FP32 bits
inline uint16_t to_bf16(double x) {
  float f = (float)x;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Upload host FP64 data converted to `bytes_per` = 8 (FP64), 4 (FP32) or 2 (BF16).
void* upload_as(hdg_ctx* h, const Vec& v, size_t bytes_per) {
  if (bytes_per == 8) return upload(h, v);
  void* d = balloc(h, v.size() * bytes_per);
  if (bytes_per == 4) {
    std::vector<float> t(v.size());
    for (size_t i = 0; i < v.size(); ++i) t[i] = (float)v[i];
    hipchk(hipMemcpy(d, t.data(), t.size() * 4, hipMemcpyHostToDevice), "upload f32");
  } else {
    std::vector<uint16_t> t(v.size());
    for (size_t i = 0; i < v.size(); ++i) t[i] = to_bf16(v[i]);
    hipchk(hipMemcpy(d, t.data(), t.size() * 2, hipMemcpyHostToDevice), "upload bf16");
  }
  return d;
}
void* upload_vec(hdg_ctx* h, const Vec& v) { return upload_as(h, v, hdg::vec_bytes(h->prec)); }

template <typename F>
hdg_status_t guarded(hdg_ctx* h, F&& body) {
  try {
    return body();
  } catch (const ArgError& e) {
    if (h) h->err = e.what();
    return HDG_ERR_INVALID_ARG;
  } catch (const HipError& e) {
    if (h) h->err = e.what();
    return HDG_ERR_HIP;
  } catch (const std::bad_alloc&) {
    if (h) h->err = "allocation failed";
    return HDG_ERR_OOM;
  } catch (const std::exception& e) {
    if (h) h->err = e.what();
    return HDG_ERR_STATE;
  }
}

// Interleaved device layout of per-face data with NE entries per face and V
// entries per 16-byte load: entry e of face f at ((tile NQ + e/V) 64 + lane) V + e%V,
// NQ = ceil(NE / V), tile = f / 64, lane = f % 64.  Packs canonical host data
// fb[f NE + e] (FP64) into that layout and uploads it in the requested precision.
void* pack_faces(hdg_ctx* h, const Vec& fb, int NE, hdg::Prec pr) {
  const int V = hdg::mat_lanes16(pr);
  const int64_t NQ = (NE + V - 1) / V;
  Vec dev((size_t)(h->ntiles * NQ * 64 * V), 0.0);
  hdg::parallel_for(h->nf, [&](int64_t f0, int64_t f1) {
    for (int64_t f = f0; f < f1; ++f) {
      const int64_t tile = f >> 6, lane = f & 63;
      for (int e = 0; e < NE; ++e)
        dev[(size_t)(((tile * NQ + e / V) * 64 + lane) * V + e % V)] = fb[(size_t)f * NE + e];
    }
  });
  return upload_as(h, dev, hdg::mat_bytes(pr));
}

// ------------------------------------------------------- element blocks, host
// All condensed blocks of level k, [n*n][4P][4P].
Vec blocks_finest(hdg_ctx* h, int p) {
  const int P = p + 1, F4 = 4 * P, P2 = P * P;
  hdg::RefDegree ref;
  ref.build(p, 1.0 / h->n, h->cfg.tau);
  const int64_t ne = (int64_t)h->n * h->n;
  Vec out((size_t)ne * F4 * F4);
  hdg::parallel_for(ne, [&](int64_t a, int64_t b) {
    Vec work((size_t)P2 * P2 + (size_t)P2 * F4);
    for (int64_t e = a; e < b; ++e)
      hdg::element_block(ref, h->kappa[e], out.data() + (size_t)e * F4 * F4, work.data());
  });
  return out;
}

Vec blocks_galerkin(hdg_ctx* h, int p_fine, const Vec& fine) {
  const Vec Pp = hdg::p_prolongation(p_fine);
  const int Ff = 4 * (p_fine + 1), Fc = 4 * p_fine;
  const int64_t ne = (int64_t)h->n * h->n;
  Vec out((size_t)ne * Fc * Fc);
  hdg::parallel_for(ne, [&](int64_t a, int64_t b) {
    for (int64_t e = a; e < b; ++e)
      hdg::galerkin_block(Pp, p_fine, fine.data() + (size_t)e * Ff * Ff, out.data() + (size_t)e * Fc * Fc);
  });
  return out;
}

// block (P x P) of the element block coupling local faces (lr, lc)
inline double blk(const double* K, int P, int lr, int lc, int a, int c) {
  return K[(size_t)(lr * P + a) * 4 * P + lc * P + c];
}

// Face-major 7-block layout, summed diagonal blocks, and the facet inverses.
void build_face_data(hdg_ctx* h, PLevel& L, const Vec& blocks) {
  const int n = h->n, P = L.P, P2 = P * P, F4 = 4 * P, NE = 7 * P2;
  const int64_t nf = h->nf;
  Vec slab((size_t)nf * NE, 0.0);   // canonical: slab[f NE + e]
  const bool face = h->cfg.smoother == HDG_SMOOTH_FACE;
  Vec dinv(face ? (size_t)nf * P2 : 0, 0.0);
  Vec diag(h->cfg.smoother == HDG_SMOOTH_CHAIN ? (size_t)nf * P2 : 0, 0.0);
  auto tp_index = [NE](int64_t f, int e, int) { return (size_t)f * NE + e; };
  hdg::parallel_for(nf, [&](int64_t a0, int64_t a1) {
    Vec D(P2);
    for (int64_t f = a0; f < a1; ++f) {
      int64_t lo, hi;
      int llo, lhi;
      hdg::face_elements(n, f, lo, hi, llo, lhi);
      const double* Klo = blocks.data() + (size_t)lo * F4 * F4;
      const double* Khi = blocks.data() + (size_t)hi * F4 * F4;
      const int ilo = (int)(lo % n), jlo = (int)(lo / n), ihi = (int)(hi % n), jhi = (int)(hi / n);
      int olo[3], ohi[3];
      hdg::other_faces(llo, olo);
      hdg::other_faces(lhi, ohi);
      for (int a = 0; a < P; ++a)
        for (int c = 0; c < P; ++c) {
          D[a * P + c] = blk(Klo, P, llo, llo, a, c) + blk(Khi, P, lhi, lhi, a, c);
          slab[tp_index(f, a * P + c, NE)] = D[a * P + c];
          for (int s = 0; s < 3; ++s) {
            const bool in_lo = hdg::element_face(n, ilo, jlo, olo[s]) >= 0;
            const bool in_hi = hdg::element_face(n, ihi, jhi, ohi[s]) >= 0;
            slab[tp_index(f, (1 + s) * P2 + a * P + c, NE)] = in_lo ? blk(Klo, P, llo, olo[s], a, c) : 0.0;
            slab[tp_index(f, (4 + s) * P2 + a * P + c, NE)] = in_hi ? blk(Khi, P, lhi, ohi[s], a, c) : 0.0;
          }
        }
      if (face) {
        Vec Di(D);
        if (!hdg::cholesky_inverse(P, Di)) throw std::runtime_error("face block not SPD");
        for (int e = 0; e < P2; ++e) dinv[(size_t)f * P2 + e] = Di[e];
      } else {
        std::copy(D.begin(), D.end(), diag.begin() + (size_t)f * P2);
      }
    }
  });
  // bfloat16 storage is used on the coarse p-levels only: the finest level's
  // residual of a smooth correction cancels far below bfloat16 resolution
  // (measured: the preconditioner diverges at lognormal sigma = 2), so it keeps FP32.
  L.mp = (h->prec == hdg::Prec::BF16 && L.p == h->k) ? hdg::Prec::F32 : h->prec;
  L.slab = pack_faces(h, slab, NE, L.mp);
  if (h->prec == hdg::Prec::F64) L.slab64 = static_cast<double*>(L.slab);
  else if (L.p == h->k) L.slab64 = static_cast<double*>(pack_faces(h, slab, NE, hdg::Prec::F64));
  if (face) {
    L.dinv = pack_faces(h, dinv, P2, L.mp);
    return;
  }
  // chain Schwarz: block cyclic reduction factors of every chain of faces
  // (the chain matrices are SPD principal submatrices of S, so every pivot
  // block met by the reduction is SPD).  Only the odd positions' records
  // [Dinv, W = Dinv A, Z = Dinv C] are stored: by the symmetry of every reduced
  // matrix (A_j = C_{j-1}^T), the even positions' multipliers are
  // M-_j = A_j Dinv_{j-1} = Z_{j-1}^T and M+_j = C_j Dinv_{j+1} = W_{j+1}^T.
  const int64_t nch = 2LL * n, nv = (int64_t)n * (n - 1);
  const int m = n - 1;
  std::vector<int> msz;
  for (int ml = m;; ml = (ml + 1) / 2) {
    msz.push_back(ml);
    if (ml == 1) break;
  }
  std::vector<int64_t> loff;  // per-level offset (doubles) of the factor records
  int64_t tot = 0;
  for (int s : msz) {
    loff.push_back(tot);
    tot += s == 1 ? (int64_t)P2 : (int64_t)3 * P2 * (s / 2);
  }
  L.cstride = tot;
  Vec fac((size_t)(nch * L.cstride), 0.0);
  auto mul = [P](const double* X, const double* Y, double* Z) {  // Z = X Y
    for (int a = 0; a < P; ++a)
      for (int b = 0; b < P; ++b) {
        double s = 0.0;
        for (int q = 0; q < P; ++q) s += X[a * P + q] * Y[q * P + b];
        Z[a * P + b] = s;
      }
  };
  hdg::parallel_for(nch, [&](int64_t c0, int64_t c1) {
    Vec T(P2);
    for (int64_t c = c0; c < c1; ++c) {
      const bool vert = c < n;
      const int64_t base = vert ? c * (n - 1) : nv + (c - n);
      const int64_t stride = vert ? 1 : n;
      const int sub = vert ? 1 : 3, sup = vert ? 4 : 6;  // slots coupling to previous / next face
      Vec A((size_t)m * P2, 0.0), D((size_t)m * P2), C((size_t)m * P2, 0.0);
      for (int i = 0; i < m; ++i) {
        const int64_t f = base + stride * i;
        for (int e = 0; e < P2; ++e) {
          D[(size_t)i * P2 + e] = diag[(size_t)f * P2 + e];
          if (i >= 1) A[(size_t)i * P2 + e] = slab[tp_index(f, sub * P2 + e, NE)];
          if (i + 1 < m) C[(size_t)i * P2 + e] = slab[tp_index(f, sup * P2 + e, NE)];
        }
      }
      double* rec = fac.data() + (size_t)c * L.cstride;
      for (size_t lv = 0; lv < msz.size(); ++lv) {
        const int ml = msz[lv];
        double* lvl = rec + loff[lv];
        if (ml == 1) {
          Vec Di(D.begin(), D.begin() + P2);
          if (!hdg::cholesky_inverse(P, Di)) throw std::runtime_error("chain pivot block not SPD");
          std::copy(Di.begin(), Di.end(), lvl);
          break;
        }
        const int no = ml / 2;
        double* odd = lvl;
        Vec Dinv((size_t)ml * P2, 0.0);
        for (int j = 1; j < ml; j += 2) {
          Vec Di(D.begin() + (size_t)j * P2, D.begin() + (size_t)(j + 1) * P2);
          if (!hdg::cholesky_inverse(P, Di)) throw std::runtime_error("chain pivot block not SPD");
          std::copy(Di.begin(), Di.end(), Dinv.begin() + (size_t)j * P2);
          const int o = j / 2;
          Vec W(P2), Z(P2);  // Dinv A, Dinv C
          mul(Di.data(), A.data() + (size_t)j * P2, W.data());
          mul(Di.data(), C.data() + (size_t)j * P2, Z.data());
          for (int e = 0; e < P2; ++e) {
            odd[(size_t)e * no + o] = Di[e];
            odd[(size_t)(P2 + e) * no + o] = W[e];
            odd[(size_t)(2 * P2 + e) * no + o] = Z[e];
          }
        }
        const int mn = (ml + 1) / 2;
        Vec An((size_t)mn * P2, 0.0), Dn((size_t)mn * P2), Cn((size_t)mn * P2, 0.0);
        Vec Mm(P2), Mp(P2);
        for (int j = 0; j < ml; j += 2) {
          std::fill(Mm.begin(), Mm.end(), 0.0);
          std::fill(Mp.begin(), Mp.end(), 0.0);
          double* Dj = Dn.data() + (size_t)(j / 2) * P2;
          std::copy(D.begin() + (size_t)j * P2, D.begin() + (size_t)(j + 1) * P2, Dj);
          if (j >= 1) {
            mul(A.data() + (size_t)j * P2, Dinv.data() + (size_t)(j - 1) * P2, Mm.data());
            mul(Mm.data(), C.data() + (size_t)(j - 1) * P2, T.data());
            for (int e = 0; e < P2; ++e) Dj[e] -= T[e];
            mul(Mm.data(), A.data() + (size_t)(j - 1) * P2, T.data());
            for (int e = 0; e < P2; ++e) An[(size_t)(j / 2) * P2 + e] = -T[e];
          }
          if (j + 1 < ml) {
            mul(C.data() + (size_t)j * P2, Dinv.data() + (size_t)(j + 1) * P2, Mp.data());
            mul(Mp.data(), A.data() + (size_t)(j + 1) * P2, T.data());
            for (int e = 0; e < P2; ++e) Dj[e] -= T[e];
            mul(Mp.data(), C.data() + (size_t)(j + 1) * P2, T.data());
            for (int e = 0; e < P2; ++e) Cn[(size_t)(j / 2) * P2 + e] = -T[e];
          }
        }
        A.swap(An);
        D.swap(Dn);
        C.swap(Cn);
      }
    }
  });
  L.chain = upload_vec(h, fac);
  if (P == 1 && hdg::chain_tri_lmax(n) > 0) {
    // the partitioned solve's factors come from the same device routine as in
    // the device set-up, on a temporary copy of these blocks
    L.tri = valloc(h, nch * hdg::chain_tri_stride(n));
    void* tmp = nullptr;
    const size_t eb_bytes = blocks.size() * sizeof(double);
    if (hipMalloc(&tmp, eb_bytes + 256) != hipSuccess) {
      (void)hipGetLastError();
      throw std::bad_alloc();
    }
    int* dfail = reinterpret_cast<int*>(static_cast<char*>(tmp) + eb_bytes);
    int failed = 0;
    hipError_t e = hipMemcpy(tmp, blocks.data(), eb_bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(dfail, 0, sizeof(int));
    if (e == hipSuccess)
      e = hdg::launch_chain_tri_factor(h->prec, static_cast<const double*>(tmp), n, L.tri, dfail, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) e = hipMemcpy(&failed, dfail, sizeof(int), hipMemcpyDeviceToHost);
    (void)hipFree(tmp);
    hipchk(e, "partitioned chain factors");
    if (failed) throw std::runtime_error("a chain pivot is not positive");
  }
  // stage the small levels' factors in LDS: at most 8 KiB beside the chain
  const size_t es = hdg::vec_bytes(h->prec);
  const int64_t rhs_bytes = (int64_t)(n - 1) * P * (int64_t)es;
  L.chain_lds_level = hdg::chain_lds_level(P, n, es, std::min<int64_t>(8192, h->lds_cap - rhs_bytes));
}

// Q1 stencil of P_J^T S0 P_J from the p = 0 element blocks (4 x 4).
Vec q1_from_p0(hdg_ctx* h, const Vec& b0) {
  const int n = h->n;
  const int64_t Nv = (int64_t)(n - 1) * (n - 1);
  Vec st((size_t)9 * Nv, 0.0);
  auto vid = [n](int i, int j) -> int64_t {
    if (i <= 0 || j <= 0 || i >= n || j >= n) return -1;
    return (int64_t)(i - 1) + (int64_t)(n - 1) * (j - 1);
  };
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      const double* K = b0.data() + (size_t)(i + (int64_t)n * j) * 16;
      // local faces l, r, b, t and their end vertices
      const int ends[4][2][2] = {{{i, j}, {i, j + 1}}, {{i + 1, j}, {i + 1, j + 1}},
                                 {{i, j}, {i + 1, j}}, {{i, j + 1}, {i + 1, j + 1}}};
      bool interior[4];
      for (int lf = 0; lf < 4; ++lf) interior[lf] = hdg::element_face(n, i, j, lf) >= 0;
      for (int f1 = 0; f1 < 4; ++f1) {
        if (!interior[f1]) continue;
        for (int f2 = 0; f2 < 4; ++f2) {
          if (!interior[f2]) continue;
          const double kv = K[f1 * 4 + f2];
          for (int a = 0; a < 2; ++a) {
            const int vi = ends[f1][a][0], vj = ends[f1][a][1];
            const int64_t v = vid(vi, vj);
            if (v < 0) continue;
            for (int b = 0; b < 2; ++b) {
              const int wi = ends[f2][b][0], wj = ends[f2][b][1];
              if (vid(wi, wj) < 0) continue;
              const int s = (wi - vi + 1) + 3 * (wj - vj + 1);
              st[(size_t)s * Nv + v] += 0.25 * kv;
            }
          }
        }
      }
    }
  return st;
}

// The coarsest Q1 level: dense Cholesky inverse of its matrix A (host), uploaded
// (update: into the existing buffer).
void coarsest_level(hdg_ctx* h, QLevel& Q, const hdg::Csr& A, bool update) {
  if (Q.Nv > 20000) throw ArgError("coarsest Q1 level too large; use a mesh size with more factors of 2");
  Q.coarsest = true;
  Vec dense((size_t)Q.Nv * Q.Nv, 0.0);
  for (int64_t r = 0; r < A.nrows; ++r)
    for (int64_t kk = A.ptr[r]; kk < A.ptr[r + 1]; ++kk) dense[(size_t)r * Q.Nv + A.col[kk]] = A.val[kk];
  if (!hdg::cholesky_inverse((int)Q.Nv, dense)) throw std::runtime_error("coarsest Q1 matrix not SPD");
  if (update) {
    hipchk(hipMemcpy(Q.inv, dense.data(), dense.size() * sizeof(double), hipMemcpyHostToDevice), "upload");
    return;
  }
  Q.inv = upload(h, dense);
  Q.x = valloc(h, Q.Nv);
  Q.b = valloc(h, Q.Nv);
}

void build_hlevels(hdg_ctx* h, const Vec& b0) {
  Vec st = q1_from_p0(h, b0);
  int m = h->n;
  int lev = 0;
  while (true) {
    QLevel Q;
    Q.m = m;
    Q.Nv = (int64_t)(m - 1) * (m - 1);
    hdg::Csr A = hdg::stencil_to_csr(m, st);
    const bool last = Q.Nv <= h->cfg.coarse_max || (m % 2) == 1 || m < 4 || lev + 1 >= HDG_MAX_HLEVELS;
    if (last) {
      coarsest_level(h, Q, A, false);
      h->ql.push_back(Q);
      break;
    }
    Vec dinv(Q.Nv);
    for (int64_t v = 0; v < Q.Nv; ++v) dinv[v] = 1.0 / st[(size_t)4 * Q.Nv + v];
    Q.lmax = h->cfg.cheb_lmax[lev] > 0 ? h->cfg.cheb_lmax[lev] : hdg::lanczos_lmax(A, dinv, 30);
    Q.st = upload_vec(h, Vec(st.begin() + 4 * Q.Nv, st.begin() + 9 * Q.Nv));  // directions 4 ... 8
    Q.dinv = upload_vec(h, dinv);
    for (void** p : {&Q.x, &Q.b, &Q.r, &Q.d, &Q.t}) *p = valloc(h, Q.Nv);
    h->ql.push_back(Q);
    const hdg::Csr I = hdg::q1_bilinear(m);
    const hdg::Csr It = hdg::csr_transpose(I);
    const hdg::Csr Ac = hdg::csr_multiply(It, hdg::csr_multiply(A, I));
    m /= 2;
    st = hdg::csr_to_stencil(m, Ac);
    ++lev;
  }
}

// ------------------------------------------------------------ device helpers
double reduce_scalar(hdg_ctx* h, int np) {
  hipchk(hdg::launch_sum_partials(h->partial, np, h->scal, h->stream), "sum");
  hipchk(hipMemcpyAsync(h->scal_h, h->scal, sizeof(double), hipMemcpyDeviceToHost, h->stream), "d2h");
  hipchk(hipStreamSynchronize(h->stream), "sync");
  return *h->scal_h;
}

double dot(hdg_ctx* h, const double* a, const double* b, int64_t n) {
  hipchk(hdg::launch_dot_partials(a, b, n, h->partial, h->stream), "dot");
  return reduce_scalar(h, hdg::reduce_grid(n));
}

// Up to three dot products of vectors in precision pr, summed in FP64; one
// synchronization.  pairs: {x0, y0, x1, y1, ...}
void dots(hdg_ctx* h, hdg::Prec pr, int nd, std::initializer_list<const void*> pairs, int64_t n, double* out) {
  hdg::DotArgs d{};
  d.ndots = nd;
  auto it = pairs.begin();
  for (int j = 0; j < nd; ++j) {
    d.x[j] = *it++;
    d.y[j] = *it++;
  }
  const int np = hdg::reduce_grid(n);
  hipchk(hdg::launch_dots(pr, d, n, h->partial, h->stream), "dots");
  hipchk(hdg::launch_sum_partials_multi(h->partial, np, nd, h->scal, h->stream), "sum");
  hipchk(hipMemcpyAsync(h->scal_h, h->scal, nd * sizeof(double), hipMemcpyDeviceToHost, h->stream), "d2h");
  hipchk(hipStreamSynchronize(h->stream), "sync");
  for (int j = 0; j < nd; ++j) out[j] = h->scal_h[j];
}

// Trace-kernel arguments of level L for FP64 (pr == F64) or the cycle precision:
// the cycle uses the level's own blocks, FP64 in a reduced-precision cycle uses
// the FP64 copy.  kprec() is the precision the kernel is launched with.
hdg::TraceArgs targs(hdg_ctx* h, const PLevel& L, hdg::Prec pr) {
  hdg::TraceArgs a{};
  const bool cyc = pr != hdg::Prec::F64 || h->prec == hdg::Prec::F64;
  a.slab = cyc ? L.slab : static_cast<const void*>(L.slab64);
  a.dinv = L.dinv;
  a.pmat = cyc ? L.pmat : static_cast<const void*>(L.pmat64);
  a.omega = L.omega;
  a.n = h->n;
  a.nf = h->nf;
  a.ntiles = h->ntiles;
  if (!a.slab) throw std::logic_error("no FP64 operator at this level");
  return a;
}

hdg::Prec kprec(const PLevel& L, hdg::Prec pr) { return pr == hdg::Prec::F64 ? pr : L.mp; }

void apply(hdg_ctx* h, int p, const void* x, void* y, hdg::Prec pr) {
  hdg::TraceArgs a = targs(h, h->pl[p], pr);
  a.x = x;
  a.y = y;
  hipchk(hdg::launch_trace(kprec(h->pl[p], pr), h->pl[p].P, hdg::TM_APPLY, a, h->stream), "trace apply");
}

// r = b - S x, optionally the squared norm partials
void residual(hdg_ctx* h, int p, const void* b, const void* x, void* r, bool norm, hdg::Prec pr) {
  hdg::TraceArgs a = targs(h, h->pl[p], pr);
  a.x = x;
  a.b = b;
  a.y = r;
  a.partial = norm ? h->partial : nullptr;
  hipchk(hdg::launch_trace(kprec(h->pl[p], pr), h->pl[p].P, hdg::TM_RESID, a, h->stream), "trace residual");
}

double residual_norm(hdg_ctx* h, int p, const double* b, const double* x, double* r) {
  residual(h, p, b, x, r, true, hdg::Prec::F64);
  return std::sqrt(reduce_scalar(h, hdg::trace_partials(h->ntiles)));
}

// nu sweeps of the level-p Schwarz smoother on x (in place, cycle precision);
// zero: x == 0 on entry
void smooth(hdg_ctx* h, int p, const void* b, void* x, int nu, bool zero) {
  PLevel& L = h->pl[p];
  const hdg::Prec pr = h->prec;
  // The partitioned chain solve (P = 1) computes each sweep's residual in its own
  // launch from the face slab, which gathers x on neighbouring chains: a sweep
  // never updates in place.  Sweeps alternate between x and L.t so that the
  // last one writes x (one copy first where the count does not work out).  The
  // launch reads the slab in the vector precision: FP64 and FP32 cycles only (a
  // bfloat16 cycle keeps bfloat16 slabs on the coarse levels, FP32 vectors).
  if (h->cfg.smoother == HDG_SMOOTH_CHAIN && L.P == 1 && pr != hdg::Prec::BF16 && L.mp == pr && L.tri &&
      hdg::chain_shape_kind(1, h->n, L.chain_shape) == HDG_CHAIN_TRI) {
    void* cur = x;
    for (int s = 0; s < nu; ++s) {
      const bool z = zero && s == 0;
      void* dst = ((nu - 1 - s) % 2 == 0) ? x : L.t;
      if (!z && cur == dst) {
        void* other = dst == x ? L.t : x;
        hipchk(hdg::launch_copy(pr, cur, other, L.N, h->stream), "copy");
        cur = other;
      }
      hdg::ChainArgs c{};
      c.lds_cap = h->lds_cap;
      c.threads = L.chain_threads;
      c.shape = L.chain_shape;
      c.tri = L.tri;
      c.omega = L.omega;
      c.n = h->n;
      c.out = dst;
      if (z) {
        c.r = b;
        c.x = nullptr;
      } else {
        c.r = nullptr;
        c.b = b;
        c.slab = L.slab;
        c.x = cur;
      }
      hipchk(hdg::launch_chain_solve(pr, L.P, c, h->stream), "chain solve");
      cur = dst;
    }
    return;
  }
  for (int s = 0; s < nu; ++s) {
    const bool z = zero && s == 0;
    if (h->cfg.smoother == HDG_SMOOTH_PATCH) {
      // x <- x + omega W M (b - S x), W = 1/2 (every interior face lies in two
      // element patches): residual, then the patch-inverse slab applied face by face
      hdg::TraceArgs a = targs(h, L, pr);
      a.slab = L.pslab;
      a.omega = 0.5 * L.omega;
      a.y = x;
      if (z) {
        a.x = b;
        a.b = nullptr;
      } else {
        residual(h, p, b, x, L.r, false, pr);
        a.x = L.r;
        a.b = x;
      }
      hipchk(hdg::launch_trace(L.mp, L.P, hdg::TM_UPDATE, a, h->stream), "patch update");
    } else if (h->cfg.smoother == HDG_SMOOTH_FACE) {
      if (z) {
        hipchk(hdg::launch_dinv_apply(L.mp, L.P, L.dinv, b, L.omega, x, h->nf, h->stream), "dinv");
      } else {
        hdg::TraceArgs a = targs(h, L, pr);
        a.x = x;
        a.b = b;
        a.y = L.t;
        hipchk(hdg::launch_trace(L.mp, L.P, hdg::TM_FACE_SWEEP, a, h->stream), "face sweep");
        hipchk(hdg::launch_copy(pr, L.t, x, L.N, h->stream), "copy");
      }
    } else {
      hdg::ChainArgs c{};
      c.lds_cap = h->lds_cap;
      c.lds_level = L.chain_lds_level;
      c.threads = L.chain_threads;
      c.shape = L.chain_shape;
      c.remap = L.chain_remap >= 0 ? L.chain_remap : hdg::chain_remap(L.P);
      c.factors = L.chain;
      c.tri = L.tri;
      c.cstride = L.cstride;
      c.omega = L.omega;
      c.n = h->n;
      c.out = x;
      if (z) {
        c.r = b;
        c.x = nullptr;
      } else {
        residual(h, p, b, x, L.r, false, pr);
        c.r = L.r;
        c.x = x;
      }
      hipchk(hdg::launch_chain_solve(pr, L.P, c, h->stream), "chain solve");
    }
  }
}

// Coefficients of the Chebyshev three-term recurrence on [cheb_lo, cheb_hi] x
// lmax of level Q: step s updates d = c1[s] d + c2[s] Dinv (b - A x), x += d.
void chebyshev_coeffs(const hdg_ctx* h, const QLevel& Q, int nu, double* c1, double* c2) {
  const double a = h->cfg.cheb_lo * Q.lmax, c = h->cfg.cheb_hi * Q.lmax;
  const double theta = 0.5 * (c + a), delta = 0.5 * (c - a), sigma = theta / delta;
  double rho = 1.0 / sigma;
  for (int s = 0; s < nu; ++s) {
    if (s == 0) {
      c1[s] = 0.0;
      c2[s] = 1.0 / theta;
    } else {
      const double rn = 1.0 / (2.0 * sigma - rho);
      c1[s] = rn * rho;
      c2[s] = 2.0 * rn / delta;
      rho = rn;
    }
  }
}

// Chebyshev on Q1 level Q; result in Q.x.  zero: initial guess 0.
void chebyshev(hdg_ctx* h, QLevel& Q, const void* b, int nu, bool zero) {
  std::vector<double> c1(nu), c2(nu);
  chebyshev_coeffs(h, Q, nu, c1.data(), c2.data());
  void* cur = Q.x;
  void* nxt = Q.t;
  for (int s = 0; s < nu; ++s) {
    const void* xin = (zero && s == 0) ? nullptr : cur;
    hipchk(hdg::launch_q1_cheb(h->prec, Q.st, Q.dinv, b, xin, Q.d, nxt, c1[s], c2[s], Q.m, h->stream), "chebyshev");
    std::swap(cur, nxt);
  }
  if (cur != Q.x) hipchk(hdg::launch_copy(h->prec, cur, Q.x, Q.Nv, h->stream), "copy");
}

// Arguments of a fused visit of level Q with nu steps (the Q1 kernels' LDS
// regions hold the level's iterates; x_in, x_out, ec, bc set by the caller).
hdg::Q1FusedArgs q1_fused_args(const hdg_ctx* h, const QLevel& Q, int nu) {
  hdg::Q1FusedArgs a;
  a.st = Q.st;
  a.dinv = Q.dinv;
  a.b = Q.b;
  a.m = Q.m;
  a.nu = nu;
  a.tile = hdg::q1_fused_tile(Q.m);
  chebyshev_coeffs(h, Q, nu, a.c1, a.c2);
  return a;
}

// Cycle at Q1 level l for A_l x = b (b in Q.b, x in Q.x); zero: x == 0 on
// entry.  The W and WH schedules repeat the coarse correction from its first result.
void qcycle(hdg_ctx* h, int l, bool zero = true) {
  QLevel& Q = h->ql[l];
  const hdg::Prec pr = h->prec;
  if (Q.coarsest) {
    hipchk(hdg::launch_dense_gemv(pr, Q.inv, Q.b, Q.x, (int)Q.Nv, h->stream), "coarse solve");
    return;
  }
  QLevel& C = h->ql[l + 1];
  const bool fused = h->cfg.q1_schedule == HDG_Q1_FUSED && h->cfg.nu1 <= hdg::kQ1MaxNu &&
                     h->cfg.nu2 <= hdg::kQ1MaxNu;
  if (fused) {
    // pre-smoothing, residual and restriction in one launch; the iterate goes
    // to Q.t (its neighbours' halos still read Q.x), and back to Q.x below
    hdg::Q1FusedArgs a = q1_fused_args(h, Q, h->cfg.nu1);
    a.x_in = zero ? nullptr : Q.x;
    a.x_out = Q.t;
    a.bc = C.b;
    hipchk(hdg::launch_q1_pre(pr, a, h->stream), "q1 pre");
  } else {
    chebyshev(h, Q, Q.b, h->cfg.nu1, zero);
    hipchk(hdg::launch_q1_resid(pr, Q.st, Q.b, Q.x, Q.r, Q.m, h->stream), "q1 resid");
    hipchk(hdg::launch_q1_restrict(pr, Q.r, C.b, Q.m, h->stream), "q1 restrict");
  }
  qcycle(h, l + 1, true);
  if (h->cfg.cycle != HDG_CYCLE_V && !C.coarsest) qcycle(h, l + 1, false);
  if (fused) {
    hdg::Q1FusedArgs a = q1_fused_args(h, Q, h->cfg.nu2);
    a.x_in = Q.t;
    a.ec = C.x;
    a.x_out = Q.x;
    hipchk(hdg::launch_q1_post(pr, a, h->stream), "q1 post");
  } else {
    hipchk(hdg::launch_q1_prolong_add(pr, C.x, Q.x, Q.m, h->stream), "q1 prolong");
    chebyshev(h, Q, Q.b, h->cfg.nu2, false);
  }
}

void krylov_correction(hdg_ctx* h, int p, void* r, void* e, int m);

// V-cycle at p-level p for S_p x = b in the cycle precision; zero: x == 0 on
// entry (its content is ignored).  A coarser p-level with inner > 0 takes its
// correction from krylov_correction (K-cycle) instead of one recursive cycle.
void pcycle(hdg_ctx* h, int p, const void* b, void* x, bool zero) {
  PLevel& L = h->pl[p];
  const hdg::Prec pr = h->prec;
  smooth(h, p, b, x, h->cfg.nu1, zero);
  if (p >= 1) {
    PLevel& C = h->pl[p - 1];
    hdg::TraceArgs a = targs(h, L, pr);
    a.x = x;
    a.b = b;
    a.y = C.b;
    hipchk(hdg::launch_trace(L.mp, L.P, hdg::TM_RESID_RESTRICT, a, h->stream), "resid restrict");
    if (C.inner > 0) {
      krylov_correction(h, p - 1, C.b, C.x, C.inner);
    } else {
      pcycle(h, p - 1, C.b, C.x, true);
      if (h->cfg.cycle == HDG_CYCLE_W) pcycle(h, p - 1, C.b, C.x, false);
    }
    hipchk(hdg::launch_p_prolong_add(pr, L.P, L.pmat, C.x, x, h->nf, h->stream), "p prolong");
  } else {
    residual(h, 0, b, x, L.r, false, pr);
    QLevel& Q = h->ql[0];
    hipchk(hdg::launch_pj_restrict(pr, L.r, Q.b, h->n, h->stream), "pj restrict");
    qcycle(h, 0, true);
    if (h->cfg.cycle != HDG_CYCLE_V && !Q.coarsest) qcycle(h, 0, false);
    hipchk(hdg::launch_pj_prolong_add(pr, Q.x, x, h->n, h->stream), "pj prolong");
  }
  smooth(h, p, b, x, h->cfg.nu2, false);
}

// Full multigrid (Sec. 7) in the cycle precision: b restricted to every level
// (the right-hand sides of the Galerkin coarse systems), the coarsest solved
// exactly, then on each finer level the prolonged coarser result starts
// `cycles` cycles of that level.  x (finest) is written, not read.  Each coarse
// level's b and x are its own work vectors, which the cycles of the finer
// levels reuse only after that level is done.
void fmg(hdg_ctx* h, const void* b, void* x, int cycles) {
  const hdg::Prec pr = h->prec;
  const int k = h->k;
  const void* bf = b;
  for (int p = k; p >= 1; --p) {
    hipchk(hdg::launch_p_restrict(pr, h->pl[p].P, h->pl[p].pmat, bf, h->pl[p - 1].b, h->nf, h->stream),
           "fmg p restrict");
    bf = h->pl[p - 1].b;
  }
  hipchk(hdg::launch_pj_restrict(pr, bf, h->ql[0].b, h->n, h->stream), "fmg pj restrict");
  int lq = 0;
  for (; !h->ql[lq].coarsest; ++lq)
    hipchk(hdg::launch_q1_restrict(pr, h->ql[lq].b, h->ql[lq + 1].b, h->ql[lq].m, h->stream), "fmg q1 restrict");
  qcycle(h, lq, true);  // the coarsest level's exact solve
  for (int l = lq - 1; l >= 0; --l) {
    QLevel& Q = h->ql[l];
    hipchk(hdg::launch_zero(pr, Q.x, Q.Nv, h->stream), "zero");
    hipchk(hdg::launch_q1_prolong_add(pr, h->ql[l + 1].x, Q.x, Q.m, h->stream), "fmg q1 prolong");
    for (int c = 0; c < cycles; ++c) qcycle(h, l, false);
  }
  for (int p = 0; p <= k; ++p) {
    PLevel& L = h->pl[p];
    void* xp = p == k ? x : L.x;
    const void* bp = p == k ? b : L.b;
    hipchk(hdg::launch_zero(pr, xp, L.N, h->stream), "zero");
    if (p == 0)
      hipchk(hdg::launch_pj_prolong_add(pr, h->ql[0].x, xp, h->n, h->stream), "fmg pj prolong");
    else
      hipchk(hdg::launch_p_prolong_add(pr, L.P, L.pmat, h->pl[p - 1].x, xp, h->nf, h->stream), "fmg p prolong");
    for (int c = 0; c < cycles; ++c) pcycle(h, p, bp, xp, false);
  }
}

// K-cycle coarse correction (Notay-Vassilevski): m steps of flexible CG, FCG(1),
// for S_p e = r from e = 0, each preconditioned by one cycle started at level p.
// r is overwritten (it becomes the running residual).  Direction update
// d = z - (z . q / d . q) d_prev, step alpha = d . r / d . q with
// d . r = z . r - beta d_prev . r.  The scalars stay on the device (slots
// sc[0..4] of this level): no host round trip, so the cycle can be captured
// in a graph.  A vanishing residual gives d . q = 0; every ratio with a
// non-positive denominator is taken as 0, which leaves e unchanged from then on.
void device_dots(hdg_ctx* h, hdg::Prec pr, int nd, std::initializer_list<const void*> pairs, int64_t n,
                 double* out_dev) {
  hdg::DotArgs d{};
  d.ndots = nd;
  auto it = pairs.begin();
  for (int j = 0; j < nd; ++j) {
    d.x[j] = *it++;
    d.y[j] = *it++;
  }
  hipchk(hdg::launch_dots(pr, d, n, h->partial, h->stream), "dots");
  hipchk(hdg::launch_sum_partials_multi(h->partial, hdg::reduce_grid(n), nd, out_dev, h->stream), "sum");
}

void krylov_correction(hdg_ctx* h, int p, void* r, void* e, int m) {
  PLevel& L = h->pl[p];
  const hdg::Prec pr = h->prec;
  const int64_t N = L.N;
  double* sc = h->dsc + 8 * p;  // 0: d.r  1: d.q  2: z.q  3: z.r  4: d_prev.r
  hipchk(hdg::launch_zero(pr, e, N, h->stream), "zero");
  for (int step = 0; step < m; ++step) {
    pcycle(h, p, r, L.kz, true);
    if (step == 0) {
      hipchk(hdg::launch_copy(pr, L.kz, L.kd, N, h->stream), "copy");
      device_dots(h, pr, 1, {L.kz, r}, N, sc);
    } else {
      hdg::DotArgs d{};
      d.ndots = 3;
      d.x[0] = L.kz, d.y[0] = L.kq;
      d.x[1] = L.kz, d.y[1] = r;
      d.x[2] = L.kd, d.y[2] = r;
      hipchk(hdg::launch_dots(pr, d, N, h->partial, h->stream), "dots");
      hipchk(hdg::launch_sum_partials_fcg(h->partial, hdg::reduce_grid(N), sc, h->stream), "sum, fcg scalars");
      hipchk(hdg::launch_xpby_dev(pr, L.kz, sc, 2, 1, -1.0, L.kd, N, h->stream), "xpby");
    }
    hdg::TraceArgs ta = targs(h, L, pr);
    ta.x = L.kd;
    ta.y = L.kq;
    ta.partial = h->partial;
    hipchk(hdg::launch_trace(L.mp, L.P, hdg::TM_APPLY_DOT, ta, h->stream), "apply dot");
    hipchk(hdg::launch_sum_partials(h->partial, hdg::trace_partials(h->ntiles), sc + 1, h->stream), "sum");
    hipchk(hdg::launch_fcg_update(pr, sc, L.kd, e, L.kq, step + 1 < m ? r : nullptr, N, h->stream), "fcg update");
  }
}

// FP64 vector <-> cycle-precision staging buffer (no-op copy-free in FP64 mode)
const void* stage_in(hdg_ctx* h, const double* v, void* buf, int64_t n) {
  if (h->prec == hdg::Prec::F64) return v;
  hipchk(hdg::launch_to_f32(v, static_cast<float*>(buf), n, h->stream), "to f32");
  return buf;
}
void stage_out(hdg_ctx* h, const void* buf, double* v, int64_t n) {
  if (h->prec == hdg::Prec::F64) return;
  hipchk(hdg::launch_to_f64(static_cast<const float*>(buf), v, n, h->stream), "to f64");
}

// One V-cycle preconditioner application z = B r at level k with FP64 vectors.
void precondition_body(hdg_ctx* h, const double* r, double* z) {
  const int64_t N = h->pl[h->k].N;
  if (h->prec == hdg::Prec::F64) {
    pcycle(h, h->k, r, z, true);
    return;
  }
  pcycle(h, h->k, stage_in(h, r, h->cva, N), h->cvb, true);
  stage_out(h, h->cvb, z, N);
}

// The solver's z = B r (r = vr, z = vz).  With cfg.graph the whole cycle,
// Krylov-accelerated levels included, is captured once on a library stream as a
// HIP graph and replayed on the handle's stream: hundreds of launches become one.
// Everything the cycle touches is owned by the handle and fixed, and it makes no
// host round trip, allocation or memset.
void precondition(hdg_ctx* h) {
  if (!h->cfg.graph) {
    precondition_body(h, h->vr, h->vz);
    return;
  }
  if (!h->graph_exec) {
    if (!h->cap_stream) hipchk(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking), "stream");
    hipStream_t user = h->stream;
    h->stream = h->cap_stream;
    hipchk(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
    try {
      precondition_body(h, h->vr, h->vz);
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(h->cap_stream, &g);
      if (g) (void)hipGraphDestroy(g);
      h->stream = user;
      throw;
    }
    h->stream = user;
    hipchk(hipStreamEndCapture(h->cap_stream, &h->graph), "end capture");
    hipchk(hipGraphInstantiate(&h->graph_exec, h->graph, nullptr, nullptr, 0), "instantiate");
  }
  hipchk(hipGraphLaunch(h->graph_exec, h->stream), "graph launch");
}

// Largest eigenvalue of D^{-1} S_p (facet blocks) by Lanczos in the D inner product.
// Wall-clock breakdown of hdg_create, printed to stderr when the environment
// variable HDG_SETUP_TIMES is set (a diagnostic; no effect otherwise).
struct SetupClock {
  bool on = std::getenv("HDG_SETUP_TIMES") != nullptr;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now(), last = t0;
  std::string log;
  void mark(const std::string& what) {
    if (!on) return;
    const auto now = std::chrono::steady_clock::now();
    log += "  " + what + ": " + std::to_string(std::chrono::duration<double>(now - last).count()) + " s\n";
    last = now;
  }
  void report() {
    if (!on) return;
    const double tot = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    std::fprintf(stderr, "hdg_create %.3f s\n%s", tot, log.c_str());
  }
};

// Largest eigenvalue of the Lanczos tridiagonal matrix (diagonal al, off-diagonal
// be), by bisection on its Sturm sequence.
double tridiag_max(const std::vector<double>& al, const std::vector<double>& be) {
  const int m = (int)al.size();
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? std::fabs(be[i - 1]) : 0.0) + (i < m - 1 ? std::fabs(be[i]) : 0.0);
    lo = std::min(lo, al[i] - r);
    hi = std::max(hi, al[i] + r);
  }
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    int c = 0;
    double d = 1.0;
    for (int i = 0; i < m; ++i) {
      d = al[i] - mid - (i > 0 ? be[i - 1] * be[i - 1] / d : 0.0);
      if (d == 0.0) d = 1e-300;
      if (d < 0) ++c;
    }
    if (c >= m) hi = mid; else lo = mid;
  }
  return hi;
}

// Device memory of one set-up pass, released when it ends.
struct DevScratch {
  hipStream_t s = nullptr;
  std::vector<void*> ptrs;
  explicit DevScratch(hipStream_t st) : s(st) {}
  template <typename T>
  T* alloc(int64_t count) {
    void* q = nullptr;
    if (hipMalloc(&q, (size_t)std::max<int64_t>(count, 1) * sizeof(T)) != hipSuccess) {
      (void)hipGetLastError();
      throw std::bad_alloc();
    }
    ptrs.push_back(q);
    return static_cast<T*>(q);
  }
  ~DevScratch() {
    if (!ptrs.empty()) (void)hipStreamSynchronize(s);
    for (void* q : ptrs) (void)hipFree(q);
  }
  DevScratch(const DevScratch&) = delete;
  DevScratch& operator=(const DevScratch&) = delete;
};

// lambda_max(diag^{-1} A) of a Q1 level by 30 Lanczos steps on the device (FP64
// stencil st, 1 / diagonal dinv), from the start vector of the host estimate.
double estimate_q1_lmax(hdg_ctx* h, const double* st, const double* dinv, int m, DevScratch& tmp, int steps = 30) {
  const int64_t N = (int64_t)(m - 1) * (m - 1);
  hipStream_t s = h->stream;
  double *v = tmp.alloc<double>(N), *z = tmp.alloc<double>(N), *w = tmp.alloc<double>(N),
         *vold = tmp.alloc<double>(N), *r = tmp.alloc<double>(N), *zero = tmp.alloc<double>(N);
  Vec hv(N);
  for (int64_t i = 0; i < N; ++i) hv[i] = 1.0 + 0.25 * std::cos(0.7 * (double)i);
  hipchk(hipMemcpyAsync(v, hv.data(), N * sizeof(double), hipMemcpyHostToDevice, s), "h2d");
  hipchk(hdg::launch_fill(0.0, vold, N, s), "fill");
  hipchk(hdg::launch_fill(0.0, zero, N, s), "fill");
  hipchk(hdg::launch_vmul(dinv, v, z, N, s), "vmul");
  const double beta = std::sqrt(dot(h, v, z, N));
  hipchk(hdg::launch_xpby(v, 1.0 / beta - 1.0, v, N, s), "scale");
  hipchk(hdg::launch_xpby(z, 1.0 / beta - 1.0, z, N, s), "scale");
  std::vector<double> al, be;
  double bprev = 0.0;
  for (int it = 0; it < steps && it < N; ++it) {
    hipchk(hdg::launch_q1_resid9(st, zero, z, r, m, s), "q1 apply");  // r = -A z
    hipchk(hdg::launch_fill(0.0, w, N, s), "fill");
    hipchk(hdg::launch_axpy(-1.0, r, w, N, s), "axpy");
    const double alpha = dot(h, w, z, N);
    hipchk(hdg::launch_axpy(-alpha, v, w, N, s), "axpy");
    hipchk(hdg::launch_axpy(-bprev, vold, w, N, s), "axpy");
    hipchk(hdg::launch_vmul(dinv, w, z, N, s), "vmul");
    const double bn = std::sqrt(std::max(dot(h, w, z, N), 0.0));
    al.push_back(alpha);
    if (bn < 1e-14 * std::fabs(alpha)) break;
    be.push_back(bn);
    hipchk(hdg::launch_copy(hdg::Prec::F64, v, vold, N, s), "copy");
    hipchk(hdg::launch_fill(0.0, v, N, s), "fill");
    hipchk(hdg::launch_axpy(1.0 / bn, w, v, N, s), "axpy");
    hipchk(hdg::launch_xpby(z, 1.0 / bn - 1.0, z, N, s), "scale");
    bprev = bn;
  }
  return tridiag_max(al, be);
}

// Q1 hierarchy on the device from the p = 0 element blocks EB0 [n*n][4][4]
// (update: the level buffers exist).
void device_hlevels(hdg_ctx* h, const double* EB0, bool update, DevScratch& tmp) {
  hipStream_t s = h->stream;
  int m = h->n;
  double* st = tmp.alloc<double>(9LL * (m - 1) * (m - 1));
  hipchk(hdg::launch_q1_stencil0(EB0, h->n, st, s), "q1 stencil");
  for (int lev = 0;; ++lev) {
    if (!update) h->ql.emplace_back();
    QLevel& Q = h->ql[lev];
    Q.m = m;
    Q.Nv = (int64_t)(m - 1) * (m - 1);
    const bool last = Q.Nv <= h->cfg.coarse_max || (m % 2) == 1 || m < 4 || lev + 1 >= HDG_MAX_HLEVELS;
    if (last) {
      Vec sth((size_t)9 * Q.Nv);
      hipchk(hipMemcpyAsync(sth.data(), st, sth.size() * sizeof(double), hipMemcpyDeviceToHost, s), "d2h");
      hipchk(hipStreamSynchronize(s), "sync");
      coarsest_level(h, Q, hdg::stencil_to_csr(m, sth), update);
      break;
    }
    if (!update) {
      Q.st = valloc(h, 5 * Q.Nv);
      Q.dinv = valloc(h, Q.Nv);
      for (void** q : {&Q.x, &Q.b, &Q.r, &Q.d, &Q.t}) *q = valloc(h, Q.Nv);
    }
    double* dinv64 = tmp.alloc<double>(Q.Nv);
    hipchk(hdg::launch_q1_finish(h->prec, st, Q.Nv, Q.st, Q.dinv, dinv64, s), "q1 finish");
    Q.lmax = h->cfg.cheb_lmax[lev] > 0 ? h->cfg.cheb_lmax[lev] : estimate_q1_lmax(h, st, dinv64, m, tmp);
    double* stc = tmp.alloc<double>(9LL * (m / 2 - 1) * (m / 2 - 1));
    hipchk(hdg::launch_q1_galerkin(st, m, stc, s), "q1 galerkin");
    st = stc;
    m /= 2;
  }
}

// Device set-up of every p-level (element blocks, face slabs, facet inverses or
// chain factors) and of the Q1 hierarchy from the coefficient in h->kappa_dev.
// update: the level buffers exist (a new coefficient on an existing handle).
void device_levels(hdg_ctx* h, SetupClock& clk, bool update) {
  const int n = h->n, k = h->k;
  const int64_t ne = (int64_t)n * n, nf = h->nf, nch = 2LL * n;
  hipStream_t s = h->stream;
  const bool redisc = h->cfg.coarse == HDG_COARSE_REDISCRETIZE;
  const bool face = h->cfg.smoother == HDG_SMOOTH_FACE;
  DevScratch tmp(s);
  double* EBcur = tmp.alloc<double>(ne * 16LL * (k + 1) * (k + 1));
  double* EBnext = k >= 1 ? tmp.alloc<double>(ne * 16LL * k * k) : nullptr;
  int* fail = tmp.alloc<int>(1);
  hipchk(hipMemsetAsync(fail, 0, sizeof(int), s), "memset");
  for (int p = k; p >= 0; --p) {
    PLevel& L = h->pl[p];
    const int P = p + 1, P2 = P * P;
    if (p == k || redisc) {
      hdg::RefDegree rd;
      rd.build(p, 1.0 / n, h->cfg.tau);
      const hdg::PencilRef pc = hdg::pencil_reference(rd);
      Vec pack;
      std::vector<size_t> at;
      for (const Vec* v : std::initializer_list<const Vec*>{&pc.V, &pc.delta, &pc.mu, &rd.Dm, &rd.G, &rd.H, &rd.E,
                                                            &rd.Mb, &rd.P1}) {
        at.push_back(pack.size());
        pack.insert(pack.end(), v->begin(), v->end());
      }
      double* rdev = tmp.alloc<double>((int64_t)pack.size());
      hipchk(hipMemcpyAsync(rdev, pack.data(), pack.size() * sizeof(double), hipMemcpyHostToDevice, s), "h2d");
      hdg::ElemGenRef r{rdev + at[0], rdev + at[1], rdev + at[2], rdev + at[3], rdev + at[4],
                        rdev + at[5], rdev + at[6], rdev + at[7], rdev + at[8], h->cfg.tau};
      hipchk(hdg::launch_elem_rows(P, r, h->kappa_dev, EBcur, ne, s), "element blocks");
      hipchk(hipStreamSynchronize(s), "sync");  // pack (a host vector) is released below
    } else {
      const Vec Pp = hdg::p_prolongation(p + 1);
      double* pdev = tmp.alloc<double>((int64_t)Pp.size());
      hipchk(hipMemcpyAsync(pdev, Pp.data(), Pp.size() * sizeof(double), hipMemcpyHostToDevice, s), "h2d");
      hipchk(hdg::launch_elem_galerkin(p + 2, pdev, EBcur, EBnext, ne, s), "galerkin blocks");
      std::swap(EBcur, EBnext);
      hipchk(hipStreamSynchronize(s), "sync");
    }
    clk.mark("element blocks p=" + std::to_string(p));
    // face slab in the cycle's matrix precision (+ FP64 copy of the finest level)
    if (!update) L.mp = (h->prec == hdg::Prec::BF16 && p == k) ? hdg::Prec::F32 : h->prec;
    const int V = hdg::mat_lanes16(L.mp);
    const int64_t nq = (7LL * P2 + V - 1) / V, nq64 = (7LL * P2 + 1) / 2;
    const bool copy64 = h->prec != hdg::Prec::F64 && p == k;
    if (!update) {
      L.slab = balloc(h, (size_t)(h->ntiles * nq * 64 * 16));
      if (h->prec == hdg::Prec::F64) L.slab64 = static_cast<double*>(L.slab);
      else if (copy64) L.slab64 = static_cast<double*>(balloc(h, (size_t)(h->ntiles * nq64 * 64 * 16)));
      if (copy64) hipchk(hipMemsetAsync(L.slab64, 0, (size_t)(h->ntiles * nq64 * 64 * 16), s), "memset");
    }
    hipchk(hdg::launch_pack_slab(L.mp, P, EBcur, n, nf, L.slab, copy64 ? L.slab64 : nullptr, s), "pack slab");
    if (face) {
      const int64_t nqd = (P2 + V - 1) / V;
      if (!update) L.dinv = balloc(h, (size_t)(h->ntiles * nqd * 64 * 16));
      hipchk(hdg::launch_face_dinv(L.mp, P, EBcur, n, nf, L.dinv, fail, s), "facet inverses");
    } else if (h->cfg.smoother == HDG_SMOOTH_PATCH) {
      double* MB = tmp.alloc<double>(ne * 16LL * P2);
      hipchk(hdg::launch_patch_inverse(P, EBcur, n, MB, fail, s), "patch inverses");
      if (!update) L.pslab = balloc(h, (size_t)(h->ntiles * nq * 64 * 16));
      hipchk(hdg::launch_pack_slab(L.mp, P, MB, n, nf, L.pslab, nullptr, s), "pack patch inverses");
    } else {
      int64_t tot = 0;
      for (int ml = n - 1;; ml = (ml + 1) / 2) {
        tot += ml == 1 ? (int64_t)P2 : (int64_t)3 * P2 * (ml / 2);
        if (ml == 1) break;
      }
      if (!update) {
        L.cstride = tot;
        L.chain = valloc(h, nch * tot);
        const size_t es = hdg::vec_bytes(h->prec);
        const int64_t rhs_bytes = (int64_t)(n - 1) * P * (int64_t)es;
        L.chain_lds_level = hdg::chain_lds_level(P, n, es, std::min<int64_t>(8192, h->lds_cap - rhs_bytes));
      }
      const int64_t wpc = hdg::chain_factor_work_doubles(P, n);
      const int64_t batch = std::max<int64_t>(1, std::min<int64_t>(nch, ((int64_t)256 << 20) / 8 / wpc));
      double* work = tmp.alloc<double>(batch * wpc);
      for (int64_t c0 = 0; c0 < nch; c0 += batch)
        hipchk(hdg::launch_chain_factor(h->prec, P, EBcur, n, c0, (int)std::min<int64_t>(batch, nch - c0), work,
                                        L.chain, L.cstride, fail, s), "chain factors");
      if (P == 1 && hdg::chain_tri_lmax(n) > 0) {
        if (!update) L.tri = valloc(h, nch * hdg::chain_tri_stride(n));
        hipchk(hdg::launch_chain_tri_factor(h->prec, EBcur, n, L.tri, fail, s), "partitioned chain factors");
      }
    }
    clk.mark("face data and smoother factors p=" + std::to_string(p));
    if (p == 0) {
      device_hlevels(h, EBcur, update, tmp);
      clk.mark("Q1 hierarchy");
    }
  }
  int failed = 0;
  hipchk(hipMemcpyAsync(&failed, fail, sizeof(int), hipMemcpyDeviceToHost, s), "d2h");
  hipchk(hipStreamSynchronize(s), "sync");
  if (failed) throw std::runtime_error("a face or chain pivot block is not SPD");
}

double estimate_face_lmax(hdg_ctx* h, int p, int steps) {
  PLevel& L = h->pl[p];
  const int64_t N = L.N;
  double *v = (double*)L.x, *z = (double*)L.b, *w = (double*)L.r, *vold = (double*)L.t;
  Vec hv(N);
  for (int64_t i = 0; i < N; ++i) hv[i] = 1.0 + 0.25 * std::cos(0.37 * (double)i);
  hipchk(hipMemcpyAsync(v, hv.data(), N * sizeof(double), hipMemcpyHostToDevice, h->stream), "h2d");
  hipchk(hdg::launch_fill(0.0, vold, N, h->stream), "fill");
  hipchk(hdg::launch_dinv_apply(hdg::Prec::F64, L.P, L.dinv, v, 1.0, z, h->nf, h->stream), "dinv");
  double beta = std::sqrt(dot(h, v, z, N));
  hipchk(hdg::launch_xpby(v, 1.0 / beta - 1.0, v, N, h->stream), "scale");  // v <- v / beta
  hipchk(hdg::launch_xpby(z, 1.0 / beta - 1.0, z, N, h->stream), "scale");
  std::vector<double> al, be;
  double bprev = 0.0;
  for (int s = 0; s < steps; ++s) {
    apply(h, p, z, w, hdg::Prec::F64);
    const double alpha = dot(h, w, z, N);
    hipchk(hdg::launch_axpy(-alpha, v, w, N, h->stream), "axpy");
    hipchk(hdg::launch_axpy(-bprev, vold, w, N, h->stream), "axpy");
    hipchk(hdg::launch_dinv_apply(hdg::Prec::F64, L.P, L.dinv, w, 1.0, z, h->nf, h->stream), "dinv");
    const double bn = std::sqrt(std::max(dot(h, w, z, N), 0.0));
    al.push_back(alpha);
    if (bn < 1e-14 * std::fabs(alpha)) break;
    be.push_back(bn);
    hipchk(hdg::launch_copy(hdg::Prec::F64, v, vold, N, h->stream), "copy");
    hipchk(hdg::launch_fill(0.0, v, N, h->stream), "fill");
    hipchk(hdg::launch_axpy(1.0 / bn, w, v, N, h->stream), "axpy");
    hipchk(hdg::launch_xpby(z, 1.0 / bn - 1.0, z, N, h->stream), "scale");
    bprev = bn;
  }
  return tridiag_max(al, be);
}

// A pair of timing events, destroyed on every exit path.
struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  EventPair() {
    hipchk(hipEventCreate(&a), "event");
    hipchk(hipEventCreate(&b), "event");
  }
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
  EventPair(const EventPair&) = delete;
  EventPair& operator=(const EventPair&) = delete;
};

// Autotuner of the chain Schwarz launch shape of level p: workgroup size,
// XCD-aware chain order, LDS staging depth and (P = 3 ... 5) the lean or wide
// batch shape of the factor loads; at P = 1 the partitioned solve's chains per
// workgroup.  Every candidate solves each chain with the same operations in the
// same order, so the choice changes the time only, never the result.  Each
// candidate is timed (best of 3, after one warm-up launch) on the level's
// scratch vectors; the fastest is kept.
// The autotuner's choices, kept for the life of the process: the fastest shape
// depends on the launch's sizes (device, mesh, P, precision, the caller's
// schedule, the LDS cap), not on the coefficients, so a further handle of the
// same sizes takes the shape found by the first instead of timing again.
struct ChainTuneKey {
  int dev, n, P, prec, shape;
  int64_t lds_cap;
  bool operator<(const ChainTuneKey& o) const {
    return std::tie(dev, n, P, prec, shape, lds_cap) < std::tie(o.dev, o.n, o.P, o.prec, o.shape, o.lds_cap);
  }
};
struct ChainTuneVal {
  int threads, remap, lds_level, shape;
};
std::mutex g_chain_tune_mu;
std::map<ChainTuneKey, ChainTuneVal> g_chain_tune;

void tune_chain_timed(hdg_ctx* h, int p);
void tune_chain(hdg_ctx* h, int p) {
  PLevel& L = h->pl[p];
  int dev = 0;
  hipchk(hipGetDevice(&dev), "device");
  const ChainTuneKey key{dev, h->n, L.P, (int)h->prec, h->cfg.chain_shape, (int64_t)h->lds_cap};
  {
    std::lock_guard<std::mutex> lk(g_chain_tune_mu);
    const auto it = g_chain_tune.find(key);
    if (it != g_chain_tune.end()) {
      L.chain_threads = it->second.threads;
      L.chain_remap = it->second.remap;
      L.chain_lds_level = it->second.lds_level;
      L.chain_shape = it->second.shape;
      return;
    }
  }
  tune_chain_timed(h, p);
  std::lock_guard<std::mutex> lk(g_chain_tune_mu);
  g_chain_tune[key] = ChainTuneVal{L.chain_threads, L.chain_remap, L.chain_lds_level, L.chain_shape};
}

void tune_chain_timed(hdg_ctx* h, int p) {
  PLevel& L = h->pl[p];
  const hdg::Prec pr = h->prec;
  hipchk(hdg::launch_zero(pr, L.r, L.N, h->stream), "zero");
  const size_t es = hdg::vec_bytes(pr);
  const int64_t rhs_bytes = (int64_t)(h->n - 1) * L.P * (int64_t)es;
  const int lds_default = L.chain_lds_level;
  const int lds_staged = hdg::chain_lds_level(L.P, h->n, es, std::min<int64_t>(24576, h->lds_cap - rhs_bytes));
  const int lds_half = hdg::chain_lds_level(L.P, h->n, es, std::min<int64_t>(65536, h->lds_cap) - rhs_bytes);
  // as much as fits: at P = 1 the whole factor set of a chain (5 entries per
  // eliminated position) fits beside the right-hand side
  const int lds_full = hdg::chain_lds_level(L.P, h->n, es, h->lds_cap - rhs_bytes);
  EventPair ev;
  hipEvent_t e0 = ev.a, e1 = ev.b;
  float best = 1e30f;
  int bt = 0, br = -1, bl = lds_default, bw = L.chain_shape;
  const bool log = std::getenv("HDG_TUNE_LOG") != nullptr;  // a diagnostic: every candidate's time
  // Each candidate is timed as the smoother runs it inside a cycle: with an
  // iterate (x = out, zero), and with the 256 MB Infinity Cache flushed before
  // each timed launch (a level's factors fit in it, and back-to-back launches
  // would time them cache-warm, which the cycle never does between sweeps).
  hipchk(hdg::launch_zero(pr, L.t, L.N, h->stream), "zero");
  // The flush reads a 320 MB buffer (a dot product into its own tail), so it
  // evicts without leaving dirty lines to be written back during the timing.
  const int64_t flush_n = (int64_t)40 << 20;  // 320 MB of FP64
  double* flush = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&flush), (size_t)(flush_n + 1024) * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    flush = nullptr;  // no flush: time cache-warm rather than fail the set-up
  }
  struct FlushGuard {
    void* q;
    ~FlushGuard() {
      if (q) (void)hipFree(q);
    }
  } flush_guard{flush};
  if (flush) hipchk(hdg::launch_fill(0.0, flush, flush_n, h->stream), "fill");
  auto flush_cache = [&]() {
    if (flush) hipchk(hdg::launch_dot_partials(flush, flush, flush_n, flush + flush_n, h->stream), "cache flush");
  };
  if (hdg::chain_shape_kind(L.P, h->n, h->cfg.chain_shape) == HDG_CHAIN_TRI) {
    // the partitioned solve (P = 1): chains per workgroup only
    for (int g : {1, 2, 4, 8}) {
      hdg::ChainArgs c{};
      c.lds_cap = h->lds_cap;
      c.shape = HDG_CHAIN_TRI;
      c.tri = L.tri;
      c.omega = L.omega;
      c.n = h->n;
      c.r = L.r;
      c.x = L.t;
      c.out = L.t;
      c.threads = 64 * g;
      if (hdg::launch_chain_solve(pr, L.P, c, h->stream) != hipSuccess) {
        (void)hipGetLastError();
        continue;
      }
      float t = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        flush_cache();
        hipchk(hipEventRecord(e0, h->stream), "event");
        hipchk(hdg::launch_chain_solve(pr, L.P, c, h->stream), "chain tune");
        hipchk(hipEventRecord(e1, h->stream), "event");
        hipchk(hipEventSynchronize(e1), "event sync");
        float ms = 0.f;
        hipchk(hipEventElapsedTime(&ms, e0, e1), "elapsed");
        t = std::min(t, ms);
      }
      if (log) std::fprintf(stderr, "chain tune p=%d shape=partitioned chains/workgroup=%d: %.2f us\n", p, g, 1e3 * t);
      if (t < best) {
        best = t;
        bt = 64 * g;
      }
    }
    L.chain_threads = bt;
    L.chain_shape = HDG_CHAIN_TRI;
    return;
  }
  for (int wd : {1, 2, 3})
  for (int th : {64, 128, 256, 512, 1024}) {
    if (h->cfg.chain_shape != HDG_CHAIN_AUTO && wd != h->cfg.chain_shape) continue;  // the caller's schedule
    if (hdg::chain_shape_kind(L.P, h->n, wd) != wd) continue;  // that shape does not exist at P
    if (wd != 3 && th > hdg::chain_max_threads(L.P, wd == 2)) continue;
    for (int rm : {0, 1})
      for (int li = 0; li < 5; ++li) {
        const int lls[5] = {lds_default, lds_staged, lds_half, lds_full, 64};
        const int ll = lls[li];
        if (wd == 3 && ll != lds_default) continue;  // the flat schedule stages no factors
        if (std::find(lls, lls + li, ll) != lls + li) continue;  // the same staging depth: timed already
        hdg::ChainArgs c{};
        c.lds_cap = h->lds_cap;
        c.shape = wd;
        c.factors = L.chain;
        c.tri = L.tri;
        c.cstride = L.cstride;
        c.omega = L.omega;
        c.n = h->n;
        c.r = L.r;
        c.x = L.t;
        c.out = L.t;
        c.threads = th;
        c.remap = rm;
        c.lds_level = ll;
        if (hdg::launch_chain_solve(pr, L.P, c, h->stream) != hipSuccess) {
          (void)hipGetLastError();
          continue;
        }
        float t = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
          flush_cache();
          hipchk(hipEventRecord(e0, h->stream), "event");
          hipchk(hdg::launch_chain_solve(pr, L.P, c, h->stream), "chain tune");
          hipchk(hipEventRecord(e1, h->stream), "event");
          hipchk(hipEventSynchronize(e1), "event sync");
          float ms = 0.f;
          hipchk(hipEventElapsedTime(&ms, e0, e1), "elapsed");
          t = std::min(t, ms);
        }
        if (log)
          std::fprintf(stderr, "chain tune p=%d shape=%s threads=%d remap=%d lds_level=%d lds=%zu B: %.2f us\n", p,
                       wd == 3 ? "flat" : (wd == 2 ? "wide" : "lean"), th, rm, ll,
                       wd == 3 ? (size_t)(h->n - 1) * L.P * es : hdg::chain_lds_bytes(L.P, h->n, es, ll), 1e3 * t);
        if (t < best) {
          best = t;
          bt = th;
          br = rm;
          bl = ll;
          bw = wd;
        }
      }
  }
  L.chain_threads = bt;
  L.chain_remap = br;
  L.chain_lds_level = bl;
  L.chain_shape = bw;
}

// ------------------------------------------ many right-hand sides (chain smoother)
void* malloc_tracked(MultiWork& W, size_t bytes) {
  void* q = nullptr;
  if (hipMalloc(&q, std::max<size_t>(bytes, 16)) != hipSuccess) {
    (void)hipGetLastError();
    throw std::bad_alloc();
  }
  W.allocs.push_back(q);
  return q;
}

// Kernel of the cycle-precision multi apply at level L for R columns: the
// config's choice, or with autotune the faster of the vector and matrix-core
// kernels timed on Y = S X ([N][R], vector precision; best of 2 launches after a
// warm-up; X is read and zeroed first only if it is scratch); otherwise the
// vector kernel.  Both kernels compute the same products.
int multi_kernel_choice(hdg_ctx* h, const PLevel& L, int R, void* X, void* Y, bool scratch) {
  if (h->prec == hdg::Prec::F64) return 0;
  if (h->cfg.multi_kernel == HDG_MULTI_VECTOR) return 0;
  if (h->cfg.multi_kernel == HDG_MULTI_MATRIX) return 1;
  if (!h->cfg.autotune) return 0;
  if (scratch) hipchk(hdg::launch_zero(h->prec, X, L.N * R, h->stream), "zero");
  EventPair ev;
  float best = 1e30f;
  int pick = 0;
  for (int kern = 0; kern < 2; ++kern) {
    hdg::MultiArgs a{};
    a.slab = L.slab;
    a.pmat = L.pmat;
    a.nrhs = R;
    a.n = h->n;
    a.nf = h->nf;
    a.ntiles = h->ntiles;
    a.remap = 1;
    a.kernel = kern;
    a.X = X;
    a.Y = Y;
    hipchk(hdg::launch_trace_multi(L.mp, L.P, a, h->stream, hdg::TM_APPLY), "multi tune");
    float t = 1e30f;
    for (int rep = 0; rep < 2; ++rep) {
      hipchk(hipEventRecord(ev.a, h->stream), "event");
      hipchk(hdg::launch_trace_multi(L.mp, L.P, a, h->stream, hdg::TM_APPLY), "multi tune");
      hipchk(hipEventRecord(ev.b, h->stream), "event");
      hipchk(hipEventSynchronize(ev.b), "event sync");
      float ms = 0.f;
      hipchk(hipEventElapsedTime(&ms, ev.a, ev.b), "elapsed");
      t = std::min(t, ms);
    }
    if (t < best) {
      best = t;
      pick = kern;
    }
  }
  return pick;
}

MultiWork& multi_work(hdg_ctx* h, int R) {
  if (h->mw && h->mw->R == R) return *h->mw;
  hipchk(hipStreamSynchronize(h->stream), "sync");
  h->mw.reset();
  auto W = std::make_unique<MultiWork>();
  W->R = R;
  const size_t vb = hdg::vec_bytes(h->prec);
  for (const PLevel& L : h->pl) {
    W->px.push_back(malloc_tracked(*W, (size_t)L.N * R * vb));
    W->pb.push_back(malloc_tracked(*W, (size_t)L.N * R * vb));
    W->pr.push_back(malloc_tracked(*W, (size_t)L.N * R * vb));
  }
  for (const QLevel& Q : h->ql)
    for (auto* v : {&W->qx, &W->qb, &W->qr, &W->qd, &W->qt}) v->push_back(malloc_tracked(*W, (size_t)Q.Nv * R * vb));
  const size_t Nk = (size_t)h->pl[h->k].N;
  for (double** v : {&W->vr, &W->vz, &W->vd, &W->vq}) *v = (double*)malloc_tracked(*W, Nk * R * 8);
  if (h->prec != hdg::Prec::F64) {
    W->cva = malloc_tracked(*W, Nk * R * vb);
    W->cvb = malloc_tracked(*W, Nk * R * vb);
  }
  W->sc = (double*)malloc_tracked(*W, 5 * (size_t)R * 8);
  for (double** v : {&W->nrm, &W->nb, &W->act}) *v = (double*)malloc_tracked(*W, (size_t)R * 8);
  W->partial = (double*)malloc_tracked(*W, (size_t)hdg::dots_m_grid((int64_t)Nk) * R * 8);
  // columns per workgroup of the chain solve: time the powers of two up to the
  // LDS limit on the level's scratch vectors (best of 2 after a warm-up) and keep
  // the fastest; the chunking does not change any column's arithmetic
  const size_t vbytes = hdg::vec_bytes(h->prec);
  EventPair ev;
  hipEvent_t e0 = ev.a, e1 = ev.b;
  for (const PLevel& L : h->pl) {
    const int rmax = hdg::chain_multi_chunk(L.P, h->n, R, vbytes, h->lds_cap);
    int best_rc = rmax;
    float best = 1e30f;
    hipchk(hdg::launch_zero(h->prec, W->pr[L.p], L.N * R, h->stream), "zero");
    for (int rc = 1; rc <= rmax; rc *= 2) {
      hdg::ChainMultiArgs c{};
      c.lds_cap = h->lds_cap;
      c.factors = L.chain;
      c.cstride = L.cstride;
      c.omega = L.omega;
      c.n = h->n;
      c.R = R;
      c.rc = rc;
      c.nchunks = (R + rc - 1) / rc;
      c.r = W->pr[L.p];
      c.x = nullptr;
      c.out = W->px[L.p];
      if (h->cfg.smoother != HDG_SMOOTH_CHAIN || hdg::launch_chain_solve_m(h->prec, L.P, c, h->stream) != hipSuccess) {
        (void)hipGetLastError();
        continue;
      }
      float t = 1e30f;
      for (int rep = 0; rep < 2; ++rep) {
        hipchk(hipEventRecord(e0, h->stream), "event");
        hipchk(hdg::launch_chain_solve_m(h->prec, L.P, c, h->stream), "chain tune");
        hipchk(hipEventRecord(e1, h->stream), "event");
        hipchk(hipEventSynchronize(e1), "event sync");
        float ms = 0.f;
        hipchk(hipEventElapsedTime(&ms, e0, e1), "elapsed");
        t = std::min(t, ms);
      }
      if (t < best) {
        best = t;
        best_rc = rc;
      }
    }
    W->rc.push_back(best_rc);
  }
  for (const PLevel& L : h->pl)
    W->mk.push_back(multi_kernel_choice(h, L, R, W->pr[L.p], W->px[L.p], true));
  h->mw = std::move(W);
  return *h->mw;
}

hdg::MultiArgs margs(hdg_ctx* h, const PLevel& L, int R, bool f64) {
  hdg::MultiArgs a{};
  if (!f64 && h->mw && h->mw->R == R && (size_t)L.p < h->mw->mk.size()) a.kernel = h->mw->mk[L.p];
  a.slab = f64 && h->prec != hdg::Prec::F64 ? static_cast<const void*>(L.slab64) : L.slab;
  a.pmat = L.pmat;
  a.nrhs = R;
  a.n = h->n;
  a.nf = h->nf;
  a.ntiles = h->ntiles;
  a.remap = 1;
  return a;
}

void smooth_m(hdg_ctx* h, MultiWork& W, int p, const void* b, void* x, int nu, bool zero) {
  PLevel& L = h->pl[p];
  const hdg::Prec pr = h->prec;
  for (int s = 0; s < nu; ++s) {
    const bool z = zero && s == 0;
    hdg::ChainMultiArgs c{};
    c.lds_cap = h->lds_cap;
    c.factors = L.chain;
    c.cstride = L.cstride;
    c.omega = L.omega;
    c.n = h->n;
    c.R = W.R;
    c.rc = W.rc[p];
    c.nchunks = (W.R + c.rc - 1) / c.rc;
    c.out = x;
    if (z) {
      c.r = b;
      c.x = nullptr;
    } else {
      hdg::MultiArgs a = margs(h, L, W.R, false);
      a.X = x;
      a.B = b;
      a.Y = W.pr[p];
      hipchk(hdg::launch_trace_multi(L.mp, L.P, a, h->stream, hdg::TM_RESID), "residual multi");
      c.r = W.pr[p];
      c.x = x;
    }
    hipchk(hdg::launch_chain_solve_m(pr, L.P, c, h->stream), "chain solve multi");
  }
}

void chebyshev_m(hdg_ctx* h, MultiWork& W, int l, int nu, bool zero) {
  QLevel& Q = h->ql[l];
  const double a0 = h->cfg.cheb_lo * Q.lmax, c0 = h->cfg.cheb_hi * Q.lmax;
  const double theta = 0.5 * (c0 + a0), delta = 0.5 * (c0 - a0), sigma = theta / delta;
  double rho = 1.0 / sigma;
  void* cur = W.qx[l];
  void* nxt = W.qt[l];
  for (int s = 0; s < nu; ++s) {
    double c1, c2;
    if (s == 0) {
      c1 = 0.0;
      c2 = 1.0 / theta;
    } else {
      const double rn = 1.0 / (2.0 * sigma - rho);
      c1 = rn * rho;
      c2 = 2.0 * rn / delta;
      rho = rn;
    }
    const void* xin = (zero && s == 0) ? nullptr : cur;
    hipchk(hdg::launch_q1_cheb_m(h->prec, Q.st, Q.dinv, W.qb[l], xin, W.qd[l], nxt, c1, c2, Q.m, W.R, h->stream),
           "chebyshev multi");
    std::swap(cur, nxt);
  }
  if (cur != W.qx[l]) hipchk(hdg::launch_copy(h->prec, cur, W.qx[l], Q.Nv * W.R, h->stream), "copy");
}

void qcycle_m(hdg_ctx* h, MultiWork& W, int l, bool zero = true) {
  QLevel& Q = h->ql[l];
  const hdg::Prec pr = h->prec;
  if (Q.coarsest) {
    hipchk(hdg::launch_dense_gemm_m(pr, Q.inv, W.qb[l], W.qx[l], (int)Q.Nv, W.R, h->stream), "coarse solve multi");
    return;
  }
  chebyshev_m(h, W, l, h->cfg.nu1, zero);
  hipchk(hdg::launch_q1_resid_m(pr, Q.st, W.qb[l], W.qx[l], W.qr[l], Q.m, W.R, h->stream), "q1 resid multi");
  hipchk(hdg::launch_q1_restrict_m(pr, W.qr[l], W.qb[l + 1], Q.m, W.R, h->stream), "q1 restrict multi");
  qcycle_m(h, W, l + 1, true);
  if (h->cfg.cycle != HDG_CYCLE_V && !h->ql[l + 1].coarsest) qcycle_m(h, W, l + 1, false);
  hipchk(hdg::launch_q1_prolong_add_m(pr, W.qx[l + 1], W.qx[l], Q.m, W.R, h->stream), "q1 prolong multi");
  chebyshev_m(h, W, l, h->cfg.nu2, false);
}

// The cycle of pcycle (V or W) for every column at once (chain smoother; Krylov
// acceleration of coarse levels is not applied here).
void pcycle_m(hdg_ctx* h, MultiWork& W, int p, const void* b, void* x, bool zero) {
  PLevel& L = h->pl[p];
  const hdg::Prec pr = h->prec;
  smooth_m(h, W, p, b, x, h->cfg.nu1, zero);
  if (p >= 1) {
    hdg::MultiArgs a = margs(h, L, W.R, false);
    a.X = x;
    a.B = b;
    a.Y = W.pb[p - 1];
    hipchk(hdg::launch_trace_multi(L.mp, L.P, a, h->stream, hdg::TM_RESID_RESTRICT), "resid restrict multi");
    pcycle_m(h, W, p - 1, W.pb[p - 1], W.px[p - 1], true);
    if (h->cfg.cycle == HDG_CYCLE_W) pcycle_m(h, W, p - 1, W.pb[p - 1], W.px[p - 1], false);
    hipchk(hdg::launch_p_prolong_add_m(pr, L.P, L.pmat, W.px[p - 1], x, h->nf, W.R, h->stream), "p prolong multi");
  } else {
    hdg::MultiArgs a = margs(h, L, W.R, false);
    a.X = x;
    a.B = b;
    a.Y = W.pr[0];
    hipchk(hdg::launch_trace_multi(L.mp, L.P, a, h->stream, hdg::TM_RESID), "residual multi");
    hipchk(hdg::launch_pj_restrict_m(pr, W.pr[0], W.qb[0], h->n, W.R, h->stream), "pj restrict multi");
    qcycle_m(h, W, 0, true);
    if (h->cfg.cycle != HDG_CYCLE_V && !h->ql[0].coarsest) qcycle_m(h, W, 0, false);
    hipchk(hdg::launch_pj_prolong_add_m(pr, W.qx[0], x, h->n, W.R, h->stream), "pj prolong multi");
  }
  smooth_m(h, W, p, b, x, h->cfg.nu2, false);
}

// Z = B R for every column (FP64 in and out; the cycle runs in the cycle precision)
void precondition_m(hdg_ctx* h, MultiWork& W) {
  const int64_t NR = h->pl[h->k].N * (int64_t)W.R;
  if (h->prec == hdg::Prec::F64) {
    pcycle_m(h, W, h->k, W.vr, W.vz, true);
    return;
  }
  hipchk(hdg::launch_to_f32(W.vr, static_cast<float*>(W.cva), NR, h->stream), "to f32");
  pcycle_m(h, W, h->k, W.cva, W.cvb, true);
  hipchk(hdg::launch_to_f64(static_cast<const float*>(W.cvb), W.vz, NR, h->stream), "to f64");
}

// LDS bytes of one chain's right-hand side and its last block (chain smoother)
int64_t chain_lds_need(int n, int k, int64_t vb) {
  return ((int64_t)(n - 1) * (k + 1) + (int64_t)(k + 1) * (k + 1)) * vb;
}

void validate_config(const hdg_config_t* c) {
  if (!c) throw ArgError("cfg is NULL");
  if (c->n < 2) throw ArgError("n must be >= 2");
  if (c->k < 0 || c->k > HDG_MAX_DEGREE) throw ArgError("k out of range [0, 8]");
  if (!(c->tau > 0.0) || !std::isfinite(c->tau)) throw ArgError("tau must be > 0 and finite");
  if (c->nu1 < 1 || c->nu2 < 1 || c->nu1 > 64 || c->nu2 > 64) throw ArgError("nu1, nu2 must be in [1, 64]");
  if (c->smoother != HDG_SMOOTH_CHAIN && c->smoother != HDG_SMOOTH_FACE && c->smoother != HDG_SMOOTH_PATCH)
    throw ArgError("bad smoother");
  if (c->smoother == HDG_SMOOTH_PATCH && c->setup_on_host)
    throw ArgError("the element-patch smoother is built by the device set-up (setup_on_host = 0)");
  if (c->coarse != HDG_COARSE_GALERKIN && c->coarse != HDG_COARSE_REDISCRETIZE) throw ArgError("bad coarse");
  if (!(c->cheb_lo > 0.0) || !(c->cheb_hi > c->cheb_lo)) throw ArgError("need 0 < cheb_lo < cheb_hi");
  if (c->coarse_max < 1) throw ArgError("coarse_max must be >= 1");
  if (c->nq < 1 || c->nq > 32) throw ArgError("nq must be in [1, 32]");
  if ((int64_t)c->n * c->n > (int64_t)1 << 31) throw ArgError("n too large");
  if (c->precision != HDG_PREC_F64 && c->precision != HDG_PREC_F32 && c->precision != HDG_PREC_BF16)
    throw ArgError("bad precision");
  if (c->graph != 0 && c->graph != 1) throw ArgError("graph must be 0 or 1");
  if (c->autotune != 0 && c->autotune != 1) throw ArgError("autotune must be 0 or 1");
  if (c->cycle != HDG_CYCLE_V && c->cycle != HDG_CYCLE_W && c->cycle != HDG_CYCLE_WH)
    throw ArgError("cycle must be HDG_CYCLE_V, HDG_CYCLE_W or HDG_CYCLE_WH");
  if (c->setup_on_host != 0 && c->setup_on_host != 1) throw ArgError("setup_on_host must be 0 or 1");
  if (c->chain_shape < HDG_CHAIN_AUTO || c->chain_shape > HDG_CHAIN_TRI)
    throw ArgError("chain_shape must be HDG_CHAIN_AUTO, _LEAN, _WIDE, _FLAT or _TRI");
  if (c->q1_schedule != HDG_Q1_FUSED && c->q1_schedule != HDG_Q1_SEPARATE)
    throw ArgError("q1_schedule must be HDG_Q1_FUSED or HDG_Q1_SEPARATE");
  if (c->multi_kernel != HDG_MULTI_AUTO && c->multi_kernel != HDG_MULTI_VECTOR && c->multi_kernel != HDG_MULTI_MATRIX)
    throw ArgError("multi_kernel must be HDG_MULTI_AUTO, HDG_MULTI_VECTOR or HDG_MULTI_MATRIX");
  for (int p = 0; p <= HDG_MAX_DEGREE; ++p) {
    if (c->inner_steps[p] < 0 || c->inner_steps[p] > 64) throw ArgError("inner_steps must be in [0, 64]");
    if (p >= c->k && c->inner_steps[p] != 0) throw ArgError("inner_steps[p] must be 0 for p >= k");
  }
  const int64_t vb = c->precision == HDG_PREC_F64 ? 8 : 4;
  if (c->smoother == HDG_SMOOTH_CHAIN && chain_lds_need(c->n, c->k, vb) > hdg::kMaxLdsBytes)
    throw ArgError("chain smoother keeps one chain and one block in LDS: needs ((n-1)(k+1) + (k+1)^2) * "
                   "(8 bytes FP64, 4 bytes otherwise) <= 163840 (160 KiB); use the face smoother or a reduced "
                   "precision");
  if (c->smoother == HDG_SMOOTH_FACE && c->precision != HDG_PREC_F64)
    for (int p = 0; p <= c->k; ++p)
      if (!(c->omega[p] > 0)) throw ArgError("facet smoother in reduced precision needs omega[p] > 0 for every p");
}

}  // namespace

// =================================================================== C ABI
extern "C" {

const char* hdg_status_string(hdg_status_t s) {
  switch (s) {
    case HDG_OK: return "ok";
    case HDG_ERR_INVALID_ARG: return "invalid argument";
    case HDG_ERR_OOM: return "out of memory";
    case HDG_ERR_HIP: return "HIP error";
    case HDG_ERR_NOT_CONVERGED: return "not converged";
    case HDG_ERR_NONFINITE: return "non-finite value";
    case HDG_ERR_STATE: return "invalid state";
    case HDG_ERR_AT_FLOOR: return "stopped at the rounding floor of the residual";
  }
  return "unknown";
}

const char* hdg_last_error(hdg_handle_t h) { return h ? h->err.c_str() : "null handle"; }

hdg_status_t hdg_config_default(int32_t n, int32_t k, hdg_config_t* cfg) {
  if (!cfg) return HDG_ERR_INVALID_ARG;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->n = n;
  cfg->k = k;
  cfg->tau = 1.0;
  cfg->nu1 = cfg->nu2 = 2;
  cfg->smoother = HDG_SMOOTH_CHAIN;
  cfg->coarse = HDG_COARSE_GALERKIN;
  cfg->cheb_lo = 0.1;
  cfg->cheb_hi = 1.1;
  cfg->coarse_max = 2000;
  cfg->nq = k + 2;
  return HDG_OK;
}

hdg_status_t hdg_quadrature_nodes(int32_t nq, double* x_host) {
  if (nq < 1 || nq > 32 || !x_host) return HDG_ERR_INVALID_ARG;
  Vec x, w;
  hdg::gauss_legendre(nq, x, w);
  std::copy(x.begin(), x.end(), x_host);
  return HDG_OK;
}

hdg_status_t hdg_create(const hdg_config_t* cfg, const double* kappa_host, void* hip_stream,
                        hdg_handle_t* out) {
  if (!out) return HDG_ERR_INVALID_ARG;
  *out = nullptr;
  std::unique_ptr<hdg_ctx> h(new hdg_ctx());
  hdg_status_t st = guarded(h.get(), [&]() -> hdg_status_t {
    validate_config(cfg);
    if (!kappa_host) throw ArgError("kappa_host is NULL");
    h->cfg = *cfg;
    h->n = cfg->n;
    h->k = cfg->k;
    h->nq = cfg->nq;
    h->stream = (hipStream_t)hip_stream;
    h->prec = cfg->precision == HDG_PREC_F64 ? hdg::Prec::F64
              : (cfg->precision == HDG_PREC_F32 ? hdg::Prec::F32 : hdg::Prec::BF16);
    SetupClock clk;
    const int64_t ne = (int64_t)h->n * h->n;
    h->kappa.assign(kappa_host, kappa_host + ne);
    for (double v : h->kappa)
      if (!(v > 0.0) || !std::isfinite(v)) throw ArgError("kappa must be > 0 and finite");
    // arguments are valid: device set-up starts here (once per device: the address
    // of the allocation-free batch apply's descriptor table)
    hipchk(hdg::batch_scratch_address(&h->batch_scratch), "scratch address");
    {  // LDS a workgroup may use (with the opt-in above the default per-block size)
      int dev = 0, dflt = 0, optin = 0;
      hipchk(hipGetDevice(&dev), "device");
      hipchk(hipDeviceGetAttribute(&dflt, hipDeviceAttributeMaxSharedMemoryPerBlock, dev), "LDS size");
      if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess) {
        (void)hipGetLastError();
        optin = 0;
      }
      h->lds_cap = std::min<int64_t>(hdg::kMaxLdsBytes, std::max(dflt, optin));
      const int64_t vb = cfg->precision == HDG_PREC_F64 ? 8 : 4;
      if (cfg->smoother == HDG_SMOOTH_CHAIN && chain_lds_need(cfg->n, cfg->k, vb) > h->lds_cap)
        throw ArgError("chain smoother needs ((n-1)(k+1) + (k+1)^2) * (8 bytes FP64, 4 otherwise) = " +
                       std::to_string(chain_lds_need(cfg->n, cfg->k, vb)) + " bytes of LDS; this device allows " +
                       std::to_string(h->lds_cap));
    }
    h->nf = hdg::n_faces(h->n);
    h->ntiles = (h->nf + 63) / 64;
    h->pl.resize(h->k + 1);
    h->kappa_dev = upload(h.get(), h->kappa);
    // reduction buffers first: the device set-up's Lanczos estimates use them
    h->npartial = std::max(hdg::trace_partials(h->ntiles), 3 * 1024);
    h->partial = dalloc(h.get(), h->npartial);
    h->scal = dalloc(h.get(), 4);
    hipchk(hipHostMalloc((void**)&h->scal_h, 4 * sizeof(double), hipHostMallocDefault), "pinned");
    const bool host = cfg->setup_on_host != 0;
    if (!host) {
      for (int p = h->k; p >= 0; --p) {
        PLevel& L = h->pl[p];
        L.p = p;
        L.P = p + 1;
        L.N = h->nf * L.P;
      }
      device_levels(h.get(), clk, false);
    }
    Vec blocks;
    for (int p = h->k; p >= 0; --p) {
      PLevel& L = h->pl[p];
      L.p = p;
      L.P = p + 1;
      L.N = h->nf * L.P;
      if (host) {
        if (p == h->k || cfg->coarse == HDG_COARSE_REDISCRETIZE) blocks = blocks_finest(h.get(), p);
        else blocks = blocks_galerkin(h.get(), p + 1, blocks);
        clk.mark("element blocks p=" + std::to_string(p));
        build_face_data(h.get(), L, blocks);
        clk.mark("face data and chain factors p=" + std::to_string(p));
      }
      if (p >= 1) {
        const Vec Pp = hdg::p_prolongation(p);
        L.pmat64 = upload(h.get(), Pp);
        L.pmat = h->prec == hdg::Prec::F64 ? static_cast<void*>(L.pmat64) : upload_vec(h.get(), Pp);
      }
      L.omega = cfg->omega[p] > 0 ? cfg->omega[p] : (cfg->smoother == HDG_SMOOTH_PATCH ? 1.0 : 0.8);
      L.chain_shape = cfg->chain_shape;
      for (void** q : {&L.x, &L.b, &L.r, &L.t}) *q = valloc(h.get(), L.N);
      L.inner = cfg->inner_steps[p];
      if (L.inner > 0)
        for (void** q : {&L.kz, &L.kd, &L.kq}) *q = valloc(h.get(), L.N);
      if (p == 0 && host) {
        build_hlevels(h.get(), blocks);
        clk.mark("Q1 hierarchy");
      }
    }
    const int64_t Nk = h->pl[h->k].N;
    h->vr = dalloc(h.get(), Nk);
    h->vz = dalloc(h.get(), Nk);
    h->vd = dalloc(h.get(), Nk);
    h->vq = dalloc(h.get(), Nk);
    h->dsc = dalloc(h.get(), 8LL * (h->k + 1));
    if (cfg->autotune && cfg->smoother == HDG_SMOOTH_CHAIN)
      for (int p = 0; p <= h->k; ++p) tune_chain(h.get(), p);
    clk.mark("chain autotune");
    if (h->prec != hdg::Prec::F64) {
      h->cva = valloc(h.get(), Nk);
      h->cvb = valloc(h.get(), Nk);
    }
    if (cfg->smoother == HDG_SMOOTH_FACE)
      for (int p = 0; p <= h->k; ++p)
        if (!(cfg->omega[p] > 0)) h->pl[p].omega = 4.0 / (3.0 * estimate_face_lmax(h.get(), p, 30));
    {  // element-local reference data of degree k (misfit gradient)
      hdg::RefDegree rd;
      rd.build(h->k, 1.0 / h->n, cfg->tau);
      const hdg::PencilRef pc = hdg::pencil_reference(rd);
      Vec pack;
      for (const Vec* v : std::initializer_list<const Vec*>{&pc.V, &pc.delta, &pc.mu, &rd.E, &rd.H, &rd.C, &rd.Bt,
                                                            &rd.Mvinv})
        pack.insert(pack.end(), v->begin(), v->end());
      h->ref_dev = upload(h.get(), pack);
    }
    hipchk(hipStreamSynchronize(h->stream), "setup sync");
    clk.mark("reference data and sync");
    clk.report();
    return HDG_OK;
  });
  if (st != HDG_OK) return st;  // ~hdg_ctx releases what setup allocated
  *out = h.release();
  return HDG_OK;
}

hdg_status_t hdg_update_coefficients(hdg_handle_t h, const double* kappa_host) {
  if (!h || !kappa_host) return HDG_ERR_INVALID_ARG;
  const int64_t ne = (int64_t)h->n * h->n;
  for (int64_t e = 0; e < ne; ++e)
    if (!(kappa_host[e] > 0.0) || !std::isfinite(kappa_host[e])) {
      h->err = "kappa must be > 0 and finite";
      return HDG_ERR_INVALID_ARG;
    }
  if (h->cfg.setup_on_host) {
    h->err = "coefficient updates need the device set-up (setup_on_host = 0)";
    return HDG_ERR_STATE;
  }
  return guarded(h, [&]() -> hdg_status_t {
    SetupClock clk;
    hipchk(hipStreamSynchronize(h->stream), "sync");
    h->kappa.assign(kappa_host, kappa_host + ne);
    hipchk(hipMemcpy(h->kappa_dev, h->kappa.data(), ne * sizeof(double), hipMemcpyHostToDevice), "upload");
    device_levels(h, clk, true);
    if (h->cfg.smoother == HDG_SMOOTH_FACE)
      for (int p = 0; p <= h->k; ++p)
        if (!(h->cfg.omega[p] > 0)) h->pl[p].omega = 4.0 / (3.0 * estimate_face_lmax(h, p, 30));
    // a captured cycle holds the old Chebyshev and damping scalars: capture again on next use
    if (h->graph_exec) {
      (void)hipGraphExecDestroy(h->graph_exec);
      h->graph_exec = nullptr;
    }
    if (h->graph) {
      (void)hipGraphDestroy(h->graph);
      h->graph = nullptr;
    }
    hipchk(hipStreamSynchronize(h->stream), "sync");
    clk.report();
    return HDG_OK;
  });
}

hdg_status_t hdg_get_face_blocks(hdg_handle_t h, int32_t p, int64_t f, double* out_host) {
  if (!h || !out_host || p < 0 || p > h->k || f < 0 || f >= h->nf) return HDG_ERR_INVALID_ARG;
  return guarded(h, [&]() -> hdg_status_t {
    const PLevel& L = h->pl[p];
    const bool f64 = L.slab64 != nullptr;
    const hdg::Prec mp = f64 ? hdg::Prec::F64 : L.mp;
    const int V = hdg::mat_lanes16(mp), NE = 7 * L.P * L.P;
    const int64_t nq = (NE + V - 1) / V;
    std::vector<unsigned char> raw((size_t)nq * 16);
    const unsigned char* base = static_cast<const unsigned char*>(f64 ? static_cast<const void*>(L.slab64) : L.slab);
    const int64_t tile = f >> 6, lane = f & 63;
    hipchk(hipStreamSynchronize(h->stream), "sync");
    hipchk(hipMemcpy2D(raw.data(), 16, base + ((tile * nq) * 64 + lane) * 16, 64 * 16, 16, (size_t)nq,
                       hipMemcpyDeviceToHost), "d2h");
    for (int e = 0; e < NE; ++e) {
      const unsigned char* w = raw.data() + (size_t)(e / V) * 16;
      double v;
      if (mp == hdg::Prec::F64) {
        std::memcpy(&v, w + (e % V) * 8, 8);
      } else if (mp == hdg::Prec::F32) {
        float x;
        std::memcpy(&x, w + (e % V) * 4, 4);
        v = x;
      } else {
        uint16_t b;
        std::memcpy(&b, w + (e % V) * 2, 2);
        const uint32_t u = (uint32_t)b << 16;
        float x;
        std::memcpy(&x, &u, 4);
        v = x;
      }
      out_host[e] = v;
    }
    return HDG_OK;
  });
}

hdg_status_t hdg_destroy(hdg_handle_t h) {
  if (!h) return HDG_ERR_INVALID_ARG;
  delete h;  // ~hdg_ctx releases everything
  return HDG_OK;
}

hdg_status_t hdg_num_dofs(hdg_handle_t h, int32_t p, int64_t* n_lambda) {
  if (!h || !n_lambda || p < 0 || p > h->k) return HDG_ERR_INVALID_ARG;
  *n_lambda = h->pl[p].N;
  return HDG_OK;
}

hdg_status_t hdg_num_hlevels(hdg_handle_t h, int32_t* nlev) {
  if (!h || !nlev) return HDG_ERR_INVALID_ARG;
  *nlev = (int32_t)h->ql.size();
  return HDG_OK;
}

hdg_status_t hdg_hlevel_mesh(hdg_handle_t h, int32_t level, int32_t* m) {
  if (!h || !m || level < 0 || level >= (int)h->ql.size()) return HDG_ERR_INVALID_ARG;
  *m = h->ql[level].m;
  return HDG_OK;
}

hdg_status_t hdg_get_params(hdg_handle_t h, double* omega_out, double* lmax_out) {
  if (!h) return HDG_ERR_INVALID_ARG;
  if (omega_out)
    for (int p = 0; p <= h->k; ++p) omega_out[p] = h->pl[p].omega;
  if (lmax_out)
    for (size_t l = 0; l < h->ql.size(); ++l) lmax_out[l] = h->ql[l].lmax;
  return HDG_OK;
}

hdg_status_t hdg_get_chain_shape(hdg_handle_t h, int32_t p, int32_t* threads, int32_t* remap, int32_t* lds_level) {
  if (!h || p < 0 || p > h->k) return HDG_ERR_INVALID_ARG;
  const PLevel& L = h->pl[p];
  const int kind = hdg::chain_shape_kind(L.P, h->n, L.chain_shape);
  const bool flat = kind == HDG_CHAIN_FLAT, tri = kind == HDG_CHAIN_TRI;
  if (threads)
    *threads = L.chain_threads > 0
                   ? L.chain_threads
                   : (tri ? 256 : (flat ? hdg::chain_flat_threads(L.P, h->n) : hdg::chain_threads(L.P, h->n)));
  if (remap) *remap = tri ? 0 : (L.chain_remap >= 0 ? L.chain_remap : hdg::chain_remap(L.P));
  if (lds_level) *lds_level = flat || tri ? 64 : L.chain_lds_level;  // these schedules stage no factors
  return HDG_OK;
}

hdg_status_t hdg_element_block_host(int32_t n, int32_t k, int32_t p, double tau, double kappa_e,
                                    int32_t coarse, double* out_host) {
  if (n < 2 || k < 0 || k > HDG_MAX_DEGREE || p < 0 || p > k || !(tau > 0) || !(kappa_e > 0) ||
      !std::isfinite(kappa_e) || !out_host || (coarse != HDG_COARSE_GALERKIN && coarse != HDG_COARSE_REDISCRETIZE))
    return HDG_ERR_INVALID_ARG;
  try {
    const int top = coarse == HDG_COARSE_REDISCRETIZE ? p : k;
    hdg::RefDegree ref;
    ref.build(top, 1.0 / n, tau);
    const int P = top + 1, F4 = 4 * P, P2 = P * P;
    Vec K((size_t)F4 * F4), work((size_t)P2 * P2 + (size_t)P2 * F4);
    hdg::element_block(ref, kappa_e, K.data(), work.data());
    for (int q = top; q > p; --q) {
      const Vec Pp = hdg::p_prolongation(q);
      Vec Kc((size_t)16 * q * q);
      hdg::galerkin_block(Pp, q, K.data(), Kc.data());
      K.swap(Kc);
    }
    std::copy(K.begin(), K.end(), out_host);
  } catch (const std::exception&) {
    return HDG_ERR_STATE;
  }
  return HDG_OK;
}

hdg_status_t hdg_get_element_block(hdg_handle_t h, int32_t p, int64_t e, double* out_host) {
  if (!h || !out_host || p < 0 || p > h->k || e < 0 || e >= (int64_t)h->n * h->n) return HDG_ERR_INVALID_ARG;
  return hdg_element_block_host(h->n, h->k, p, h->cfg.tau, h->kappa[e], h->cfg.coarse, out_host);
}

hdg_status_t hdg_assemble_rhs(hdg_handle_t h, const double* f_qp_host, const double* gD_qp_host,
                              double* b) {
  if (!h || !f_qp_host || !b) return HDG_ERR_INVALID_ARG;
  return guarded(h, [&]() -> hdg_status_t {
    const int n = h->n, p = h->k, P = p + 1, P2 = P * P, F4 = 4 * P, nq = h->nq;
    const double hh = 1.0 / n;
    hdg::RefDegree ref;
    ref.build(p, hh, h->cfg.tau);
    Vec xq, wq;
    hdg::gauss_legendre(nq, xq, wq);
    const Vec nodes = hdg::trace_nodes(p);
    Vec Lq((size_t)nq * P);
    for (int q = 0; q < nq; ++q) hdg::lagrange_eval(nodes, xq[q], Lq.data() + (size_t)q * P);
    // boundary traces: L2 projection onto Q_p(e) of the data at the GL points
    Vec lam_bd((size_t)4 * n * P, 0.0);
    if (gD_qp_host) {
      Vec M1inv(ref.M1);
      if (!hdg::cholesky_inverse(P, M1inv)) throw std::runtime_error("mass");
      for (int nb = 0; nb < 4 * n; ++nb) {
        Vec mom(P, 0.0);
        for (int q = 0; q < nq; ++q)
          for (int a = 0; a < P; ++a) mom[a] += wq[q] * gD_qp_host[(size_t)nb * nq + q] * Lq[(size_t)q * P + a];
        for (int a = 0; a < P; ++a) {
          double s = 0.0;
          for (int c = 0; c < P; ++c) s += M1inv[a * P + c] * mom[c];
          lam_bd[(size_t)nb * P + a] = s;
        }
      }
    }
    const int64_t ne = (int64_t)n * n;
    Vec g((size_t)ne * F4), Fall((size_t)ne * P2);
    hdg::parallel_for(ne, [&](int64_t e0, int64_t e1) {
      Vec work((size_t)P2 * P2 + (size_t)P2 * F4), K((size_t)F4 * F4);
      for (int64_t e = e0; e < e1; ++e) {
        double* F = Fall.data() + (size_t)e * P2;
        const double* fq = f_qp_host + (size_t)e * nq * nq;
        for (int i2 = 0; i2 < P; ++i2)
          for (int i1 = 0; i1 < P; ++i1) {
            double s = 0.0;
            for (int bq = 0; bq < nq; ++bq)
              for (int aq = 0; aq < nq; ++aq)
                s += wq[aq] * wq[bq] * fq[aq + nq * bq] * Lq[(size_t)aq * P + i1] * Lq[(size_t)bq * P + i2];
            F[i1 + P * i2] = 0.25 * hh * hh * s;
          }
        double* ge = g.data() + (size_t)e * F4;
        hdg::element_source(ref, h->kappa[e], F, ge, work.data());
        const int i = (int)(e % n), j = (int)(e / n);
        const bool touches = i == 0 || j == 0 || i == n - 1 || j == n - 1;
        if (touches && gD_qp_host) {
          hdg::element_block(ref, h->kappa[e], K.data(), work.data());
          int nbf[4] = {i == 0 ? 3 * n + j : -1, i == n - 1 ? n + j : -1, j == 0 ? i : -1,
                        j == n - 1 ? 2 * n + i : -1};
          for (int r = 0; r < F4; ++r) {
            double s = 0.0;
            for (int lf = 0; lf < 4; ++lf)
              if (nbf[lf] >= 0)
                for (int c = 0; c < P; ++c) s += K[(size_t)r * F4 + lf * P + c] * lam_bd[(size_t)nbf[lf] * P + c];
            ge[r] -= s;
          }
        }
      }
    });
    Vec bh((size_t)h->nf * P);
    hdg::parallel_for(h->nf, [&](int64_t f0, int64_t f1) {
      for (int64_t f = f0; f < f1; ++f) {
        int64_t lo, hi;
        int llo, lhi;
        hdg::face_elements(n, f, lo, hi, llo, lhi);
        for (int a = 0; a < P; ++a)
          bh[(size_t)f * P + a] = g[(size_t)lo * F4 + llo * P + a] + g[(size_t)hi * F4 + lhi * P + a];
      }
    });
    hipchk(hipMemcpyAsync(b, bh.data(), bh.size() * sizeof(double), hipMemcpyHostToDevice, h->stream), "h2d");
    // source state for hdg_reconstruct / the misfit gradient
    if (!h->F_dev) {
      h->F_dev = dalloc(h, ne * P2);
      h->lambd_dev = dalloc(h, 4LL * n * P);
    }
    hipchk(hipMemcpyAsync(h->F_dev, Fall.data(), Fall.size() * sizeof(double), hipMemcpyHostToDevice, h->stream),
           "h2d");
    hipchk(hipMemcpyAsync(h->lambd_dev, lam_bd.data(), lam_bd.size() * sizeof(double), hipMemcpyHostToDevice,
                          h->stream), "h2d");
    hipchk(hipStreamSynchronize(h->stream), "sync");
    h->have_source = true;
    return HDG_OK;
  });
}

namespace {
hdg_status_t need_f64_level(hdg_handle_t h, int p) {
  if (h->pl[p].slab64) return HDG_OK;
  h->err = "reduced-precision handle keeps the FP64 operator at p = k only";
  return HDG_ERR_STATE;
}
}  // namespace

hdg_status_t hdg_apply_trace_operator(hdg_handle_t h, int32_t p, const double* x, double* y) {
  if (!h || !x || !y || p < 0 || p > h->k || x == y) return HDG_ERR_INVALID_ARG;
  if (need_f64_level(h, p) != HDG_OK) return HDG_ERR_STATE;
  return guarded(h, [&]() -> hdg_status_t {
    apply(h, p, x, y, hdg::Prec::F64);
    return HDG_OK;
  });
}

hdg_status_t hdg_apply_abs(hdg_handle_t h, int32_t p, const double* x, double* y) {
  if (!h || !x || !y || p < 0 || p > h->k || x == y) return HDG_ERR_INVALID_ARG;
  if (need_f64_level(h, p) != HDG_OK) return HDG_ERR_STATE;
  return guarded(h, [&]() -> hdg_status_t {
    hdg::TraceArgs a = targs(h, h->pl[p], hdg::Prec::F64);
    a.x = x;
    a.y = y;
    hipchk(hdg::launch_trace(hdg::Prec::F64, h->pl[p].P, hdg::TM_ABS, a, h->stream), "trace abs");
    return HDG_OK;
  });
}

hdg_status_t hdg_apply_trace_operator_timed(hdg_handle_t h, int32_t p, int32_t precision, const void* x, void* y,
                                            double* kernel_us) {
  if (!h || !x || !y || !kernel_us || p < 0 || p > h->k || x == y) return HDG_ERR_INVALID_ARG;
  if (precision != HDG_PREC_F64 && precision != (int32_t)h->prec) return HDG_ERR_INVALID_ARG;
  if (precision == HDG_PREC_F64 && need_f64_level(h, p) != HDG_OK) return HDG_ERR_STATE;
  return guarded(h, [&]() -> hdg_status_t {
    if (!h->ev0) {
      hipchk(hipEventCreate(&h->ev0), "event");
      hipchk(hipEventCreate(&h->ev1), "event");
    }
    const hdg::Prec pr = precision == HDG_PREC_F64 ? hdg::Prec::F64 : h->prec;
    hdg::TraceArgs a = targs(h, h->pl[p], pr);
    a.x = x;
    a.y = y;
    a.ev_start = h->ev0;
    a.ev_stop = h->ev1;
    hipchk(hdg::launch_trace(kprec(h->pl[p], pr), h->pl[p].P, hdg::TM_APPLY, a, h->stream), "trace apply");
    hipchk(hipEventSynchronize(h->ev1), "event sync");
    float ms = 0.f;
    hipchk(hipEventElapsedTime(&ms, h->ev0, h->ev1), "elapsed");
    *kernel_us = 1e3 * (double)ms;
    return HDG_OK;
  });
}

hdg_status_t hdg_apply_trace_operator_multi(hdg_handle_t h, int32_t p, int32_t precision, int32_t nrhs,
                                            const void* X, void* Y) {
  if (!h || !X || !Y || p < 0 || p > h->k || X == Y || nrhs < 1 || nrhs > 4096) return HDG_ERR_INVALID_ARG;
  if (precision != HDG_PREC_F64 && precision != (int32_t)h->prec) return HDG_ERR_INVALID_ARG;
  if (precision == HDG_PREC_F64 && need_f64_level(h, p) != HDG_OK) return HDG_ERR_STATE;
  return guarded(h, [&]() -> hdg_status_t {
    const hdg::Prec pr = precision == HDG_PREC_F64 ? hdg::Prec::F64 : h->prec;
    const PLevel& L = h->pl[p];
    hdg::MultiArgs a{};
    a.slab = pr == hdg::Prec::F64 && h->prec != hdg::Prec::F64 ? static_cast<const void*>(L.slab64) : L.slab;
    a.X = X;
    a.Y = Y;
    a.nrhs = nrhs;
    a.n = h->n;
    a.nf = h->nf;
    a.ntiles = h->ntiles;
    a.remap = 1;
    if (pr != hdg::Prec::F64) {
      // kernel of this level and column count: config, or timed once (autotune)
      const int64_t key = (int64_t)p * 8192 + nrhs;
      auto it = h->multi_pick.find(key);
      if (it == h->multi_pick.end())
        it = h->multi_pick.emplace(key, multi_kernel_choice(h, L, nrhs, const_cast<void*>(X), Y, false)).first;
      a.kernel = it->second;
    }
    hipchk(hdg::launch_trace_multi(kprec(L, pr), L.P, a, h->stream), "trace apply multi");
    return HDG_OK;
  });
}

hdg_status_t hdg_apply_trace_operator_batch(int32_t count, const hdg_handle_t* handles, const int32_t* p,
                                            const double* const* X, double* const* Y) {
  if (count < 1 || !handles || !p || !X || !Y) return HDG_ERR_INVALID_ARG;
  for (int i = 0; i < count; ++i) {
    hdg_handle_t h = handles[i];
    if (!h || p[i] < 0 || p[i] > h->k || !X[i] || !Y[i] || (const void*)X[i] == (const void*)Y[i])
      return HDG_ERR_INVALID_ARG;
    if (need_f64_level(h, p[i]) != HDG_OK) return HDG_ERR_STATE;
  }
  hdg_handle_t h0 = handles[0];
  return guarded(h0, [&]() -> hdg_status_t {
    h0->batch_host.resize(count);
    int64_t tot = 0;
    int pmax = 1;
    for (int i = 0; i < count; ++i) {
      const hdg_handle_t h = handles[i];
      const PLevel& L = h->pl[p[i]];
      hdg::BatchMesh& M = h0->batch_host[i];
      M.slab = L.slab64;
      M.x = X[i];
      M.y = Y[i];
      M.nf = h->nf;
      M.ntiles = h->ntiles;
      M.tile0 = tot;
      M.n = h->n;
      M.P = L.P;
      M.mp = (int)hdg::Prec::F64;
      pmax = std::max(pmax, L.P);
      tot += h->ntiles;
    }
    if (h0->batch_cap < count) {
      h0->batch_dev = static_cast<hdg::BatchMesh*>(balloc(h0, sizeof(hdg::BatchMesh) * (size_t)count));
      h0->batch_cap = count;
    }
    hipchk(hipMemcpyAsync(h0->batch_dev, h0->batch_host.data(), sizeof(hdg::BatchMesh) * (size_t)count,
                          hipMemcpyHostToDevice, h0->stream), "h2d");
    // a fixed grid: 8 workgroups per compute unit, or fewer for small batches
    const int64_t need = (tot + 3) / 4;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(need, 256 * 8));
    hipchk(hdg::launch_trace_batch(h0->batch_dev, count, tot, grid, pmax, h0->stream), "trace apply batch");
    hipchk(hipStreamSynchronize(h0->stream), "sync");  // the descriptor table is reused by the next call
    return HDG_OK;
  });
}

hdg_status_t hdg_apply_trace_operator_batch_lp(int32_t count, const hdg_handle_t* handles, const int32_t* p,
                                               const float* const* X, float* const* Y) {
  if (count < 1 || !handles || !p || !X || !Y) return HDG_ERR_INVALID_ARG;
  for (int i = 0; i < count; ++i) {
    hdg_handle_t h = handles[i];
    if (!h || p[i] < 0 || p[i] > h->k || !X[i] || !Y[i] || (const void*)X[i] == (const void*)Y[i])
      return HDG_ERR_INVALID_ARG;
    if (h->prec == hdg::Prec::F64) {
      h->err = "handle was created with FP64 cycle precision";
      return HDG_ERR_STATE;
    }
  }
  hdg_handle_t h0 = handles[0];
  return guarded(h0, [&]() -> hdg_status_t {
    h0->batch_host.resize(count);
    int64_t tot = 0;
    int pmax = 1;
    for (int i = 0; i < count; ++i) {
      const hdg_handle_t h = handles[i];
      const PLevel& L = h->pl[p[i]];
      hdg::BatchMesh& M = h0->batch_host[i];
      M.slab = L.slab;  // the cycle precision's blocks, as hdg_apply_trace_operator_lp reads them
      M.x = X[i];
      M.y = Y[i];
      M.nf = h->nf;
      M.ntiles = h->ntiles;
      M.tile0 = tot;
      M.n = h->n;
      M.P = L.P;
      M.mp = (int)L.mp;
      pmax = std::max(pmax, L.P);
      tot += h->ntiles;
    }
    if (h0->batch_cap < count) {
      h0->batch_dev = static_cast<hdg::BatchMesh*>(balloc(h0, sizeof(hdg::BatchMesh) * (size_t)count));
      h0->batch_cap = count;
    }
    hipchk(hipMemcpyAsync(h0->batch_dev, h0->batch_host.data(), sizeof(hdg::BatchMesh) * (size_t)count,
                          hipMemcpyHostToDevice, h0->stream), "h2d");
    const int64_t need = (tot + 3) / 4;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(need, 256 * 8));
    hipchk(hdg::launch_trace_batch(h0->batch_dev, count, tot, grid, pmax, h0->stream, true), "trace apply batch lp");
    hipchk(hipStreamSynchronize(h0->stream), "sync");  // the descriptor table is reused by the next call
    return HDG_OK;
  });
}

static_assert(HDG_BATCH_NOALLOC_MAX == hdg::kBatchNoallocMax, "descriptor table size");

hdg_status_t hdg_apply_trace_operator_batch_noalloc(int32_t count, const hdg_handle_t* handles, const int32_t* p,
                                                    const double* const* X, double* const* Y) {
  if (count < 1 || !handles || !p || !X || !Y) return HDG_ERR_INVALID_ARG;
  if (count > HDG_BATCH_NOALLOC_MAX) {
    if (handles[0]) handles[0]->err = "the allocation-free batch apply takes at most HDG_BATCH_NOALLOC_MAX meshes";
    return HDG_ERR_INVALID_ARG;
  }
  for (int i = 0; i < count; ++i) {
    hdg_handle_t h = handles[i];
    if (!h || p[i] < 0 || p[i] > h->k || !X[i] || !Y[i] || (const void*)X[i] == (const void*)Y[i])
      return HDG_ERR_INVALID_ARG;
    if (need_f64_level(h, p[i]) != HDG_OK) return HDG_ERR_STATE;
  }
  hdg_handle_t h0 = handles[0];
  if (!h0->batch_scratch) {
    h0->err = "no device scratch address for this handle";
    return HDG_ERR_STATE;
  }
  return guarded(h0, [&]() -> hdg_status_t {
    hdg::BatchMesh tab[hdg::kBatchNoallocMax];  // host copy on this call's stack: nothing allocated
    int64_t tot = 0;
    int pmax = 1;
    for (int i = 0; i < count; ++i) {
      const hdg_handle_t h = handles[i];
      const PLevel& L = h->pl[p[i]];
      hdg::BatchMesh& M = tab[i];
      M.slab = L.slab64;
      M.x = X[i];
      M.y = Y[i];
      M.nf = h->nf;
      M.ntiles = h->ntiles;
      M.tile0 = tot;
      M.n = h->n;
      M.P = L.P;
      M.mp = (int)hdg::Prec::F64;
      pmax = std::max(pmax, L.P);
      tot += h->ntiles;
    }
    hipchk(hipMemcpyAsync(h0->batch_scratch, tab, sizeof(hdg::BatchMesh) * (size_t)count, hipMemcpyHostToDevice,
                          h0->stream), "h2d");
    const int64_t need = (tot + 3) / 4;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(need, 256 * 8));
    hipchk(hdg::launch_trace_batch(static_cast<const hdg::BatchMesh*>(h0->batch_scratch), count, tot, grid, pmax,
                                   h0->stream), "trace apply batch");
    // the host table lives on this stack frame and the device table is shared by
    // every call on this GPU: both are released only after the kernel has run
    hipchk(hipStreamSynchronize(h0->stream), "sync");
    return HDG_OK;
  });
}

hdg_status_t hdg_apply_trace_operator_lp(hdg_handle_t h, int32_t p, const float* x, float* y) {
  if (!h || !x || !y || p < 0 || p > h->k || (const void*)x == (const void*)y) return HDG_ERR_INVALID_ARG;
  if (h->prec == hdg::Prec::F64) {
    h->err = "handle was created with FP64 cycle precision";
    return HDG_ERR_STATE;
  }
  return guarded(h, [&]() -> hdg_status_t {
    apply(h, p, x, y, h->prec);
    return HDG_OK;
  });
}

hdg_status_t hdg_residual(hdg_handle_t h, int32_t p, const double* b, const double* x, double* r,
                          double* norm2_host) {
  if (!h || !b || !x || !r || p < 0 || p > h->k || r == x) return HDG_ERR_INVALID_ARG;
  if (need_f64_level(h, p) != HDG_OK) return HDG_ERR_STATE;
  return guarded(h, [&]() -> hdg_status_t {
    if (norm2_host) {
      const double v = residual_norm(h, p, b, x, r);
      *norm2_host = v;
      if (!std::isfinite(v)) {
        h->err = "non-finite residual norm";
        return HDG_ERR_NONFINITE;
      }
    } else {
      residual(h, p, b, x, r, false, hdg::Prec::F64);
    }
    return HDG_OK;
  });
}

hdg_status_t hdg_smooth(hdg_handle_t h, int32_t p, const double* b, double* x, int32_t sweeps) {
  if (!h || !b || !x || p < 0 || p > h->k || sweeps < 0) return HDG_ERR_INVALID_ARG;
  return guarded(h, [&]() -> hdg_status_t {
    const int64_t N = h->pl[p].N;
    if (h->prec == hdg::Prec::F64) {
      smooth(h, p, b, x, sweeps, false);
    } else {
      const void* bl = stage_in(h, b, h->cva, N);
      smooth(h, p, bl, const_cast<void*>(stage_in(h, x, h->cvb, N)), sweeps, false);
      stage_out(h, h->cvb, x, N);
    }
    return HDG_OK;
  });
}

hdg_status_t hdg_restrict(hdg_handle_t h, int32_t p_fine, const double* r_fine, double* r_coarse) {
  if (!h || !r_fine || !r_coarse || p_fine < 1 || p_fine > h->k) return HDG_ERR_INVALID_ARG;
  return guarded(h, [&]() -> hdg_status_t {
    hipchk(hdg::launch_p_restrict(hdg::Prec::F64, p_fine + 1, h->pl[p_fine].pmat64, r_fine, r_coarse, h->nf,
                                  h->stream),
           "restrict");
    return HDG_OK;
  });
}

hdg_status_t hdg_prolong(hdg_handle_t h, int32_t p_fine, const double* e_coarse, double* x_fine) {
  if (!h || !e_coarse || !x_fine || p_fine < 1 || p_fine > h->k) return HDG_ERR_INVALID_ARG;
  return guarded(h, [&]() -> hdg_status_t {
    hipchk(hdg::launch_p_prolong_add(hdg::Prec::F64, p_fine + 1, h->pl[p_fine].pmat64, e_coarse, x_fine, h->nf,
                                     h->stream),
           "prolong");
    return HDG_OK;
  });
}

hdg_status_t hdg_fmg(hdg_handle_t h, const double* b, double* x, int32_t cycles) {
  if (!h || !b || !x || b == x || cycles < 1 || cycles > 64) return HDG_ERR_INVALID_ARG;
  return guarded(h, [&]() -> hdg_status_t {
    const int64_t N = h->pl[h->k].N;
    if (h->prec == hdg::Prec::F64) {
      fmg(h, b, x, cycles);
    } else {
      fmg(h, stage_in(h, b, h->cva, N), h->cvb, cycles);
      stage_out(h, h->cvb, x, N);
    }
    return HDG_OK;
  });
}

hdg_status_t hdg_vcycle(hdg_handle_t h, const double* b, double* x) {
  if (!h || !b || !x || b == x) return HDG_ERR_INVALID_ARG;
  return guarded(h, [&]() -> hdg_status_t {
    const int64_t N = h->pl[h->k].N;
    if (h->prec == hdg::Prec::F64) {
      pcycle(h, h->k, b, x, false);
    } else {
      const void* bl = stage_in(h, b, h->cva, N);
      pcycle(h, h->k, bl, const_cast<void*>(stage_in(h, x, h->cvb, N)), false);
      stage_out(h, h->cvb, x, N);
    }
    return HDG_OK;
  });
}

namespace {
hdg::ElemArgs elem_args(hdg_handle_t h) {
  hdg::ElemArgs a{};
  a.ref = h->ref_dev;
  a.kappa = h->kappa_dev;
  a.lam_bd = h->lambd_dev;
  a.F = h->F_dev;
  a.n = h->n;
  return a;
}
hdg_status_t need_source(hdg_handle_t h) {
  if (h->have_source) return HDG_OK;
  h->err = "no source state: call hdg_assemble_rhs first";
  return HDG_ERR_STATE;
}
}  // namespace

hdg_status_t hdg_reconstruct(hdg_handle_t h, const double* lam, double* U, double* Q) {
  if (!h || !lam || !U) return HDG_ERR_INVALID_ARG;
  if (need_source(h) != HDG_OK) return HDG_ERR_STATE;
  return guarded(h, [&]() -> hdg_status_t {
    hdg::ElemArgs a = elem_args(h);
    a.lam = lam;
    a.Uout = U;
    a.Qout = Q;
    hipchk(hdg::launch_elem_reconstruct(h->k + 1, a, h->stream), "reconstruct");
    return HDG_OK;
  });
}

hdg_status_t hdg_misfit_adjoint_rhs(hdg_handle_t h, const double* U, const double* U_obs, double* c,
                                    double* misfit_host) {
  if (!h || !U || !U_obs || !c) return HDG_ERR_INVALID_ARG;
  return guarded(h, [&]() -> hdg_status_t {
    const int64_t ne = (int64_t)h->n * h->n;
    const int P = h->k + 1;
    if (!h->elem_t) {
      h->elem_t = dalloc(h, ne * 4 * P);
      h->elem_m = dalloc(h, ne);
    }
    hdg::ElemArgs a = elem_args(h);
    a.U = U;
    a.Uobs = U_obs;
    a.tout = h->elem_t;
    a.misfit = h->elem_m;
    hipchk(hdg::launch_elem_adjoint(P, a, h->stream), "adjoint element");
    hipchk(hdg::launch_face_gather(P, h->elem_t, c, h->n, h->stream), "face gather");
    if (misfit_host) {
      hipchk(hdg::launch_sum_partials(h->elem_m, (int)ne, h->scal, h->stream), "sum");
      hipchk(hipMemcpyAsync(h->scal_h, h->scal, sizeof(double), hipMemcpyDeviceToHost, h->stream), "d2h");
      hipchk(hipStreamSynchronize(h->stream), "sync");
      *misfit_host = *h->scal_h;
    }
    return HDG_OK;
  });
}

hdg_status_t hdg_misfit_gradient(hdg_handle_t h, const double* lam, const double* U, const double* U_obs,
                                 const double* mu, double* grad) {
  if (!h || !lam || !U || !U_obs || !mu || !grad) return HDG_ERR_INVALID_ARG;
  if (need_source(h) != HDG_OK) return HDG_ERR_STATE;
  return guarded(h, [&]() -> hdg_status_t {
    hdg::ElemArgs a = elem_args(h);
    a.lam = lam;
    a.U = U;
    a.Uobs = U_obs;
    a.mu = mu;
    a.grad = grad;
    hipchk(hdg::launch_elem_gradient(h->k + 1, a, h->stream), "gradient");
    return HDG_OK;
  });
}

hdg_status_t hdg_solve_multi(hdg_handle_t h, int32_t nrhs, const double* B, double* X, double rtol, int32_t maxit,
                             int32_t* iters_host, double* relres_host) {
  if (!h || !B || !X || B == X || nrhs < 1 || nrhs > 256 || maxit < 0 || !(rtol >= 0.0))
    return HDG_ERR_INVALID_ARG;
  if (h->cfg.smoother != HDG_SMOOTH_CHAIN) {
    h->err = "the solve for many right-hand sides uses the chain smoother";
    return HDG_ERR_STATE;
  }
  return guarded(h, [&]() -> hdg_status_t {
    const int R = nrhs;
    MultiWork& W = multi_work(h, R);
    const int k = h->k;
    PLevel& Lk = h->pl[k];
    const int64_t N = Lk.N;
    hipStream_t s = h->stream;
    std::vector<double> nb(R), rn(R), act(R);
    std::vector<int> its(R, 0);
    auto host_col = [&](const double* dev, std::vector<double>& out) {
      hipchk(hipMemcpyAsync(out.data(), dev, R * sizeof(double), hipMemcpyDeviceToHost, s), "d2h");
      hipchk(hipStreamSynchronize(s), "sync");
    };
    hipchk(hdg::launch_dots_m(hdg::Prec::F64, B, B, N, R, W.partial, W.nb, s), "dots");
    host_col(W.nb, nb);
    {  // R0 = B - S X with the FP64 operator
      hdg::MultiArgs a = margs(h, Lk, R, true);
      a.X = X;
      a.B = B;
      a.Y = W.vr;
      hipchk(hdg::launch_trace_multi(hdg::Prec::F64, Lk.P, a, s, hdg::TM_RESID), "residual multi");
    }
    hipchk(hdg::launch_dots_m(hdg::Prec::F64, W.vr, W.vr, N, R, W.partial, W.nrm, s), "dots");
    host_col(W.nrm, rn);
    int nact = 0;
    for (int r = 0; r < R; ++r) {
      nb[r] = std::sqrt(nb[r]);
      rn[r] = std::sqrt(rn[r]);
      if (!std::isfinite(rn[r]) || !std::isfinite(nb[r])) {
        h->err = "non-finite residual";
        return HDG_ERR_NONFINITE;
      }
      act[r] = rn[r] > rtol * nb[r] ? 1.0 : 0.0;
      nact += act[r] > 0;
    }
    hipchk(hipMemcpyAsync(W.act, act.data(), R * sizeof(double), hipMemcpyHostToDevice, s), "h2d");
    double* sc = W.sc;  // [5][R]: d.r, d.q, z.q, z.r, d.r (previous direction)
    // As in hdg_solve: each phase runs FCG until every active column's recursive
    // residual is below its tolerance; then the true residuals B - S X are
    // recomputed, and a column above its tolerance restarts from its true residual
    // while each restart at least halves it (else it has reached the rounding
    // floor of S x and is reported as not converged).
    std::vector<double> last_true(rn);
    int it = 0;
    bool stalled = false;
    for (;;) {
      int itp = 0;
      while (nact > 0 && it < maxit) {
        precondition_m(h, W);
        if (itp == 0) {
          hipchk(hdg::launch_copy(hdg::Prec::F64, W.vz, W.vd, N * R, s), "copy");
          hipchk(hdg::launch_dots_m(hdg::Prec::F64, W.vz, W.vr, N, R, W.partial, sc, s), "dots");
        } else {
          hipchk(hdg::launch_dots_m(hdg::Prec::F64, W.vz, W.vq, N, R, W.partial, sc + 2 * R, s), "dots");
          hipchk(hdg::launch_dots_m(hdg::Prec::F64, W.vz, W.vr, N, R, W.partial, sc + 3 * R, s), "dots");
          hipchk(hdg::launch_dots_m(hdg::Prec::F64, W.vd, W.vr, N, R, W.partial, sc + 4 * R, s), "dots");
          hipchk(hdg::launch_fcg_scalars_m(sc, R, s), "fcg scalars");
          hipchk(hdg::launch_xpby_m(hdg::Prec::F64, W.vz, sc + 2 * R, sc + R, -1.0, W.vd, N, R, s), "xpby");
        }
        hdg::MultiArgs a = margs(h, Lk, R, true);
        a.X = W.vd;
        a.Y = W.vq;
        hipchk(hdg::launch_trace_multi(hdg::Prec::F64, Lk.P, a, s, hdg::TM_APPLY), "apply multi");
        hipchk(hdg::launch_dots_m(hdg::Prec::F64, W.vd, W.vq, N, R, W.partial, sc + R, s), "dots");
        hipchk(hdg::launch_axpy_m(hdg::Prec::F64, sc, sc + R, W.act, 1.0, W.vd, X, N, R, s), "axpy");
        hipchk(hdg::launch_axpy_m(hdg::Prec::F64, sc, sc + R, W.act, -1.0, W.vq, W.vr, N, R, s), "axpy");
        hipchk(hdg::launch_dots_m(hdg::Prec::F64, W.vr, W.vr, N, R, W.partial, W.nrm, s), "dots");
        host_col(W.nrm, rn);
        ++it;
        ++itp;
        nact = 0;
        for (int r = 0; r < R; ++r) {
          if (act[r] == 0.0) continue;
          const double v = std::sqrt(rn[r]);
          if (!std::isfinite(v)) {
            h->err = "non-finite residual";
            return HDG_ERR_NONFINITE;
          }
          its[r] = it;
          if (v <= rtol * nb[r]) act[r] = 0.0;
          else ++nact;
        }
        hipchk(hipMemcpyAsync(W.act, act.data(), R * sizeof(double), hipMemcpyHostToDevice, s), "h2d");
      }
      {  // true residuals R = B - S X with the FP64 operator
        hdg::MultiArgs a = margs(h, Lk, R, true);
        a.X = X;
        a.B = B;
        a.Y = W.vr;
        hipchk(hdg::launch_trace_multi(hdg::Prec::F64, Lk.P, a, s, hdg::TM_RESID), "residual multi");
      }
      hipchk(hdg::launch_dots_m(hdg::Prec::F64, W.vr, W.vr, N, R, W.partial, W.nrm, s), "dots");
      host_col(W.nrm, rn);
      nact = 0;
      stalled = false;
      for (int r = 0; r < R; ++r) {
        rn[r] = std::sqrt(rn[r]);
        if (!std::isfinite(rn[r])) {
          h->err = "non-finite residual";
          return HDG_ERR_NONFINITE;
        }
        act[r] = 0.0;
        if (rn[r] <= rtol * nb[r]) continue;
        if (it < maxit && rn[r] <= 0.5 * last_true[r]) {
          act[r] = 1.0;
          last_true[r] = rn[r];
          ++nact;
        } else {
          stalled = true;
        }
      }
      if (nact == 0) break;
      hipchk(hipMemcpyAsync(W.act, act.data(), R * sizeof(double), hipMemcpyHostToDevice, s), "h2d");
    }
    for (int r = 0; r < R; ++r) {
      if (iters_host) iters_host[r] = its[r];
      if (relres_host) relres_host[r] = nb[r] > 0 ? rn[r] / nb[r] : rn[r];
    }
    if (stalled) {
      h->err = "maximum number of iterations reached, or a true residual stalled above the tolerance";
      return HDG_ERR_NOT_CONVERGED;
    }
    return HDG_OK;
  });
}

hdg_status_t hdg_solve(hdg_handle_t h, const double* b, double* x, double rtol, int32_t maxit,
                       int32_t mode, int32_t* iters, double* relres, double* history_host) {
  if (!h || !b || !x || b == x || maxit < 0 || !(rtol >= 0.0) ||
      (mode != HDG_SOLVE_PCG && mode != HDG_SOLVE_VCYCLE && mode != HDG_SOLVE_FCG))
    return HDG_ERR_INVALID_ARG;
  if (mode == HDG_SOLVE_PCG)
    for (const PLevel& L : h->pl)
      if (L.inner > 0) {
        h->err = "a cycle with Krylov-accelerated levels is nonlinear: use HDG_SOLVE_FCG or HDG_SOLVE_VCYCLE";
        return HDG_ERR_INVALID_ARG;
      }
  return guarded(h, [&]() -> hdg_status_t {
    const int k = h->k;
    const int64_t N = h->pl[k].N;
    const double nb = std::sqrt(dot(h, b, b, N));
    double rn = residual_norm(h, k, b, x, h->vr);
    int it = 0;
    if (history_host) history_host[0] = rn;
    auto finish = [&](hdg_status_t s) {
      if (iters) *iters = it;
      if (relres) *relres = nb > 0 ? rn / nb : rn;
      return s;
    };
    if (!std::isfinite(rn) || !std::isfinite(nb)) {
      h->err = "non-finite residual";
      return finish(HDG_ERR_NONFINITE);
    }
    const double tol = rtol * nb;
    if (mode == HDG_SOLVE_VCYCLE) {
      // stationary iteration on the correction: x += B (b - S x), B one V-cycle
      while (rn > tol && it < maxit) {
        precondition(h);
        hipchk(hdg::launch_axpy(1.0, h->vz, x, N, h->stream), "axpy");
        rn = residual_norm(h, k, b, x, h->vr);
        ++it;
        if (history_host) history_host[it] = rn;
        if (!std::isfinite(rn)) {
          h->err = "non-finite residual";
          return finish(HDG_ERR_NONFINITE);
        }
      }
    } else if (rn > tol && maxit > 0) {
      // conjugate gradients (PCG), or flexible CG, FCG(1) (Notay): the direction is
      // A-orthogonalised against the previous one, d = z - (z . q / d . q) d, and
      // alpha = d . r / d . q with d . r = z . r - beta d_prev . r.
      // The loop stops on the recursively updated residual r <- r - alpha S d.  The
      // true residual b - S x is then recomputed; if it is still above tol, the
      // iteration restarts from it (residual replacement: h->vr holds b - S x)
      // unless it lies within twice the rounding floor u || |S| |x| || of the
      // computed residual (AT_FLOOR), or the previous restart failed to halve it
      // (NOT_CONVERGED).  rn, relres and the last history entry are the true value.
      const bool flex = mode == HDG_SOLVE_FCG;
      double last_true = rn;
      for (;;) {
        precondition(h);
        hipchk(hdg::launch_copy(hdg::Prec::F64, h->vz, h->vd, N, h->stream), "copy");
        double rz = dot(h, h->vr, h->vz, N);
        double dr = rz;
        while (rn > tol && it < maxit) {
          hdg::TraceArgs ta = targs(h, h->pl[k], hdg::Prec::F64);
          ta.x = h->vd;
          ta.y = h->vq;
          ta.partial = h->partial;
          hipchk(hdg::launch_trace(hdg::Prec::F64, h->pl[k].P, hdg::TM_APPLY_DOT, ta, h->stream), "apply dot");
          const double dq = reduce_scalar(h, hdg::trace_partials(h->ntiles));
          const double alpha = dr / dq;
          hipchk(hdg::launch_axpy(alpha, h->vd, x, N, h->stream), "axpy");
          hipchk(hdg::launch_axpy_norm(alpha, h->vq, h->vr, N, h->partial, h->stream), "axpy norm");
          rn = std::sqrt(reduce_scalar(h, hdg::reduce_grid(N)));
          ++it;
          if (history_host) history_host[it] = rn;
          if (!std::isfinite(rn)) {
            h->err = "non-finite residual";
            return finish(HDG_ERR_NONFINITE);
          }
          if (rn <= tol) break;
          precondition(h);
          if (flex) {
            double v[3];
            dots(h, hdg::Prec::F64, 3, {h->vz, h->vq, h->vz, h->vr, h->vd, h->vr}, N, v);
            const double beta = v[0] / dq;
            hipchk(hdg::launch_xpby(h->vz, -beta, h->vd, N, h->stream), "xpby");
            dr = v[1] - beta * v[2];
          } else {
            const double rz_new = dot(h, h->vr, h->vz, N);
            hipchk(hdg::launch_xpby(h->vz, rz_new / rz, h->vd, N, h->stream), "xpby");
            rz = rz_new;
            dr = rz;
          }
        }
        rn = residual_norm(h, k, b, x, h->vr);
        if (history_host) history_host[it] = rn;
        if (!std::isfinite(rn)) {
          h->err = "non-finite residual";
          return finish(HDG_ERR_NONFINITE);
        }
        if (rn <= tol || it >= maxit) break;
        // rounding floor of the computed residual: u || |S| |x| ||, u = 2^-53
        hdg::TraceArgs fa = targs(h, h->pl[k], hdg::Prec::F64);
        fa.x = x;
        fa.y = h->vq;
        hipchk(hdg::launch_trace(hdg::Prec::F64, h->pl[k].P, hdg::TM_ABS, fa, h->stream), "trace abs");
        const double floor_rn = 0x1p-53 * std::sqrt(dot(h, h->vq, h->vq, N));
        if (rn <= 2.0 * floor_rn) {
          h->err = "the true residual b - S x is within twice its rounding floor, above the tolerance";
          return finish(HDG_ERR_AT_FLOOR);
        }
        if (!(rn <= 0.5 * last_true)) {
          h->err = "the true residual b - S x stalled above the tolerance";
          return finish(HDG_ERR_NOT_CONVERGED);
        }
        last_true = rn;
      }
    }
    if (rn > tol) {
      h->err = "maximum number of iterations reached";
      return finish(HDG_ERR_NOT_CONVERGED);
    }
    return finish(HDG_OK);
  });
}

}  // extern "C"
