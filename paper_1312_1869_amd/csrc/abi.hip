// C ABI (include/lrinv.h): argument checks, workspace layout, launch order.
// Every check runs on the host before the first launch, so an argument error
// writes nothing. All work is enqueued on the caller's stream; nothing here
// synchronises or allocates.
#include <math.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "lrinv.h"

using namespace lr;

namespace {

constexpr int kMaxDevices = 64;
int g_num_cu[kMaxDevices];
std::once_flag g_cu_once[kMaxDevices];

int num_cu_current() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 256;
  std::call_once(g_cu_once[dev], [dev]() {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    g_num_cu[dev] = v;
  });
  return g_num_cu[dev];
}

// Scratch of lr_sketch_noalloc: a file-scope device array (each GPU the
// library runs on holds its own copy until the process ends). In host code
// the name is only a host-side stand-in; the device address comes from
// hipGetSymbolAddress, once per device, and is the only thing passed to
// kernels.
constexpr size_t kNoAllocBytes = LR_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char lr_scratch[kNoAllocBytes];
void* g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];
std::once_flag g_scratch_once[kMaxDevices];

// Device address of this GPU's scratch array (nullptr on failure).
void* scratch_current() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::call_once(g_scratch_once[dev], [dev]() {
    void* ptr = nullptr;
    g_scratch_err[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(lr_scratch));
    g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? ptr : nullptr;
  });
  return g_scratch_ptr[dev];
}

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }
bool is_fin(double x) { return isfinite(x) != 0; }
bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }
size_t real_size(int32_t prec) { return prec == LR_PREC_F64 ? 8 : 4; }
bool valid_prec(int32_t prec) {
  return prec == LR_PREC_F64 || prec == LR_PREC_F32 || prec == LR_PREC_BF16 || prec == LR_PREC_BF16X2;
}
bool bf16_sketch(int32_t prec) { return prec == LR_PREC_BF16 || prec == LR_PREC_BF16X2; }

lr_status check_ws(size_t need, const void* ws, size_t ws_bytes) {
  if (need == 0) return LR_OK;
  if (ws == nullptr || ws_bytes < need || !aligned(ws, 256)) return LR_ERR_WORKSPACE;
  return LR_OK;
}

lr_status check_hyper(const lr_hyper* h) {
  if (h == nullptr) return LR_ERR_ARG;
  if (h->kernel != LR_KERNEL_SE && h->kernel != LR_KERNEL_MATERN32) return LR_ERR_ARG;
  if (h->reserved != 0) return LR_ERR_ARG;
  if (!is_fin(h->ell) || !(h->ell > 0.0) || !is_fin(h->s) || h->s < 0.0) return LR_ERR_ARG;
  return LR_OK;
}

lr_status check_omega(const lr_omega* o, int64_t n, int32_t d, int32_t prec) {
  if (o == nullptr) return LR_ERR_ARG;
  if (o->n != n || o->d != d) return LR_ERR_SHAPE;
  if (o->kind == LR_OMEGA_SRHT) {
    if ((n & (n - 1)) != 0) return LR_ERR_NOT_POW2;
    if (o->signs == nullptr || o->cols == nullptr) return LR_ERR_ARG;
    if (bf16_sketch(prec)) return LR_ERR_UNSUPPORTED;
    return LR_OK;
  }
  if (o->kind == LR_OMEGA_GAUSS) {
    if (o->dense_t == nullptr || !aligned(o->dense_t, 16)) return LR_ERR_ARG;
    if (o->ld < n || o->ld % 8 != 0) return LR_ERR_SHAPE;
    // the bf16 sketch addresses Omega through 31-bit buffer extents
    if (bf16_sketch(prec) && n > ((int64_t)1 << 25)) return LR_ERR_UNSUPPORTED;
    return LR_OK;
  }
  return LR_ERR_ARG;
}

lr_status check_sizes(int64_t n, int32_t d) {
  if (n < 1 || d < 1 || d > 1024 || (int64_t)d > n) return LR_ERR_SHAPE;
  if (n > ((int64_t)1 << 40)) return LR_ERR_SHAPE;
  return LR_OK;
}

TnOperand omega_operand(const lr_omega* o, int32_t prec, double* scale) {
  TnOperand op{};
  if (o->kind == LR_OMEGA_SRHT) {
    op.kind = 2;
    op.signs = o->signs;
    op.cols = o->cols;
    *scale = 1.0 / sqrt((double)o->n);
  } else {
    op.kind = 1;
    op.dtype = prec == LR_PREC_F64 ? 0 : (prec == LR_PREC_F32 ? 1 : 2);
    op.ptr = o->dense_t;
    op.ld = o->ld;
    *scale = 1.0;
  }
  return op;
}

TnOperand real_operand(const void* p, int64_t ld, int32_t prec) {
  TnOperand op{};
  op.kind = 0;
  op.dtype = prec == LR_PREC_F64 ? 0 : 1;
  op.ptr = p;
  op.ld = ld;
  return op;
}

#define LR_HIP(x)                            \
  do {                                       \
    if ((x) != hipSuccess) return LR_ERR_HIP; \
  } while (0)

// ---------------------------------------------------------------- sketch

// prescaled points, padded with kPointPad zero rows so kernels may read a
// whole step of columns past n without a bounds check
size_t sketch_pts_bytes(int64_t n, int32_t D, int32_t prec) {
  return al((size_t)(n + kPointPad) * point_stride(D) * real_size(prec));
}

// prescaled points; for the bf16 sketch with D <= 3 also the fragment-order
// copy of a Gaussian Omega
size_t sketch_ws(int64_t n, int32_t D, int32_t d, int32_t prec) {
  size_t b = sketch_pts_bytes(n, D, prec);
  if (bf16_sketch(prec) && D <= 3) b += al(omega_frag_bytes(n, d));
  return b;
}

lr_status sketch_impl(hipStream_t st, int64_t n, int32_t D, const float* X, const lr_hyper* hyp,
                      const lr_omega* omega, double nu, int32_t prec, void* Y, void* Yp, void* ws) {
  const int PD = point_stride(D);
  const double scale = coord_scale(hyp->kernel, hyp->ell);
  const double s2 = hyp->s * hyp->s;
  const int ncu = num_cu_current();
  const int d = omega->d;
  if (omega->kind == LR_OMEGA_SRHT) {
    const double c = 1.0 / sqrt((double)n);
    if (prec == LR_PREC_F64) {
      double* pts = static_cast<double*>(ws);
      LR_HIP(launch_prep_points<double>(st, X, n, D, PD, scale, omega->signs, pts));
      LR_HIP(launch_sketch_srht<double>(st, hyp->kernel, D, pts, omega->cols, n, d, c * s2, nu * c,
                                        static_cast<double*>(Y), static_cast<double*>(Yp), ncu));
    } else {
      float* pts = static_cast<float*>(ws);
      LR_HIP(launch_prep_points<float>(st, X, n, D, PD, scale, omega->signs, pts));
      LR_HIP(launch_sketch_srht<float>(st, hyp->kernel, D, pts, omega->cols, n, d, c * s2, nu * c,
                                       static_cast<float*>(Y), static_cast<float*>(Yp), ncu));
    }
    return LR_OK;
  }
  if (prec == LR_PREC_F64) {
    LR_HIP(launch_prep_points<double>(st, X, n, D, PD, scale, nullptr, static_cast<double*>(ws)));
  } else {
    LR_HIP(launch_prep_points<float>(st, X, n, D, PD, scale, nullptr, static_cast<float*>(ws)));
  }
  void* frag = nullptr;
  if (bf16_sketch(prec) && D <= 3) {
    frag = static_cast<char*>(ws) + sketch_pts_bytes(n, D, prec);
    LR_HIP(launch_omega_frag(st, omega->dense_t, omega->ld, n, d, frag));
  }
  if (Y != nullptr)
    LR_HIP(launch_sketch_dense(st, prec, hyp->kernel, D, ws, omega->dense_t, omega->ld, n, d, s2, nu, Y, false, frag,
                               ncu));
  if (Yp != nullptr)
    LR_HIP(launch_sketch_dense(st, prec, hyp->kernel, D, ws, omega->dense_t, omega->ld, n, d, s2, 0.0, Yp, true, frag,
                               ncu));
  return LR_OK;
}

// ---------------------------------------------------------------- lowrank solve

struct SolveWs {
  size_t off_f, off_z, off_w, off_wm, off_tn, total;
};

SolveWs solve_layout(int64_t n, int32_t d, int32_t m) {
  SolveWs w;
  const size_t dm = (size_t)d * (m > 0 ? m : 1) * 8;
  size_t off = 0;
  w.off_f = off;
  off = al(off + (size_t)d * d * 8);
  w.off_z = off;
  off = al(off + dm);
  w.off_w = off;
  off = al(off + dm);
  w.off_wm = off;
  off = al(off + dm);
  w.off_tn = off;
  size_t tn = tn_workspace(n, d, d);
  if (m > 0) {
    size_t t2 = tn_workspace(n, d, m);
    if (t2 > tn) tn = t2;
  }
  off = al(off + tn);
  w.total = off;
  return w;
}

// Z = Q^T A (float64 sums of exact products), W = S^{-1} Z, Wmix = W - Z/sigma2
// (d x m float64 each).
lr_status project_solve(hipStream_t st, int64_t n, int32_t d, int32_t m, int32_t prec, const void* Q,
                        const double* L, double sigma2, const int32_t* info, const void* A, double* Z, double* W,
                        double* Wmix, void* tnws) {
  LR_HIP(launch_gemm_tn(st, n, d, m, real_operand(Q, d, prec), real_operand(A, m, prec), 1.0, Z, tnws, true));
  LR_HIP(launch_core_apply(st, d, m, L, Z, sigma2, info, W, Wmix));
  return LR_OK;
}

// X = K~^{-1} A = A/sigma2 + Q Wmix given Q and the Cholesky factor, in float64
// and rounded once to the working precision.
lr_status woodbury_apply(hipStream_t st, int64_t n, int32_t d, int32_t m, int32_t prec, const void* Q,
                         const double* L, double sigma2, const int32_t* info, const void* A, void* X, double* Z,
                         double* W, double* Wmix, void* tnws) {
  if (m <= 0) return LR_OK;
  lr_status s = project_solve(st, n, d, m, prec, Q, L, sigma2, info, A, Z, W, Wmix, tnws);
  if (s != LR_OK) return s;
  LR_HIP(launch_rowmix_info(st, n, d, m, Q, Wmix, 1.0 / sigma2, A, X, prec == LR_PREC_F64, info));
  return LR_OK;
}

// ---------------------------------------------------------------- backward

struct BackWs {
  size_t off_yp, off_sk, off_tn, off_za, off_wa, off_xa, off_zb, off_wb, off_xb, off_u64, off_b64, off_e, off_p,
      off_phi, off_sinv, off_t, off_g2, off_h, off_u, off_eu, off_ca, off_aa, off_xy, off_by, off_xbm, off_u1, off_u2,
      off_eu1, off_eu2, off_cqb, off_oo, off_v1, off_pta, off_oa, off_fa, off_oou, off_m1, off_m2, off_z1, off_z2,
      off_ox, off_ob, off_fqx, off_fqb, off_oou2, off_tdm, total;
};

BackWs back_layout(int64_t n, int32_t D, int32_t d, int32_t m, int32_t prec) {
  BackWs w;
  const size_t rs = real_size(prec);
  const size_t mm = m > 0 ? (size_t)m : 1;
  const size_t dd8 = (size_t)d * d * 8, dm8 = (size_t)d * mm * 8;
  size_t off = 0;
  auto take = [&](size_t& field, size_t bytes) {
    field = off;
    off = al(off + bytes);
  };
  take(w.off_yp, (size_t)n * d * rs);
  take(w.off_sk, sketch_ws(n, D, d, prec));
  const int big = (int)(mm > (size_t)d ? mm : (size_t)d);
  take(w.off_tn, tn_workspace(n, big, big));
  take(w.off_za, dm8);
  take(w.off_wa, dm8);
  take(w.off_xa, dm8);
  take(w.off_zb, dm8);
  take(w.off_wb, dm8);
  take(w.off_xb, dm8);
  take(w.off_u64, (size_t)n * mm * 8);
  take(w.off_b64, (size_t)n * mm * 8);
  take(w.off_e, dd8);
  take(w.off_p, dd8);
  take(w.off_phi, dd8);
  take(w.off_sinv, dd8);
  take(w.off_t, dd8);
  take(w.off_g2, dd8);
  take(w.off_h, (size_t)d * 8);
  take(w.off_u, (size_t)d * 8);
  take(w.off_eu, (size_t)d * 8);
  take(w.off_ca, (size_t)d * 8);
  take(w.off_aa, 8);
  take(w.off_xy, dm8);
  take(w.off_by, dm8);
  take(w.off_xbm, mm * mm * 8);
  take(w.off_u1, dm8);
  take(w.off_u2, dm8);
  take(w.off_eu1, dm8);
  take(w.off_eu2, dm8);
  take(w.off_cqb, dm8);
  // shift terms
  take(w.off_oo, dd8);
  take(w.off_v1, (size_t)d * 8);
  take(w.off_pta, (size_t)d * 8);
  take(w.off_oa, (size_t)d * 8);
  take(w.off_fa, (size_t)d * 8);
  take(w.off_oou, (size_t)d * 8);
  take(w.off_m1, dm8);
  take(w.off_m2, dm8);
  take(w.off_z1, dm8);
  take(w.off_z2, dm8);
  take(w.off_ox, dm8);
  take(w.off_ob, dm8);
  take(w.off_fqx, dm8);
  take(w.off_fqb, dm8);
  take(w.off_oou2, dm8);
  take(w.off_tdm, dm8);
  w.total = off;
  return w;
}

TnOperand f64_operand(const double* p, int64_t ld) {
  TnOperand op{};
  op.kind = 0;
  op.dtype = 0;
  op.ptr = p;
  op.ld = ld;
  return op;
}

// ---------------------------------------------------------------- projection variant

// the float64 second pass for F64, float32 for the float and bf16 paths (Q is float)
int32_t projection_pass_prec(int32_t prec) { return prec == LR_PREC_F64 ? LR_PREC_F64 : LR_PREC_F32; }
// Newton-Schulz steps of the PSD part: an eigenvalue of B / ||B||_F down to
// ~1e-13 reaches its sign (x1.5 per step while small, then quadratically)
constexpr int kPsdSteps = 96;

struct ProjWs {
  size_t off_pts, off_qt, off_y2, off_b, off_psd, off_solve, total;
  SolveWs solve;
  int64_t ld;
};

ProjWs proj_layout(int64_t n, int32_t D, int32_t d, int32_t m, int32_t prec) {
  ProjWs w;
  const int32_t p2 = projection_pass_prec(prec);
  const size_t es = real_size(p2);
  w.ld = (n + 63) / 64 * 64;
  size_t off = 0;
  w.off_pts = off;
  off = al(off + sketch_pts_bytes(n, D, p2));
  w.off_qt = off;
  off = al(off + (size_t)d * w.ld * es);
  w.off_y2 = off;
  off = al(off + (size_t)n * d * es);
  w.off_b = off;
  off = al(off + (size_t)d * d * 8);
  w.off_psd = off;
  off = al(off + (size_t)3 * d * d * 8);
  w.off_solve = off;
  w.solve = solve_layout(n, d, m);
  w.total = off + w.solve.total;
  return w;
}

lr_status projection_impl(hipStream_t st, int64_t n, int32_t D, int32_t d, const float* X, const lr_hyper* hyp,
                          int32_t prec, const void* Q, double sigma2, int32_t clip, int32_t m, const void* A,
                          void* Xout, double* B, double* L, double* logdet, int32_t* info, void* ws) {
  const ProjWs w = proj_layout(n, D, d, m, prec);
  const int32_t p2 = projection_pass_prec(prec);
  const bool f64 = p2 == LR_PREC_F64;
  char* base = static_cast<char*>(ws);
  void* pts = base + w.off_pts;
  void* qt = base + w.off_qt;
  void* y2 = base + w.off_y2;
  double* b0 = reinterpret_cast<double*>(base + w.off_b);
  double* psd = reinterpret_cast<double*>(base + w.off_psd);
  char* sb = base + w.off_solve;
  double* Z = reinterpret_cast<double*>(sb + w.solve.off_z);
  double* W = reinterpret_cast<double*>(sb + w.solve.off_w);
  double* Wm = reinterpret_cast<double*>(sb + w.solve.off_wm);
  void* tn = sb + w.solve.off_tn;
  const int PD = point_stride(D);
  const double scale = coord_scale(hyp->kernel, hyp->ell);
  if (f64)
    LR_HIP(launch_prep_points<double>(st, X, n, D, PD, scale, nullptr, static_cast<double*>(pts)));
  else
    LR_HIP(launch_prep_points<float>(st, X, n, D, PD, scale, nullptr, static_cast<float*>(pts)));
  // second pass Y2 = K_f Q, with Q^T in the transposed dense-Omega layout
  LR_HIP(launch_transpose(st, n, d, Q, w.ld, qt, f64));
  LR_HIP(launch_sketch_dense(st, p2, hyp->kernel, D, pts, qt, w.ld, n, d, hyp->s * hyp->s, 0.0, y2, false, nullptr,
                             num_cu_current()));
  // B = Q^T K_f Q, summed exactly in float64, then exactly symmetric
  LR_HIP(launch_gemm_tn(st, n, d, d, real_operand(Q, d, p2), real_operand(y2, d, p2), 1.0, b0, tn, true));
  LR_HIP(launch_symmetrize(st, d, b0));
  if (clip)
    LR_HIP(launch_psd_part(st, d, b0, B, psd, kPsdSteps));
  else
    LR_HIP(hipMemcpyAsync(B, b0, (size_t)d * d * sizeof(double), hipMemcpyDeviceToDevice, st));
  LR_HIP(launch_chol_core(st, n, d, B, sigma2, L, logdet, info));
  return woodbury_apply(st, n, d, m, p2, Q, L, sigma2, info, A, Xout, Z, W, Wm, tn);
}

}  // namespace

extern "C" {

int32_t lr_version(void) { return (2 << 16) | 1; }

const char* lr_status_string(int32_t s) {
  switch (s) {
    case LR_OK: return "LR_OK";
    case LR_ERR_ARG: return "LR_ERR_ARG";
    case LR_ERR_SHAPE: return "LR_ERR_SHAPE";
    case LR_ERR_NOT_POW2: return "LR_ERR_NOT_POW2";
    case LR_ERR_WORKSPACE: return "LR_ERR_WORKSPACE";
    case LR_ERR_HIP: return "LR_ERR_HIP";
    case LR_ERR_UNSUPPORTED: return "LR_ERR_UNSUPPORTED";
    case LR_ERR_SCRATCH_LIMIT: return "LR_ERR_SCRATCH_LIMIT";
    default: return "LR_UNKNOWN_STATUS";
  }
}

lr_status lr_check_srht_cols(const int32_t* cols, int32_t d, int64_t n) {
  if (cols == nullptr || d < 1 || n < 1) return LR_ERR_ARG;
  // distinctness by a sorted copy would allocate; d <= 1024 so a quadratic scan is fine
  for (int32_t i = 0; i < d; ++i) {
    if (cols[i] < 0 || (int64_t)cols[i] >= n) return LR_ERR_ARG;
    for (int32_t j = 0; j < i; ++j)
      if (cols[j] == cols[i]) return LR_ERR_ARG;
  }
  return LR_OK;
}

lr_status lr_structured_omega(void* stream, int32_t transform, int64_t n, int32_t d, const int8_t* signs,
                              const int32_t* cols, int32_t prec, void* omega_t, int64_t ld) {
  if (transform != LR_TRANSFORM_DCT && transform != LR_TRANSFORM_DHT && transform != LR_TRANSFORM_WHT)
    return LR_ERR_ARG;
  if (!valid_prec(prec)) return LR_ERR_ARG;
  lr_status s = check_sizes(n, d);
  if (s != LR_OK) return s;
  if (n > ((int64_t)1 << 30)) return LR_ERR_SHAPE;  // (2j+1) p stays below 2^62
  if (ld < n || ld % 8 != 0) return LR_ERR_SHAPE;
  if (transform == LR_TRANSFORM_WHT && (n & (n - 1)) != 0) return LR_ERR_NOT_POW2;
  if (signs == nullptr || cols == nullptr || omega_t == nullptr || !aligned(omega_t, 16)) return LR_ERR_ARG;
  LR_HIP(launch_structured_omega(static_cast<hipStream_t>(stream), transform, n, d, signs, cols, prec, omega_t, ld,
                                 num_cu_current()));
  return LR_OK;
}

size_t lr_sketch_workspace_bytes(int64_t n, int32_t D, int32_t d, int32_t prec) {
  if (n < 1 || D < 1 || D > 15 || !valid_prec(prec)) return 0;
  return sketch_ws(n, D, d, prec);
}

lr_status lr_sketch(void* stream, int64_t n, int32_t D, const float* X, const lr_hyper* hyp, const lr_omega* omega,
                    double nu, int32_t prec, void* Y, void* Yprime, void* ws, size_t ws_bytes) {
  if (!valid_prec(prec)) return LR_ERR_ARG;
  if (D < 1 || D > 15) return LR_ERR_SHAPE;
  if (omega == nullptr) return LR_ERR_ARG;
  lr_status s = check_sizes(n, omega->d);
  if (s != LR_OK) return s;
  if (X == nullptr || (Y == nullptr && Yprime == nullptr)) return LR_ERR_ARG;
  if ((s = check_hyper(hyp)) != LR_OK) return s;
  if ((s = check_omega(omega, n, omega->d, prec)) != LR_OK) return s;
  if (prec == LR_PREC_BF16X2 && D > 3) return LR_ERR_UNSUPPORTED;
  if (!is_fin(nu) || nu < 0.0) return LR_ERR_ARG;
  if ((s = check_ws(sketch_ws(n, D, omega->d, prec), ws, ws_bytes)) != LR_OK) return s;
  return sketch_impl(static_cast<hipStream_t>(stream), n, D, X, hyp, omega, nu, prec, Y, Yprime, ws);
}

size_t lr_sketch_grid_workspace_bytes(int64_t n, int32_t D, int32_t d, int32_t prec) {
  return lr_sketch_workspace_bytes(n, D, d, prec);
}

lr_status lr_sketch_grid(void* stream, int64_t n, int32_t D, const float* X, int32_t ntheta, const lr_hyper* hyps,
                         const lr_omega* omega, double nu, int32_t prec, void* Y, void* ws, size_t ws_bytes) {
  if (!valid_prec(prec)) return LR_ERR_ARG;
  if (D < 1 || D > 15) return LR_ERR_SHAPE;
  if (omega == nullptr || hyps == nullptr || X == nullptr || Y == nullptr) return LR_ERR_ARG;
  if (ntheta < 1 || ntheta > 4096) return LR_ERR_SHAPE;
  lr_status s = check_sizes(n, omega->d);
  if (s != LR_OK) return s;
  for (int32_t g = 0; g < ntheta; ++g) {
    if ((s = check_hyper(&hyps[g])) != LR_OK) return s;
    if (hyps[g].kernel != hyps[0].kernel) return LR_ERR_ARG;
  }
  if ((s = check_omega(omega, n, omega->d, prec)) != LR_OK) return s;
  if (!is_fin(nu) || nu < 0.0) return LR_ERR_ARG;
  if (prec == LR_PREC_BF16X2 && D > 3) return LR_ERR_UNSUPPORTED;
  if ((s = check_ws(sketch_ws(n, D, omega->d, prec), ws, ws_bytes)) != LR_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int d = omega->d;
  const size_t es = prec == LR_PREC_F64 ? sizeof(double) : sizeof(float);
  if (omega->kind != LR_OMEGA_SRHT) {
    for (int32_t g = 0; g < ntheta; ++g) {
      void* yg = static_cast<char*>(Y) + (size_t)g * n * d * es;
      if ((s = sketch_impl(st, n, D, X, &hyps[g], omega, nu, prec, yg, nullptr, ws)) != LR_OK) return s;
    }
    return LR_OK;
  }
  // SRHT: points prescaled once for ell = 1; kernel g scales the squared
  // distance by 1/ell_g^2 and its output by c s_g^2
  const int PD = point_stride(D);
  const double c = 1.0 / sqrt((double)n);
  std::vector<double> a(ntheta), so(ntheta);
  for (int32_t g = 0; g < ntheta; ++g) {
    a[g] = 1.0 / (hyps[g].ell * hyps[g].ell);
    so[g] = c * hyps[g].s * hyps[g].s;
  }
  const double scale1 = coord_scale(hyps[0].kernel, 1.0);
  const int ncu = num_cu_current();
  if (prec == LR_PREC_F64) {
    double* pts = static_cast<double*>(ws);
    LR_HIP(launch_prep_points<double>(st, X, n, D, PD, scale1, omega->signs, pts));
    LR_HIP(launch_sketch_srht_grid<double>(st, hyps[0].kernel, D, pts, omega->cols, n, d, ntheta, a.data(),
                                           so.data(), nu * c, static_cast<double*>(Y), ncu));
  } else {
    float* pts = static_cast<float*>(ws);
    LR_HIP(launch_prep_points<float>(st, X, n, D, PD, scale1, omega->signs, pts));
    LR_HIP(launch_sketch_srht_grid<float>(st, hyps[0].kernel, D, pts, omega->cols, n, d, ntheta, a.data(),
                                          so.data(), nu * c, static_cast<float*>(Y), ncu));
  }
  return LR_OK;
}

lr_status lr_sketch_noalloc(void* stream, int64_t n, int32_t D, const float* X, const lr_hyper* hyp,
                            const lr_omega* omega, double nu, int32_t prec, void* Y, void* Yprime) {
  if (!valid_prec(prec)) return LR_ERR_ARG;
  if (D < 1 || D > 15) return LR_ERR_SHAPE;
  if (omega == nullptr) return LR_ERR_ARG;
  lr_status s = check_sizes(n, omega->d);
  if (s != LR_OK) return s;
  if (X == nullptr || (Y == nullptr && Yprime == nullptr)) return LR_ERR_ARG;
  if ((s = check_hyper(hyp)) != LR_OK) return s;
  if ((s = check_omega(omega, n, omega->d, prec)) != LR_OK) return s;
  if (!is_fin(nu) || nu < 0.0) return LR_ERR_ARG;
  // the bf16 matrix-core sketch with D <= 3 reads a 2 n d byte operand copy of Omega
  if (bf16_sketch(prec) && D <= 3 && omega->kind == LR_OMEGA_GAUSS) return LR_ERR_UNSUPPORTED;
  if (prec == LR_PREC_BF16X2 && D > 3) return LR_ERR_UNSUPPORTED;
  if (sketch_ws(n, D, omega->d, prec) > kNoAllocBytes) return LR_ERR_SCRATCH_LIMIT;
  void* ws = scratch_current();
  if (ws == nullptr) return LR_ERR_HIP;
  return sketch_impl(static_cast<hipStream_t>(stream), n, D, X, hyp, omega, nu, prec, Y, Yprime, ws);
}

size_t lr_tsqr_workspace_bytes(int64_t n, int32_t d, int32_t leaf_rows, int32_t prec) {
  if (check_sizes(n, d) != LR_OK || leaf_rows < d || leaf_rows > 8192 || !valid_prec(prec)) return 0;
  return tsqr_workspace(n, d, leaf_rows, prec == LR_PREC_F64);
}

lr_status lr_tsqr(void* stream, int64_t n, int32_t d, int32_t leaf_rows, int32_t prec, const void* Y, void* Q,
                  double* R, void* ws, size_t ws_bytes) {
  if (!valid_prec(prec)) return LR_ERR_ARG;
  lr_status s = check_sizes(n, d);
  if (s != LR_OK) return s;
  if (leaf_rows < d || leaf_rows > 8192) return LR_ERR_SHAPE;
  const int64_t nleaf = (n + leaf_rows - 1) / leaf_rows;
  if (n - (nleaf - 1) * leaf_rows < d) return LR_ERR_SHAPE;
  if (Y == nullptr || Q == nullptr || R == nullptr) return LR_ERR_ARG;
  if ((s = check_ws(tsqr_workspace(n, d, leaf_rows, prec == LR_PREC_F64), ws, ws_bytes)) != LR_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (prec == LR_PREC_F64)
    e = tsqr_run<double>(st, n, d, leaf_rows, static_cast<const double*>(Y), static_cast<double*>(Q), R, ws);
  else
    e = tsqr_run<float>(st, n, d, leaf_rows, static_cast<const float*>(Y), static_cast<float*>(Q), R, ws);
  return e == hipSuccess ? LR_OK : LR_ERR_HIP;
}

size_t lr_tsqr_tree_workspace_bytes(int64_t n, int32_t d, int32_t leaf_rows, int32_t group, int32_t prec) {
  if (!valid_prec(prec) || check_sizes(n, d) != LR_OK || leaf_rows < d || leaf_rows > 8192 || group < 1) return 0;
  if (group == 1) return tsqr_workspace(n, d, leaf_rows, prec == LR_PREC_F64);
  if (n % leaf_rows != 0 || (n / leaf_rows) % group != 0 || d + leaf_rows > 8192) return 0;
  return tsqr_domino_workspace(n, d, leaf_rows, group, prec == LR_PREC_F64);
}

lr_status lr_tsqr_tree(void* stream, int64_t n, int32_t d, int32_t leaf_rows, int32_t group, int32_t prec,
                       const void* Y, void* Q, double* R, void* ws, size_t ws_bytes) {
  if (!valid_prec(prec)) return LR_ERR_ARG;
  lr_status s = check_sizes(n, d);
  if (s != LR_OK) return s;
  if (leaf_rows < d || leaf_rows > 8192 || group < 1) return LR_ERR_SHAPE;
  const int64_t nleaf = (n + leaf_rows - 1) / leaf_rows;
  if (group == 1) {
    if (n - (nleaf - 1) * leaf_rows < d) return LR_ERR_SHAPE;
  } else {
    if (n % leaf_rows != 0 || nleaf % group != 0 || d + leaf_rows > 8192) return LR_ERR_SHAPE;
  }
  if (Y == nullptr || R == nullptr) return LR_ERR_ARG;
  if ((s = check_ws(lr_tsqr_tree_workspace_bytes(n, d, leaf_rows, group, prec), ws, ws_bytes)) != LR_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (prec == LR_PREC_F64) {
    e = group == 1 ? tsqr_run<double>(st, n, d, leaf_rows, static_cast<const double*>(Y), static_cast<double*>(Q), R,
                                      ws)
                   : tsqr_domino_run<double>(st, n, d, leaf_rows, group, static_cast<const double*>(Y),
                                             static_cast<double*>(Q), R, ws);
  } else {
    e = group == 1 ? tsqr_run<float>(st, n, d, leaf_rows, static_cast<const float*>(Y), static_cast<float*>(Q), R, ws)
                   : tsqr_domino_run<float>(st, n, d, leaf_rows, group, static_cast<const float*>(Y),
                                            static_cast<float*>(Q), R, ws);
  }
  return e == hipSuccess ? LR_OK : LR_ERR_HIP;
}

size_t lr_lowrank_solve_workspace_bytes(int64_t n, int32_t d, int32_t m, int32_t prec) {
  if (check_sizes(n, d) != LR_OK || m < 0 || m > 64 || !valid_prec(prec)) return 0;
  return solve_layout(n, d, m).total;
}

lr_status lr_lowrank_solve(void* stream, int64_t n, int32_t d, int32_t m, const lr_omega* omega, int32_t prec,
                           const void* Q, const double* R, double sigma2, double nu, const void* A, void* X,
                           double* C, double* L, double* Flu, int32_t* piv, double* logdet, int32_t* info, void* ws,
                           size_t ws_bytes) {
  if (!valid_prec(prec)) return LR_ERR_ARG;
  lr_status s = check_sizes(n, d);
  if (s != LR_OK) return s;
  if (m < 0 || m > 64) return LR_ERR_SHAPE;
  if ((s = check_omega(omega, n, d, prec)) != LR_OK) return s;
  if (!is_fin(sigma2) || !(sigma2 > 0.0) || !is_fin(nu) || nu < 0.0) return LR_ERR_ARG;
  if (Q == nullptr || R == nullptr || C == nullptr || L == nullptr || Flu == nullptr || piv == nullptr ||
      logdet == nullptr || info == nullptr)
    return LR_ERR_ARG;
  if (m > 0 && (A == nullptr || X == nullptr || A == X)) return LR_ERR_ARG;
  const SolveWs w = solve_layout(n, d, m);
  if ((s = check_ws(w.total, ws, ws_bytes)) != LR_OK) return s;

  hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  double* F = reinterpret_cast<double*>(base + w.off_f);
  double* Z = reinterpret_cast<double*>(base + w.off_z);
  double* W = reinterpret_cast<double*>(base + w.off_w);
  double* Wm = reinterpret_cast<double*>(base + w.off_wm);
  void* tn = base + w.off_tn;
  const bool f64 = prec == LR_PREC_F64;
  double oscale = 1.0;
  const TnOperand om = omega_operand(omega, prec, &oscale);
  LR_HIP(launch_gemm_tn(st, n, d, d, om, real_operand(Q, d, prec), oscale, F, tn, f64));
  LR_HIP(launch_core(st, n, d, F, R, sigma2, nu, Flu, piv, C, L, logdet, info));
  return woodbury_apply(st, n, d, m, prec, Q, L, sigma2, info, A, X, Z, W, Wm, tn);
}

size_t lr_projection_solve_workspace_bytes(int64_t n, int32_t D, int32_t d, int32_t m, int32_t prec) {
  if (check_sizes(n, d) != LR_OK || D < 1 || D > 15 || m < 0 || m > 64 || !valid_prec(prec)) return 0;
  return proj_layout(n, D, d, m, prec).total;
}

lr_status lr_projection_solve(void* stream, int64_t n, int32_t D, int32_t d, const float* X, const lr_hyper* hyp,
                              int32_t prec, const void* Q, double sigma2, int32_t clip, int32_t m, const void* A,
                              void* Xout, double* B, double* L, double* logdet, int32_t* info, void* ws,
                              size_t ws_bytes) {
  if (!valid_prec(prec)) return LR_ERR_ARG;
  if (D < 1 || D > 15) return LR_ERR_SHAPE;
  lr_status s = check_sizes(n, d);
  if (s != LR_OK) return s;
  if (m < 0 || m > 64) return LR_ERR_SHAPE;
  if (clip != 0 && clip != 1) return LR_ERR_ARG;
  if ((s = check_hyper(hyp)) != LR_OK) return s;
  if (!is_fin(sigma2) || !(sigma2 > 0.0)) return LR_ERR_ARG;
  if (X == nullptr || Q == nullptr || B == nullptr || L == nullptr || logdet == nullptr || info == nullptr)
    return LR_ERR_ARG;
  if (m > 0 && (A == nullptr || Xout == nullptr || A == Xout)) return LR_ERR_ARG;
  if ((s = check_ws(proj_layout(n, D, d, m, prec).total, ws, ws_bytes)) != LR_OK) return s;
  return projection_impl(static_cast<hipStream_t>(stream), n, D, d, X, hyp, prec, Q, sigma2, clip, m, A, Xout, B, L,
                         logdet, info, ws);
}

size_t lr_psd_part_workspace_bytes(int32_t d) {
  if (d < 1 || d > 1024) return 0;
  return al((size_t)3 * d * d * sizeof(double));
}

lr_status lr_psd_part(void* stream, int32_t d, const double* B, double* Bplus, void* ws, size_t ws_bytes) {
  if (d < 1 || d > 1024) return LR_ERR_SHAPE;
  if (B == nullptr || Bplus == nullptr || B == Bplus) return LR_ERR_ARG;
  lr_status s = check_ws(lr_psd_part_workspace_bytes(d), ws, ws_bytes);
  if (s != LR_OK) return s;
  LR_HIP(launch_psd_part(static_cast<hipStream_t>(stream), d, B, Bplus, static_cast<double*>(ws), kPsdSteps));
  return LR_OK;
}

lr_status lr_loglik(void* stream, int64_t n, int32_t prec, const void* y, const void* alpha, const double* logdet,
                    const int32_t* info, double* out) {
  if (!valid_prec(prec)) return LR_ERR_ARG;
  if (n < 1) return LR_ERR_SHAPE;
  if (y == nullptr || alpha == nullptr || logdet == nullptr || out == nullptr) return LR_ERR_ARG;
  LR_HIP(launch_loglik(static_cast<hipStream_t>(stream), n, prec == LR_PREC_F64, y, alpha, logdet, info, out));
  return LR_OK;
}

size_t lr_backward_workspace_bytes(int64_t n, int32_t D, int32_t d, int32_t m, int32_t prec) {
  if (check_sizes(n, d) != LR_OK || D < 1 || D > 15 || m < 0 || m > 64 || !valid_prec(prec)) return 0;
  return back_layout(n, D, d, m, prec).total;
}

lr_status lr_backward(void* stream, int64_t n, int32_t D, const float* X, const lr_hyper* hyp, const lr_omega* omega,
                      int32_t prec, const void* Q, const double* R, const double* C, const double* L,
                      const double* Flu, const int32_t* piv, double sigma2, double nu, int32_t mode, int32_t m,
                      const void* A, const void* V, const void* Yprime, double* dtheta, void* dA, void* ws,
                      size_t ws_bytes) {
  if (!valid_prec(prec)) return LR_ERR_ARG;
  if (D < 1 || D > 15) return LR_ERR_SHAPE;
  if (omega == nullptr) return LR_ERR_ARG;
  const int32_t d = omega->d;
  lr_status s = check_sizes(n, d);
  if (s != LR_OK) return s;
  if ((s = check_hyper(hyp)) != LR_OK) return s;
  if ((s = check_omega(omega, n, d, prec)) != LR_OK) return s;
  if (prec == LR_PREC_BF16X2 && D > 3) return LR_ERR_UNSUPPORTED;
  if (mode != 0 && mode != 1) return LR_ERR_ARG;
  if (mode == 0 && m != 1) return LR_ERR_SHAPE;
  if (mode == 1 && (m < 1 || m > 64)) return LR_ERR_SHAPE;
  if (!is_fin(sigma2) || !(sigma2 > 0.0) || !is_fin(nu) || nu < 0.0) return LR_ERR_ARG;
  if (X == nullptr || Q == nullptr || C == nullptr || L == nullptr || Flu == nullptr || piv == nullptr ||
      A == nullptr || dtheta == nullptr || (mode == 1 && V == nullptr) || (nu != 0.0 && R == nullptr))
    return LR_ERR_ARG;
  const BackWs w = back_layout(n, D, d, m, prec);
  if ((s = check_ws(w.total, ws, ws_bytes)) != LR_OK) return s;

  hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  auto dptr = [&](size_t off) { return reinterpret_cast<double*>(base + off); };
  void* tn = base + w.off_tn;
  const void* yp = Yprime;
  if (yp == nullptr) {
    void* ypw = base + w.off_yp;
    s = sketch_impl(st, n, D, X, hyp, omega, 0.0, prec, nullptr, ypw, base + w.off_sk);
    if (s != LR_OK) return s;
    yp = ypw;
  }
  double oscale = 1.0;
  const TnOperand om = omega_operand(omega, prec, &oscale);
  const TnOperand ypo = real_operand(yp, d, prec);
  const TnOperand qo = real_operand(Q, d, prec);
  const double inv_s2 = 1.0 / sigma2;
  // every n-length product below sums exact products in float64
  double* E = dptr(w.off_e);
  double* Phi = dptr(w.off_phi);
  LR_HIP(launch_gemm_tn(st, n, d, d, om, ypo, oscale, E, tn, true));
  LR_HIP(launch_trsm_cols(st, false, d, d, Flu, piv, 2, nullptr, Phi, d, nullptr));

  BackwardScalars b{};
  b.mode = mode;
  b.n = n;
  b.d = d;
  b.m = m;
  b.sigma2 = sigma2;
  b.E = E;
  b.C = C;
  b.dtheta = dtheta;
  b.nu = nu;
  const bool shifted = nu != 0.0;
  double* OO = nullptr;  // Omega^T Omega (SRHT: the identity, not formed)
  if (shifted && omega->kind == LR_OMEGA_GAUSS) {
    OO = dptr(w.off_oo);
    LR_HIP(launch_gemm_tn(st, n, d, d, om, om, oscale * oscale, OO, tn, true));
  }
  b.OO = OO;
  double* za = dptr(w.off_za);
  double* wa = dptr(w.off_wa);
  double* xa = dptr(w.off_xa);
  double* u64 = dptr(w.off_u64);
  // a = S^{-1} Q^T A, and alpha (or X) = K~^{-1} A recomputed in float64
  if ((s = project_solve(st, n, d, m, prec, Q, L, sigma2, nullptr, A, za, wa, xa, tn)) != LR_OK) return s;
  LR_HIP(launch_rowmix_f64out(st, n, d, m, Q, xa, inv_s2, A, u64, prec == LR_PREC_F64));
  const TnOperand uo = f64_operand(u64, m);
  if (mode == 0) {
    double* P = dptr(w.off_p);
    double* Sinv = dptr(w.off_sinv);
    double* T = dptr(w.off_t);
    double* G2 = dptr(w.off_g2);
    double* h = dptr(w.off_h);
    double* u = dptr(w.off_u);
    double* Eu = dptr(w.off_eu);
    double* Ca = dptr(w.off_ca);
    double* aa = dptr(w.off_aa);
    LR_HIP(launch_gemm_tn(st, n, d, 1, ypo, uo, 1.0, h, tn, true));
    LR_HIP(launch_gemm_tn(st, n, 1, 1, uo, uo, 1.0, aa, tn, true));
    LR_HIP(launch_gemm_tn(st, n, d, d, qo, ypo, 1.0, P, tn, true));
    LR_HIP(launch_trsm_cols(st, true, d, d, L, nullptr, 2, nullptr, Sinv, d, nullptr));
    LR_HIP(launch_gemm_dd(st, d, 1, d, 1.0, Phi, d, true, wa, 1, false, 0.0, u, 1));
    LR_HIP(launch_gemm_dd(st, d, d, d, 1.0, Sinv, d, false, Phi, d, false, 0.0, T, d));
    LR_HIP(launch_gemm_dd(st, d, d, d, 1.0, Phi, d, true, T, d, false, 0.0, G2, d));
    LR_HIP(launch_gemm_dd(st, d, 1, d, 1.0, E, d, false, u, 1, false, 0.0, Eu, 1));
    LR_HIP(launch_gemm_dd(st, d, 1, d, 1.0, C, d, false, wa, 1, false, 0.0, Ca, 1));
    b.a = wa;
    b.h = h;
    b.aa = aa;
    b.u = u;
    b.Eu = Eu;
    b.Ca = Ca;
    b.T = T;
    b.P = P;
    b.G2 = G2;
    b.Sinv = Sinv;
    if (shifted) {
      double* v1 = dptr(w.off_v1);
      double* Pta = dptr(w.off_pta);
      double* oa = dptr(w.off_oa);
      double* Fa = dptr(w.off_fa);
      LR_HIP(launch_trsm_upper(st, d, 1, R, wa, v1, 1));
      LR_HIP(launch_gemm_dd(st, d, 1, d, 1.0, P, d, true, wa, 1, false, 0.0, Pta, 1));
      LR_HIP(launch_gemm_tn(st, n, d, 1, om, uo, oscale, oa, tn, true));
      LR_HIP(launch_lu_apply(st, d, 1, Flu, piv, wa, Fa, 1));
      b.v1 = v1;
      b.Pta = Pta;
      b.oa = oa;
      b.Fa = Fa;
      if (OO != nullptr) {
        double* OOu = dptr(w.off_oou);
        LR_HIP(launch_gemm_dd(st, d, 1, d, 1.0, OO, d, false, u, 1, false, 0.0, OOu, 1));
        b.OOu = OOu;
      }
    }
  } else {
    double* zb = dptr(w.off_zb);
    double* wb = dptr(w.off_wb);
    double* xb = dptr(w.off_xb);
    double* b64 = dptr(w.off_b64);
    double* XY = dptr(w.off_xy);
    double* BY = dptr(w.off_by);
    double* XB = dptr(w.off_xbm);
    double* U1 = dptr(w.off_u1);
    double* U2 = dptr(w.off_u2);
    double* EU1 = dptr(w.off_eu1);
    double* EU2 = dptr(w.off_eu2);
    double* CQB = dptr(w.off_cqb);
    if ((s = project_solve(st, n, d, m, prec, Q, L, sigma2, nullptr, V, zb, wb, xb, tn)) != LR_OK) return s;
    LR_HIP(launch_rowmix_f64out(st, n, d, m, Q, xb, inv_s2, V, b64, prec == LR_PREC_F64));
    if (dA != nullptr) LR_HIP(launch_rowmix_info(st, n, d, m, Q, xb, inv_s2, V, dA, prec == LR_PREC_F64, nullptr));
    const TnOperand bo = f64_operand(b64, m);
    // X^T Y' and B^T Y' (m x d): for m <= 16 as Y'^T X (d x m) on the skinny
    // product, then transposed
    if (m <= 16) {
      double* tdm = dptr(w.off_tdm);
      LR_HIP(launch_gemm_tn(st, n, d, m, ypo, uo, 1.0, tdm, tn, true));
      LR_HIP(launch_transpose(st, d, m, tdm, d, XY, true));
      LR_HIP(launch_gemm_tn(st, n, d, m, ypo, bo, 1.0, tdm, tn, true));
      LR_HIP(launch_transpose(st, d, m, tdm, d, BY, true));
    } else {
      LR_HIP(launch_gemm_tn(st, n, m, d, uo, ypo, 1.0, XY, tn, true));
      LR_HIP(launch_gemm_tn(st, n, m, d, bo, ypo, 1.0, BY, tn, true));
    }
    LR_HIP(launch_gemm_tn(st, n, m, m, uo, bo, 1.0, XB, tn, true));
    LR_HIP(launch_gemm_dd(st, d, m, d, 1.0, Phi, d, true, wa, m, false, 0.0, U1, m));
    LR_HIP(launch_gemm_dd(st, d, m, d, 1.0, Phi, d, true, wb, m, false, 0.0, U2, m));
    LR_HIP(launch_gemm_dd(st, d, m, d, 1.0, E, d, false, U1, m, false, 0.0, EU1, m));
    LR_HIP(launch_gemm_dd(st, d, m, d, 1.0, E, d, false, U2, m, false, 0.0, EU2, m));
    LR_HIP(launch_gemm_dd(st, d, m, d, 1.0, C, d, false, wb, m, false, 0.0, CQB, m));
    b.U1 = U1;
    b.U2 = U2;
    b.EU1 = EU1;
    b.EU2 = EU2;
    b.QX = wa;
    b.CQB = CQB;
    b.XY = XY;
    b.BY = BY;
    b.XB = XB;
    if (shifted) {
      double* P = dptr(w.off_p);
      double* M1 = dptr(w.off_m1);
      double* M2 = dptr(w.off_m2);
      double* Z1 = dptr(w.off_z1);
      double* Z2 = dptr(w.off_z2);
      double* OX = dptr(w.off_ox);
      double* OB = dptr(w.off_ob);
      double* FQX = dptr(w.off_fqx);
      double* FQB = dptr(w.off_fqb);
      const size_t mdb = (size_t)m * d * sizeof(double);
      LR_HIP(launch_gemm_tn(st, n, d, d, qo, ypo, 1.0, P, tn, true));
      LR_HIP(hipMemcpyAsync(M1, XY, mdb, hipMemcpyDeviceToDevice, st));
      LR_HIP(hipMemcpyAsync(M2, BY, mdb, hipMemcpyDeviceToDevice, st));
      LR_HIP(launch_gemm_dd(st, m, d, d, -1.0, wa, m, true, P, d, false, 1.0, M1, d));
      LR_HIP(launch_gemm_dd(st, m, d, d, -1.0, wb, m, true, P, d, false, 1.0, M2, d));
      LR_HIP(launch_trsm_upper(st, d, m, R, wb, Z1, m));
      LR_HIP(launch_trsm_upper(st, d, m, R, wa, Z2, m));
      LR_HIP(launch_gemm_tn(st, n, d, m, om, uo, oscale, OX, tn, true));
      LR_HIP(launch_gemm_tn(st, n, d, m, om, bo, oscale, OB, tn, true));
      LR_HIP(launch_lu_apply(st, d, m, Flu, piv, wa, FQX, m));
      LR_HIP(launch_lu_apply(st, d, m, Flu, piv, wb, FQB, m));
      b.M1 = M1;
      b.M2 = M2;
      b.Z1 = Z1;
      b.Z2 = Z2;
      b.OX = OX;
      b.OB = OB;
      b.FQX = FQX;
      b.FQB = FQB;
      if (OO != nullptr) {
        double* OOU2 = dptr(w.off_oou2);
        LR_HIP(launch_gemm_dd(st, d, m, d, 1.0, OO, d, false, U2, m, false, 0.0, OOU2, m));
        b.OOU2 = OOU2;
      }
    }
  }
  LR_HIP(launch_backward_scalars(st, b));
  return LR_OK;
}

}  // extern "C"
