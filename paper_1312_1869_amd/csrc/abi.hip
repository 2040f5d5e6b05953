// C ABI (include/lrinv.h): argument checks, workspace layout, launch order.
// Every check runs on the host before the first launch, so an argument error
// writes nothing. All work is enqueued on the caller's stream; nothing here
// synchronises or allocates.
#include <math.h>
#include <string.h>

#include <mutex>

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

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }
bool is_fin(double x) { return isfinite(x) != 0; }
bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }
size_t real_size(int32_t prec) { return prec == LR_PREC_F64 ? 8 : 4; }
bool valid_prec(int32_t prec) { return prec == LR_PREC_F64 || prec == LR_PREC_F32 || prec == LR_PREC_BF16; }

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
    if (prec == LR_PREC_BF16) return LR_ERR_UNSUPPORTED;
    return LR_OK;
  }
  if (o->kind == LR_OMEGA_GAUSS) {
    if (o->dense_t == nullptr || !aligned(o->dense_t, 16)) return LR_ERR_ARG;
    if (o->ld < n || o->ld % 8 != 0) return LR_ERR_SHAPE;
    // the bf16 sketch addresses Omega through 31-bit buffer extents
    if (prec == LR_PREC_BF16 && n > ((int64_t)1 << 25)) return LR_ERR_UNSUPPORTED;
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
  if (prec == LR_PREC_BF16 && D <= 3) b += al(omega_frag_bytes(n, d));
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
  if (prec == LR_PREC_BF16 && D <= 3) {
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
  size_t off_f, off_z, off_w, off_tn, total;
};

SolveWs solve_layout(int64_t n, int32_t d, int32_t m) {
  SolveWs w;
  size_t off = 0;
  w.off_f = off;
  off = al(off + (size_t)d * d * 8);
  w.off_z = off;
  off = al(off + (size_t)d * (m > 0 ? m : 1) * 8);
  w.off_w = off;
  off = al(off + (size_t)d * (m > 0 ? m : 1) * 8);
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

// X = K~^{-1} A given Q and the Cholesky factor (used by solve and backward).
lr_status woodbury_apply(hipStream_t st, int64_t n, int32_t d, int32_t m, int32_t prec, const void* Q,
                         const double* L, double sigma2, const int32_t* info, const void* A, void* X, double* Z,
                         double* W, void* tnws) {
  if (m <= 0) return LR_OK;
  const bool f64 = prec == LR_PREC_F64;
  LR_HIP(launch_gemm_tn(st, n, d, m, real_operand(Q, d, prec), real_operand(A, m, prec), 1.0, Z, tnws, f64));
  LR_HIP(launch_core_apply(st, d, m, L, Z, sigma2, info, W));
  LR_HIP(launch_rowmix_info(st, n, d, m, Q, W, 1.0 / sigma2, A, X, f64, info));
  return LR_OK;
}

// ---------------------------------------------------------------- backward

struct BackWs {
  size_t off_yp, off_sk, off_tn, off_e, off_a, off_h, off_p, off_aa, off_qx, off_qb, off_xy, off_by, off_xb, off_b,
      off_z, off_w, off_phi, off_sinv, off_scr, total;
};

BackWs back_layout(int64_t n, int32_t D, int32_t d, int32_t m, int32_t prec) {
  BackWs w;
  const size_t rs = real_size(prec);
  const int mm = m > 0 ? m : 1;
  size_t off = 0;
  w.off_yp = off;
  off = al(off + (size_t)n * d * rs);
  w.off_sk = off;
  off = al(off + sketch_ws(n, D, d, prec));
  size_t tn = tn_workspace(n, d, d);
  size_t t2 = tn_workspace(n, mm > d ? mm : d, mm > d ? mm : d);
  if (t2 > tn) tn = t2;
  w.off_tn = off;
  off = al(off + tn);
  w.off_e = off;
  off = al(off + (size_t)d * d * 8);
  w.off_a = off;
  off = al(off + (size_t)d * 8);
  w.off_h = off;
  off = al(off + (size_t)d * 8);
  w.off_p = off;
  off = al(off + (size_t)d * d * 8);
  w.off_aa = off;
  off = al(off + 8);
  w.off_qx = off;
  off = al(off + (size_t)d * mm * 8);
  w.off_qb = off;
  off = al(off + (size_t)d * mm * 8);
  w.off_xy = off;
  off = al(off + (size_t)mm * d * 8);
  w.off_by = off;
  off = al(off + (size_t)mm * d * 8);
  w.off_xb = off;
  off = al(off + (size_t)mm * mm * 8);
  w.off_b = off;
  off = al(off + (size_t)n * mm * rs);
  w.off_z = off;
  off = al(off + (size_t)d * mm * 8);
  w.off_w = off;
  off = al(off + (size_t)d * mm * 8);
  w.off_phi = off;
  off = al(off + (size_t)d * d * 8);
  w.off_sinv = off;
  off = al(off + (size_t)d * d * 8);
  w.off_scr = off;
  off = al(off + (size_t)3 * d * d * 8);
  w.total = off;
  return w;
}

}  // namespace

extern "C" {

int32_t lr_version(void) { return (1 << 16) | 0; }

const char* lr_status_string(int32_t s) {
  switch (s) {
    case LR_OK: return "LR_OK";
    case LR_ERR_ARG: return "LR_ERR_ARG";
    case LR_ERR_SHAPE: return "LR_ERR_SHAPE";
    case LR_ERR_NOT_POW2: return "LR_ERR_NOT_POW2";
    case LR_ERR_WORKSPACE: return "LR_ERR_WORKSPACE";
    case LR_ERR_HIP: return "LR_ERR_HIP";
    case LR_ERR_UNSUPPORTED: return "LR_ERR_UNSUPPORTED";
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
  if (!is_fin(nu) || nu < 0.0) return LR_ERR_ARG;
  if ((s = check_ws(sketch_ws(n, D, omega->d, prec), ws, ws_bytes)) != LR_OK) return s;
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
  void* tn = base + w.off_tn;
  const bool f64 = prec == LR_PREC_F64;
  double oscale = 1.0;
  const TnOperand om = omega_operand(omega, prec, &oscale);
  LR_HIP(launch_gemm_tn(st, n, d, d, om, real_operand(Q, d, prec), oscale, F, tn, f64));
  LR_HIP(launch_core(st, n, d, F, R, sigma2, nu, Flu, piv, C, L, logdet, info));
  return woodbury_apply(st, n, d, m, prec, Q, L, sigma2, info, A, X, Z, W, tn);
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
                      int32_t prec, const void* Q, const double* C, const double* L, const double* Flu,
                      const int32_t* piv, double sigma2, int32_t mode, int32_t m, const void* U, const void* V,
                      const void* Yprime, double* dtheta, void* dA, void* ws, size_t ws_bytes) {
  if (!valid_prec(prec)) return LR_ERR_ARG;
  if (D < 1 || D > 15) return LR_ERR_SHAPE;
  if (omega == nullptr) return LR_ERR_ARG;
  const int32_t d = omega->d;
  lr_status s = check_sizes(n, d);
  if (s != LR_OK) return s;
  if ((s = check_hyper(hyp)) != LR_OK) return s;
  if ((s = check_omega(omega, n, d, prec)) != LR_OK) return s;
  if (mode != 0 && mode != 1) return LR_ERR_ARG;
  if (mode == 0 && m != 1) return LR_ERR_SHAPE;
  if (mode == 1 && (m < 1 || m > 64)) return LR_ERR_SHAPE;
  if (!is_fin(sigma2) || !(sigma2 > 0.0)) return LR_ERR_ARG;
  if (X == nullptr || Q == nullptr || C == nullptr || L == nullptr || Flu == nullptr || piv == nullptr ||
      U == nullptr || dtheta == nullptr || (mode == 1 && V == nullptr))
    return LR_ERR_ARG;
  const BackWs w = back_layout(n, D, d, m, prec);
  if ((s = check_ws(w.total, ws, ws_bytes)) != LR_OK) return s;

  hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  const bool f64 = prec == LR_PREC_F64;
  const size_t rs = real_size(prec);
  (void)rs;
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
  BackwardSmall b{};
  b.mode = mode;
  b.n = n;
  b.d = d;
  b.m = m;
  b.sigma2 = sigma2;
  b.Flu = Flu;
  b.C = C;
  b.L = L;
  b.piv = piv;
  b.E = reinterpret_cast<double*>(base + w.off_e);
  b.scratch = reinterpret_cast<double*>(base + w.off_scr);
  b.dtheta = dtheta;
  double* phi = reinterpret_cast<double*>(base + w.off_phi);
  LR_HIP(launch_identity(st, phi, d));
  LR_HIP(launch_solve_cols(st, 0, d, d, Flu, piv, nullptr, phi, d, nullptr));
  b.Phi = phi;
  if (mode == 0) {
    double* sinv = reinterpret_cast<double*>(base + w.off_sinv);
    LR_HIP(launch_identity(st, sinv, d));
    LR_HIP(launch_solve_cols(st, 1, d, d, L, nullptr, nullptr, sinv, d, nullptr));
    b.Sinv = sinv;
  }
  LR_HIP(launch_gemm_tn(st, n, d, d, om, ypo, oscale, const_cast<double*>(b.E), tn, f64));
  if (mode == 0) {
    const TnOperand al_ = real_operand(U, 1, prec);
    double* a = reinterpret_cast<double*>(base + w.off_a);
    double* h = reinterpret_cast<double*>(base + w.off_h);
    double* P = reinterpret_cast<double*>(base + w.off_p);
    double* aa = reinterpret_cast<double*>(base + w.off_aa);
    LR_HIP(launch_gemm_tn(st, n, d, 1, qo, al_, 1.0, a, tn, f64));
    LR_HIP(launch_gemm_tn(st, n, d, 1, ypo, al_, 1.0, h, tn, f64));
    LR_HIP(launch_gemm_tn(st, n, d, d, qo, ypo, 1.0, P, tn, f64));
    LR_HIP(launch_gemm_tn(st, n, 1, 1, al_, al_, 1.0, aa, tn, f64));
    b.a = a;
    b.h = h;
    b.P = P;
    b.aa = aa;
  } else {
    void* B = dA != nullptr ? dA : (void*)(base + w.off_b);
    double* Zb = reinterpret_cast<double*>(base + w.off_z);
    double* Wb = reinterpret_cast<double*>(base + w.off_w);
    s = woodbury_apply(st, n, d, m, prec, Q, L, sigma2, nullptr, V, B, Zb, Wb, tn);
    if (s != LR_OK) return s;
    const TnOperand xo = real_operand(U, m, prec);
    const TnOperand bo = real_operand(B, m, prec);
    double* QX = reinterpret_cast<double*>(base + w.off_qx);
    double* QB = reinterpret_cast<double*>(base + w.off_qb);
    double* XY = reinterpret_cast<double*>(base + w.off_xy);
    double* BY = reinterpret_cast<double*>(base + w.off_by);
    double* XB = reinterpret_cast<double*>(base + w.off_xb);
    LR_HIP(launch_gemm_tn(st, n, d, m, qo, xo, 1.0, QX, tn, f64));
    LR_HIP(launch_gemm_tn(st, n, d, m, qo, bo, 1.0, QB, tn, f64));
    LR_HIP(launch_gemm_tn(st, n, m, d, xo, ypo, 1.0, XY, tn, f64));
    LR_HIP(launch_gemm_tn(st, n, m, d, bo, ypo, 1.0, BY, tn, f64));
    LR_HIP(launch_gemm_tn(st, n, m, m, xo, bo, 1.0, XB, tn, f64));
    b.QX = QX;
    b.QB = QB;
    b.XY = XY;
    b.BY = BY;
    b.XB = XB;
  }
  LR_HIP(launch_backward_small(st, b));
  return LR_OK;
}

}  // extern "C"
