// Host-side launchers of the lrinv device code (all enqueue on `st`, no sync).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lr {

// sketch.hip
template <typename T>
hipError_t launch_prep_points(hipStream_t st, const float* X, int64_t n, int D, int PD, double scale,
                              const int8_t* signs, T* out);
template <typename T>
hipError_t launch_sketch_srht(hipStream_t st, int kernel, int D, const T* pts, const int32_t* cols, int64_t n,
                              int d, double scale_out, double nu_c, T* Y, T* Yp, int num_cu);
hipError_t launch_sketch_dense(hipStream_t st, int prec, int kernel, int D, const void* pts, const void* omt,
                               int64_t ld, int64_t n, int d, double scale_out, double nu, void* Y, bool deriv,
                               const void* frag, int num_cu);
// Omega (bf16, d x ld transposed) in matrix-core fragment order for the bf16
// sketch with D <= 3; omega_frag_bytes gives the size of that copy.
hipError_t launch_omega_frag(hipStream_t st, const void* omt, int64_t ld, int64_t n, int d, void* frag);
size_t omega_frag_bytes(int64_t n, int d);

// tsqr.hip
size_t tsqr_workspace(int64_t n, int d, int leaf_rows, bool f64);
template <typename T>
hipError_t tsqr_run(hipStream_t st, int64_t n, int d, int leaf_rows, const T* Y, T* Q, double* R, void* ws);

// linalg.hip
// Operand of a transposed product sum_r X(r, i) Y(r, j) over rows r.
struct TnOperand {
  int kind;          // 0 = row-major real (x[r*ld + i]); 1 = transposed dense Omega (x[i*ld + r]); 2 = SRHT
  int dtype;         // 0 = f64, 1 = f32, 2 = bf16 bits
  const void* ptr;
  int64_t ld;
  const int8_t* signs;  // SRHT
  const int32_t* cols;  // SRHT
};
// out (M x N, double) = sum_r X(r, :)^T Y(r, :) over r < n; partials in ws.
size_t tn_workspace(int64_t n, int M, int N);
hipError_t launch_gemm_tn(hipStream_t st, int64_t n, int M, int N, const TnOperand& X, const TnOperand& Y,
                          double x_scale, double* out, void* ws, bool f64);
// out (n x m, real) = alpha A + Q W   (Q n x d real, W d x m double); with `info`,
// nothing is written when *info != 0.
hipError_t launch_rowmix(hipStream_t st, int64_t n, int d, int m, const void* Q, const double* W, double alpha,
                         const void* A, void* out, bool f64);
hipError_t launch_rowmix_info(hipStream_t st, int64_t n, int d, int m, const void* Q, const double* W, double alpha,
                              const void* A, void* out, bool f64, const int32_t* info);
hipError_t launch_fill(hipStream_t st, double* out, int64_t count, double v);

// core.hip
hipError_t launch_core(hipStream_t st, int64_t n, int d, const double* F, const double* R, double sigma2, double nu,
                       double* Flu, int32_t* piv, double* C, double* L, double* logdet, int32_t* info);
// W' = S^{-1} Z - Z / sigma2 (d x m), S = L L^T; skipped when *info != 0.
hipError_t launch_core_apply(hipStream_t st, int d, int m, const double* L, const double* Z, double sigma2,
                             const int32_t* info, double* Wout);
hipError_t launch_loglik(hipStream_t st, int64_t n, bool f64, const void* y, const void* alpha, const double* logdet,
                         const int32_t* info, double* out);
// Backward small d x d work (see lr_backward).
struct BackwardSmall {
  int mode;
  int64_t n;
  int d, m;
  double sigma2;
  const double *Flu, *C, *L;
  const int32_t* piv;
  const double* a;      // mode 0: Q^T alpha (d)
  const double* h;      // mode 0: Y'^T alpha (d)
  const double* P;      // mode 0: Q^T Y' (d x d)
  const double* E;      // Omega^T Y' (d x d)
  const double* aa;     // mode 0: alpha^T alpha (1)
  const double* QX;     // mode 1: Q^T X (d x m)
  const double* QB;     // mode 1: Q^T B (d x m)
  const double* XY;     // mode 1: X^T Y' (m x d)
  const double* BY;     // mode 1: B^T Y' (m x d)
  const double* XB;     // mode 1: X^T B (m x m)
  const double* Phi;    // F^{-1} (d x d)
  const double* Sinv;   // mode 0: S^{-1} (d x d)
  double* scratch;      // 3 d*d doubles
  double* dtheta;
};
hipError_t launch_backward_small(hipStream_t st, const BackwardSmall& b);
// Column-wise dense solves (see core.hip): mode 0 LU (P L U), 1 Cholesky (L L^T),
// 2 LU with the right-hand side read transposed from src. Skipped when *info != 0.
hipError_t launch_solve_cols(hipStream_t st, int mode, int d, int nrhs, const double* Fm, const int32_t* piv,
                             const double* src, double* X, int ldx, const int32_t* info);
hipError_t launch_identity(hipStream_t st, double* X, int d);

}  // namespace lr
