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
// out (d x N, float64) = scale * Omega^T M for an SRHT Omega (signs, cols) and
// a row-major real M (n x N, leading dimension N), in slabs of S rows
// (srht_left_slab: the largest slab whose transposed copy fits ws_bytes next
// to an N x d float64 accumulator; 0 when the product does not fit this path).
int64_t srht_left_slab(int64_t n, int d, int N, size_t elem, size_t ws_bytes);
template <typename T>
hipError_t launch_srht_left(hipStream_t st, int64_t n, int d, const int8_t* signs, const int32_t* cols, const T* M,
                            int N, double scale, double* out, void* ws, int64_t S);
// SRHT sketches Y_g (g < ntheta, Y_g = Y + g n d) for a batch of kernels that
// differ in ell and s: points prescaled for ell = 1, squared distances times
// dist_scale[g] = 1/ell_g^2, outputs times scale_out[g].
template <typename T>
hipError_t launch_sketch_srht_grid(hipStream_t st, int kernel, int D, const T* pts, const int32_t* cols, int64_t n,
                                   int d, int ntheta, const double* dist_scale, const double* scale_out, double nu_c,
                                   T* Y, int num_cu);
hipError_t launch_sketch_dense(hipStream_t st, int prec, int kernel, int D, const void* pts, const void* omt,
                               int64_t ld, int64_t n, int d, double scale_out, double nu, void* Y, bool deriv,
                               const void* frag, int num_cu);
// Dense transposed Omega of a structured transform (lr_structured_omega).
hipError_t launch_structured_omega(hipStream_t st, int transform, int64_t n, int d, const int8_t* signs,
                                   const int32_t* cols, int prec, void* out, int64_t ld, int num_cu);
// Omega (bf16, d x ld transposed) in matrix-core fragment order for the bf16
// sketch with D <= 3; omega_frag_bytes gives the size of that copy.
hipError_t launch_omega_frag(hipStream_t st, const void* omt, int64_t ld, int64_t n, int d, void* frag);
size_t omega_frag_bytes(int64_t n, int d);

// tsqr.hip
size_t tsqr_workspace(int64_t n, int d, int leaf_rows, bool f64);
template <typename T>
hipError_t tsqr_run(hipStream_t st, int64_t n, int d, int leaf_rows, const T* Y, T* Q, double* R, void* ws);
// Sequential groups of `group` blocks (Eq. 5), then the binary tree over the
// groups; n a multiple of leaf_rows, the block count a multiple of group,
// d + leaf_rows <= 8192. Q may be NULL (R only).
size_t tsqr_domino_workspace(int64_t n, int d, int leaf_rows, int group, bool f64);
template <typename T>
hipError_t tsqr_domino_run(hipStream_t st, int64_t n, int d, int leaf_rows, int group, const T* Y, T* Q, double* R,
                           void* ws);

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
// out (n x m, float64) = alpha A + Q W for real (float or double) Q and A: the
// products and sums in float64 on float64 matrix cores.
hipError_t launch_rowmix_f64out(hipStream_t st, int64_t n, int d, int m, const void* Q, const double* W,
                                double alpha, const void* A, double* out, bool in_f64);
// out (n x m, float) = float(in), in float64.
hipError_t launch_narrow(hipStream_t st, int64_t count, const double* in, float* out);
// out = W - Z / sigma2 (count doubles); skipped when *info != 0.
hipError_t launch_wmix(hipStream_t st, int64_t count, const double* W, const double* Z, double sigma2,
                       const int32_t* info, double* out);
hipError_t launch_fill(hipStream_t st, double* out, int64_t count, double v);
// out (d x ld) = Q^T for a row-major n x d Q (float or double), zero columns past n.
hipError_t launch_transpose(hipStream_t st, int64_t n, int d, const void* Q, int64_t ld, void* out, bool f64);

// core.hip
hipError_t launch_core(hipStream_t st, int64_t n, int d, const double* F, const double* R, double sigma2, double nu,
                       double* Flu, int32_t* piv, double* C, double* L, double* logdet, int32_t* info);
// Wfull = S^{-1} Z and Wmix = Wfull - Z / sigma2 (d x m), S = L L^T; skipped
// when *info != 0.
hipError_t launch_core_apply(hipStream_t st, int d, int m, const double* L, const double* Z, double sigma2,
                             const int32_t* info, double* Wfull, double* Wmix);
// S = sym(B) + sigma2 I, its Cholesky factor in L (lower) and the
// log-determinant; *info = 0 first, the failing pivot on breakdown.
hipError_t launch_chol_core(hipStream_t st, int64_t n, int d, const double* B, double sigma2, double* L,
                            double* logdet, int32_t* info);
hipError_t launch_loglik(hipStream_t st, int64_t n, bool f64, const void* y, const void* alpha, const double* logdet,
                         const int32_t* info, double* out);
// Scalars of the hyperparameter adjoint (see lr_backward and dense.hip).
struct BackwardScalars {
  int mode;
  int64_t n;
  int d, m;
  double sigma2;
  // mode 0 (log-likelihood)
  const double* a;      // S^{-1} Q^T y (d)
  const double* h;      // Y'^T alpha (d)
  const double* aa;     // alpha^T alpha (1)
  const double* u;      // Phi^T a (d)
  const double* Eu;     // E u (d)
  const double* Ca;     // C a (d)
  const double* T;      // S^{-1} Phi (d x d)
  const double* P;      // Q^T Y' (d x d)
  const double* G2;     // Phi^T S^{-1} Phi (d x d)
  const double* E;      // Omega^T Y' (d x d)
  const double* Sinv;   // S^{-1} (d x d)
  const double* C;      // C (d x d)
  // mode 1 (solve)
  const double* U1;     // Phi^T QX (d x m), QX = S^{-1} Q^T A
  const double* U2;     // Phi^T QB (d x m), QB = S^{-1} Q^T Abar
  const double* EU1;    // E U1 (d x m)
  const double* EU2;    // E U2 (d x m)
  const double* QX;     // (d x m)
  const double* CQB;    // C QB (d x m)
  const double* XY;     // X^T Y' (m x d)
  const double* BY;     // B^T Y' (m x d)
  const double* XB;     // X^T B (m x m)
  // shift nu != 0 (Y = (K_f + nu I) Omega): projector and Omega terms
  double nu;
  const double* OO;     // Omega^T Omega (d x d), NULL for SRHT (= I)
  const double* v1;     // mode 0: R^{-1} a (d)
  const double* Pta;    // mode 0: P^T a (d)
  const double* oa;     // mode 0: Omega^T alpha (d)
  const double* Fa;     // mode 0: F a (d)
  const double* OOu;    // mode 0: Omega^T Omega u (d), NULL for SRHT
  const double* M1;     // mode 1: XY - QX^T P (m x d)
  const double* M2;     // mode 1: BY - QB^T P (m x d)
  const double* Z1;     // mode 1: R^{-1} QB (d x m)
  const double* Z2;     // mode 1: R^{-1} QX (d x m)
  const double* OX;     // mode 1: Omega^T X (d x m)
  const double* OB;     // mode 1: Omega^T B (d x m)
  const double* FQX;    // mode 1: F QX (d x m)
  const double* FQB;    // mode 1: F QB (d x m)
  const double* OOU2;   // mode 1: Omega^T Omega U2 (d x m), NULL for SRHT
  double* dtheta;
};
hipError_t launch_backward_scalars(hipStream_t st, const BackwardScalars& b);
// dense.hip: out = alpha op(A) op(B) + beta out (row-major float64).
hipError_t launch_gemm_dd(hipStream_t st, int M, int N, int K, double alpha, const double* A, int lda, bool ta,
                          const double* B, int ldb, bool tb, double beta, double* out, int ldo);
// dense.hip: blocked solves with nrhs right-hand sides (d <= 1024), written to X
// (d x nrhs, leading dimension ldx). chol = false: X <- U^{-1} L^{-1} P B with the
// getrf factors Fm/piv; chol = true: X <- L^{-T} L^{-1} B, Fm = L lower.
// src_kind: 0 = B is X, 1 = column c of B is row c of src (d x d), 2 = B = I,
// 3 = B is src (d x nrhs, leading dimension ldx).
// Skipped when *info != 0.
hipError_t launch_trsm_cols(hipStream_t st, bool chol, int d, int nrhs, const double* Fm, const int32_t* piv,
                            int src_kind, const double* src, double* X, int ldx, const int32_t* info);
// dense.hip: X <- U^{-1} src for the upper triangle of U (d x d), nrhs columns.
hipError_t launch_trsm_upper(hipStream_t st, int d, int nrhs, const double* U, const double* src, double* X,
                             int ldx);
// dense.hip: out = F B, F given by its getrf factors (B, out d x nrhs, leading dimension ld).
hipError_t launch_lu_apply(hipStream_t st, int d, int nrhs, const double* Flu, const int32_t* piv, const double* B,
                           double* out, int ld);
hipError_t launch_identity(hipStream_t st, double* X, int d);
// The positive semidefinite part of a symmetric d x d matrix (dense.hip);
// ws holds 3 d^2 doubles.
hipError_t launch_psd_part(hipStream_t st, int d, const double* B, double* Bplus, double* ws, int steps);
hipError_t launch_symmetrize(hipStream_t st, int d, double* M);

}  // namespace lr
