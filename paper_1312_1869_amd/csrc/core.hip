// The d x d float64 core of the Woodbury-form approximation and of its adjoint.
//
// Forward (d <= 1024):
//   LU with partial pivoting of F = Omega^T Q (one 1024-thread workgroup;
//   LAPACK getrf convention: whole rows swapped, first index of the largest
//   magnitude as pivot); C = F^{-1} R^T by forward/backward substitution, one
//   wave per right-hand side; C <- (C + C^T)/2, S = C + (sigma2 - nu) I,
//   Cholesky S = L L^T and log|K~| = (n - d) log sigma2 + 2 sum log L_jj (one
//   workgroup).
//   info = -k for a zero LU pivot at step k, k for the k-th non-positive
//   Cholesky pivot (1-based), 0 on success.
// The small solve W' = S^{-1} Z - Z / sigma2 uses the same column solver.
// The backward kernel evaluates the d x d contractions of the hyperparameter
// adjoint (formulas in lrinv.h / the oracle's grad module).
#include "common.hpp"
#include "kernels.hpp"

namespace lr {

constexpr int kCoreThreads = 1024;
constexpr int kCoreWaves = kCoreThreads / 64;

__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
  return s;
}

// arg max |v| over the block; ties -> smallest index.
__device__ __forceinline__ int block_argmax(double v, int idx, double* redv, int* redi) {
  double a = fabs(v);
  int i = idx;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double oa = __shfl_xor(a, off, 64);
    const int oi = __shfl_xor(i, off, 64);
    if (oa > a || (oa == a && oi < i)) {
      a = oa;
      i = oi;
    }
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) {
    redv[w] = a;
    redi[w] = i;
  }
  __syncthreads();
  double ba = -1.0;
  int bi = 0x7fffffff;
  for (int k = 0; k < kCoreWaves; ++k) {
    if (redv[k] > ba || (redv[k] == ba && redi[k] < bi)) {
      ba = redv[k];
      bi = redi[k];
    }
  }
  return bi;
}

// LU with partial pivoting in place (row-major d x d). Returns 0 or -(k+1).
__device__ int lu_inplace(double* A, int32_t* piv, int d, double* redv, int* redi) {
  const int t = threadIdx.x;
  for (int k = 0; k < d; ++k) {
    double v = -1.0;
    int vi = 0x7fffffff;
    double best = -1.0;
    for (int i = k + t; i < d; i += kCoreThreads) {
      const double a = fabs(A[(int64_t)i * d + k]);
      if (a > best) {
        best = a;
        vi = i;
        v = a;
      }
    }
    if (vi == 0x7fffffff) v = -1.0;
    int p = block_argmax(v, vi, redv, redi);
    if (p < k || p >= d) p = k;  // column entirely NaN
    if (t == 0) piv[k] = p;
    const double pv = A[(int64_t)p * d + k];
    __syncthreads();  // every thread has read the pivot before rows move
    if (!(fabs(pv) > 0.0)) return -(k + 1);
    if (p != k) {
      for (int j = t; j < d; j += kCoreThreads) {
        const double x = A[(int64_t)k * d + j];
        A[(int64_t)k * d + j] = A[(int64_t)p * d + j];
        A[(int64_t)p * d + j] = x;
      }
    }
    __syncthreads();
    const double inv = 1.0 / A[(int64_t)k * d + k];
    for (int i = k + 1 + t; i < d; i += kCoreThreads) A[(int64_t)i * d + k] *= inv;
    __syncthreads();
    const int w = d - k - 1;
    const int64_t cnt = (int64_t)w * w;
    for (int64_t e = t; e < cnt; e += kCoreThreads) {
      const int i = k + 1 + (int)(e / w);
      const int j = k + 1 + (int)(e % w);
      A[(int64_t)i * d + j] -= A[(int64_t)i * d + k] * A[(int64_t)k * d + j];
    }
    __syncthreads();
  }
  return 0;
}

// Cholesky in place on the lower triangle of L (row-major). Returns 0 or k+1.
__device__ int chol_inplace(double* L, int d) {
  const int t = threadIdx.x;
  for (int k = 0; k < d; ++k) {
    const double akk = L[(int64_t)k * d + k];
    __syncthreads();
    if (!(akk > 0.0)) return k + 1;
    const double lkk = sqrt(akk);
    const double inv = 1.0 / lkk;
    for (int i = k + 1 + t; i < d; i += kCoreThreads) L[(int64_t)i * d + k] *= inv;
    __syncthreads();
    if (t == 0) L[(int64_t)k * d + k] = lkk;
    const int w = d - k - 1;
    const int64_t cnt = (int64_t)w * w;
    for (int64_t e = t; e < cnt; e += kCoreThreads) {
      const int i = k + 1 + (int)(e / w);
      const int j = k + 1 + (int)(e % w);
      if (j <= i) L[(int64_t)i * d + j] -= L[(int64_t)i * d + k] * L[(int64_t)j * d + k];
    }
    __syncthreads();
  }
  return 0;
}

// ---- forward core, three launches: LU(F); C = F^{-1} R^T (one wave per
// right-hand side); symmetrise + shift + Cholesky + log-determinant.

__global__ __launch_bounds__(kCoreThreads) void lu_kernel(int d, const double* __restrict__ F, double* Flu,
                                                          int32_t* piv, int32_t* info, double* logdet) {
  __shared__ double redv[kCoreWaves];
  __shared__ int redi[kCoreWaves];
  const int t = threadIdx.x;
  const int64_t dd = (int64_t)d * d;
  for (int64_t e = t; e < dd; e += kCoreThreads) Flu[e] = F[e];
  __syncthreads();
  const int lu = lu_inplace(Flu, piv, d, redv, redi);
  if (t == 0) {
    *info = lu;
    if (lu != 0) *logdet = __builtin_nan("");
  }
}

// Solve in place, for every column c of X (d x nrhs, leading dimension ldx):
//   mode 0: X <- A^{-1} X with A = P L U from lu_inplace (pivots applied first);
//   mode 1: X <- S^{-1} X with S = L L^T (lower Cholesky factor);
//   mode 2: as 0, with the right-hand side read as B[c][i] = src[c * d + i]
//           (i.e. the solve of A X = src^T), written to X.
// One wave per column; the column lives in LDS; the next row of the factor is
// prefetched into registers while the current row's dot product completes.
// Skipped when *info != 0.
constexpr int kSolveWaves = 4;
constexpr int kSolvePer = 16;  // d / 64 rounded up, d <= 1024

template <bool UNIT, bool LOWER, bool TRANSF>
__device__ __forceinline__ void wave_trisolve(const double* __restrict__ Fm, int d, double* y, int lane) {
  // LOWER: y_i = (y_i - sum_{k<i} F[i][k] y_k) / (UNIT ? 1 : F[i][i])
  // !LOWER with TRANSF: y_i = (y_i - sum_{k>i} F[k][i] y_k) / F[i][i]   (F^T upper)
  // !LOWER without TRANSF: y_i = (y_i - sum_{k>i} F[i][k] y_k) / F[i][i]
  double nxt[kSolvePer];
  auto load_row = [&](int i, double (&buf)[kSolvePer]) {
#pragma unroll
    for (int q = 0; q < kSolvePer; ++q) {
      const int k = lane + 64 * q;
      bool use;
      if (LOWER) use = k < i;
      else use = k > i && k < d;
      buf[q] = use ? (TRANSF ? Fm[(int64_t)k * d + i] : Fm[(int64_t)i * d + k]) : 0.0;
    }
  };
  const int first = LOWER ? 0 : d - 1;
  const int step = LOWER ? 1 : -1;
  load_row(first, nxt);
  for (int it = 0; it < d; ++it) {
    const int i = first + step * it;
    double cur[kSolvePer];
#pragma unroll
    for (int q = 0; q < kSolvePer; ++q) cur[q] = nxt[q];
    if (it + 1 < d) load_row(i + step, nxt);
    double part = 0.0;
#pragma unroll
    for (int q = 0; q < kSolvePer; ++q) {
      const int k = lane + 64 * q;
      if (k < d) part += cur[q] * y[k];
    }
    part = wave_sum(part);
    const double diag = UNIT ? 1.0 : Fm[(int64_t)i * d + i];
    const double yi = (y[i] - part) / diag;
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) y[i] = yi;
    __builtin_amdgcn_wave_barrier();
  }
}

__global__ __launch_bounds__(64 * kSolveWaves) void solve_cols_kernel(int mode, int d, int nrhs, const double* Fm,
                                                                      const int32_t* __restrict__ piv,
                                                                      const double* __restrict__ src, double* X,
                                                                      int ldx, const int32_t* __restrict__ info) {
  extern __shared__ double ybuf[];
  if (info != nullptr && *info != 0) return;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = blockIdx.x * kSolveWaves + w;
  if (c >= nrhs) return;
  double* y = ybuf + (int64_t)w * d;
  for (int i = lane; i < d; i += 64) y[i] = (mode == 2) ? src[(int64_t)c * d + i] : X[(int64_t)i * ldx + c];
  __builtin_amdgcn_wave_barrier();
  if (mode != 1) {
    if (lane == 0) {
      for (int k = 0; k < d; ++k) {
        const int p = piv[k];
        if (p != k) {
          const double tmp = y[k];
          y[k] = y[p];
          y[p] = tmp;
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
    wave_trisolve<true, true, false>(Fm, d, y, lane);   // unit lower L
    wave_trisolve<false, false, false>(Fm, d, y, lane); // upper U
  } else {
    wave_trisolve<false, true, false>(Fm, d, y, lane);  // L
    wave_trisolve<false, false, true>(Fm, d, y, lane);  // L^T
  }
  __builtin_amdgcn_wave_barrier();
  for (int i = lane; i < d; i += 64) X[(int64_t)i * ldx + c] = y[i];
}

hipError_t launch_solve_cols(hipStream_t st, int mode, int d, int nrhs, const double* Fm, const int32_t* piv,
                             const double* src, double* X, int ldx, const int32_t* info) {
  if (nrhs <= 0) return hipSuccess;
  const size_t lds = (size_t)kSolveWaves * d * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)solve_cols_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(solve_cols_kernel, dim3((unsigned)((nrhs + kSolveWaves - 1) / kSolveWaves)),
                     dim3(64 * kSolveWaves), lds, st, mode, d, nrhs, Fm, piv, src, X, ldx, info);
  return hipGetLastError();
}

__global__ __launch_bounds__(kCoreThreads) void chol_kernel(int64_t n, int d, double sigma2, double nu, double* C,
                                                            double* L, double* logdet, int32_t* info) {
  __shared__ double red[kCoreWaves];
  if (*info != 0) return;
  const int t = threadIdx.x;
  const int64_t dd = (int64_t)d * d;
  const double shift = sigma2 - nu;
  for (int64_t e = t; e < dd; e += kCoreThreads) {
    const int i = (int)(e / d), j = (int)(e % d);
    if (i < j) {
      const double s = 0.5 * (C[e] + C[(int64_t)j * d + i]);
      C[e] = s;
      C[(int64_t)j * d + i] = s;
    }
  }
  __syncthreads();
  for (int64_t e = t; e < dd; e += kCoreThreads) {
    const int i = (int)(e / d), j = (int)(e % d);
    L[e] = (j <= i) ? C[e] + (i == j ? shift : 0.0) : 0.0;
  }
  __syncthreads();
  const int ch = chol_inplace(L, d);
  if (ch != 0) {
    if (t == 0) {
      *info = ch;
      *logdet = __builtin_nan("");
    }
    return;
  }
  double part = 0.0;
  for (int k = t; k < d; k += kCoreThreads) part += log(L[(int64_t)k * d + k]);
  const double s = block_sum(part, red);
  if (t == 0) *logdet = (double)(n - d) * log(sigma2) + 2.0 * s;
}

hipError_t launch_core(hipStream_t st, int64_t n, int d, const double* F, const double* R, double sigma2, double nu,
                       double* Flu, int32_t* piv, double* C, double* L, double* logdet, int32_t* info) {
  hipLaunchKernelGGL(lu_kernel, dim3(1), dim3(kCoreThreads), 0, st, d, F, Flu, piv, info, logdet);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // C = F^{-1} R^T: column c of R^T is row c of R
  e = launch_solve_cols(st, 2, d, d, Flu, piv, R, C, d, info);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(chol_kernel, dim3(1), dim3(kCoreThreads), 0, st, n, d, sigma2, nu, C, L, logdet, info);
  return hipGetLastError();
}

// ------------------------------------------------------------------ log-likelihood

template <typename R>
__global__ __launch_bounds__(kCoreThreads) void loglik_kernel(int64_t n, const R* __restrict__ y,
                                                              const R* __restrict__ alpha,
                                                              const double* __restrict__ logdet,
                                                              const int32_t* __restrict__ info, double* out) {
  __shared__ double red[kCoreWaves];
  double part = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kCoreThreads) part += (double)y[i] * (double)alpha[i];
  const double s = block_sum(part, red);
  if (threadIdx.x == 0) {
    const bool ok = info == nullptr || *info == 0;
    *out = ok ? -0.5 * s - 0.5 * logdet[0] : __builtin_nan("");
  }
}

hipError_t launch_loglik(hipStream_t st, int64_t n, bool f64, const void* y, const void* alpha, const double* logdet,
                         const int32_t* info, double* out) {
  if (f64)
    hipLaunchKernelGGL(loglik_kernel<double>, dim3(1), dim3(kCoreThreads), 0, st, n, (const double*)y,
                       (const double*)alpha, logdet, info, out);
  else
    hipLaunchKernelGGL(loglik_kernel<float>, dim3(1), dim3(kCoreThreads), 0, st, n, (const float*)y,
                       (const float*)alpha, logdet, info, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ S^{-1} Z

__global__ void sub_scaled_kernel(int64_t count, const double* __restrict__ Z, double inv_sigma2,
                                  const int32_t* __restrict__ info, double* __restrict__ W) {
  if (info != nullptr && *info != 0) return;
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx < count) W[idx] -= Z[idx] * inv_sigma2;
}

hipError_t launch_core_apply(hipStream_t st, int d, int m, const double* L, const double* Z, double sigma2,
                             const int32_t* info, double* Wout) {
  if (m <= 0) return hipSuccess;
  const int64_t count = (int64_t)d * m;
  hipError_t e = hipMemcpyAsync(Wout, Z, (size_t)count * sizeof(double), hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  e = launch_solve_cols(st, 1, d, m, L, nullptr, nullptr, Wout, m, info);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sub_scaled_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, count, Z,
                     1.0 / sigma2, info, Wout);
  return hipGetLastError();
}

// ------------------------------------------------------------------ backward d x d

// out = A B (d x d), all row-major in global memory.
__device__ void matmul_dd(const double* A, const double* B, double* out, int d) {
  const int64_t dd = (int64_t)d * d;
  for (int64_t e = threadIdx.x; e < dd; e += kCoreThreads) {
    const int i = (int)(e / d), j = (int)(e % d);
    double s = 0.0;
    for (int k = 0; k < d; ++k) s += A[(int64_t)i * d + k] * B[(int64_t)k * d + j];
    out[e] = s;
  }
}

__global__ __launch_bounds__(kCoreThreads) void backward_small_kernel(BackwardSmall b) {
  __shared__ double red[kCoreWaves];
  const int t = threadIdx.x;
  const int d = b.d;
  const int64_t dd = (int64_t)d * d;
  const double* Phi = b.Phi;          // F^{-1} (precomputed)
  double* Mq = b.scratch;             // Q^T G Q
  double* T1 = b.scratch + dd;        // work
  double* T2 = b.scratch + 2 * dd;    // work

  double dlogell_t1 = 0.0, trace_g = 0.0;
  if (b.mode == 0) {
    const double* Sinv = b.Sinv;      // S^{-1} (precomputed)
    // Mq = (a a^T - S^{-1}) / 2 ; tr S^{-1}
    double tr = 0.0;
    for (int64_t e = t; e < dd; e += kCoreThreads) {
      const int i = (int)(e / d), j = (int)(e % d);
      Mq[e] = 0.5 * (b.a[i] * b.a[j] - Sinv[e]);
      if (i == j) tr += Sinv[e];
    }
    const double tr_sinv = block_sum(tr, red);
    // (Phi^T a) . h
    double p1 = 0.0;
    for (int i = t; i < d; i += kCoreThreads) {
      double u = 0.0;
      for (int k = 0; k < d; ++k) u += Phi[(int64_t)k * d + i] * b.a[k];
      p1 += u * b.h[i];
    }
    const double t1a = block_sum(p1, red);
    __syncthreads();
    // <S^{-1} Phi, P>
    matmul_dd(Sinv, Phi, T2, d);
    __syncthreads();
    double p2 = 0.0;
    for (int64_t e = t; e < dd; e += kCoreThreads) p2 += T2[e] * b.P[e];
    const double t1b = block_sum(p2, red);
    dlogell_t1 = t1a - t1b;
    trace_g = 0.5 * (b.aa[0] - ((double)(b.n - d) / b.sigma2 + tr_sinv));
  } else {
    const int m = b.m;
    // Mq = -(QX QB^T + QB QX^T)/2 ; T1 = QB XY + QX BY
    for (int64_t e = t; e < dd; e += kCoreThreads) {
      const int i = (int)(e / d), j = (int)(e % d);
      double s1 = 0.0, s2 = 0.0;
      for (int c = 0; c < m; ++c) {
        s1 += b.QX[(int64_t)i * m + c] * b.QB[(int64_t)j * m + c] + b.QB[(int64_t)i * m + c] * b.QX[(int64_t)j * m + c];
        s2 += b.QB[(int64_t)i * m + c] * b.XY[(int64_t)c * d + j] + b.QX[(int64_t)i * m + c] * b.BY[(int64_t)c * d + j];
      }
      Mq[e] = -0.5 * s1;
      T1[e] = s2;
    }
    __syncthreads();
    double p = 0.0;
    for (int64_t e = t; e < dd; e += kCoreThreads) p += Phi[e] * T1[e];
    dlogell_t1 = -block_sum(p, red);
    double tr = 0.0;
    for (int c = t; c < m; c += kCoreThreads) tr += b.XB[(int64_t)c * m + c];
    trace_g = -block_sum(tr, red);
  }
  __syncthreads();
  // T2' = <Mq Phi, Phi E>
  matmul_dd(Mq, Phi, T1, d);
  matmul_dd(Phi, b.E, T2, d);
  __syncthreads();
  double p3 = 0.0, p4 = 0.0;
  for (int64_t e = t; e < dd; e += kCoreThreads) {
    p3 += T1[e] * T2[e];
    p4 += Mq[e] * b.C[e];
  }
  const double t2 = block_sum(p3, red);
  const double mc = block_sum(p4, red);
  if (t == 0) {
    b.dtheta[0] = dlogell_t1 - t2;
    b.dtheta[1] = 2.0 * mc;
    b.dtheta[2] = b.sigma2 * trace_g;
  }
}

hipError_t launch_backward_small(hipStream_t st, const BackwardSmall& b) {
  hipLaunchKernelGGL(backward_small_kernel, dim3(1), dim3(kCoreThreads), 0, st, b);
  return hipGetLastError();
}

}  // namespace lr
