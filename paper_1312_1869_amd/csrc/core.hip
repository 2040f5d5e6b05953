// The d x d float64 core of the Woodbury-form approximation and of its adjoint.
//
// Forward (one 1024-thread workgroup; d <= 1024):
//   LU with partial pivoting of F = Omega^T Q (LAPACK getrf convention: whole
//   rows swapped, first index of the largest magnitude as pivot), C = F^{-1} R^T
//   by forward/backward substitution (one thread per right-hand side),
//   C <- (C + C^T)/2, S = C + (sigma2 - nu) I, Cholesky S = L L^T, and
//   log|K~| = (n - d) log sigma2 + 2 sum log L_jj.
//   info = -k for a zero LU pivot at step k, k for the k-th non-positive
//   Cholesky pivot (1-based), 0 on success.
// The small solve W' = S^{-1} Z - Z / sigma2 runs one wave per column of Z.
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

// X (d x nrhs, row-major, column c handled by thread c) <- A^{-1} X with the
// LU factors and pivots of lu_inplace.
__device__ void lu_solve_cols(const double* LU, const int32_t* piv, int d, double* X, int nrhs, int ldx) {
  for (int c = threadIdx.x; c < nrhs; c += kCoreThreads) {
    for (int k = 0; k < d; ++k) {
      const int p = piv[k];
      if (p != k) {
        const double x = X[(int64_t)k * ldx + c];
        X[(int64_t)k * ldx + c] = X[(int64_t)p * ldx + c];
        X[(int64_t)p * ldx + c] = x;
      }
    }
    for (int i = 1; i < d; ++i) {
      double s = X[(int64_t)i * ldx + c];
      for (int k = 0; k < i; ++k) s -= LU[(int64_t)i * d + k] * X[(int64_t)k * ldx + c];
      X[(int64_t)i * ldx + c] = s;
    }
    for (int i = d - 1; i >= 0; --i) {
      double s = X[(int64_t)i * ldx + c];
      for (int k = i + 1; k < d; ++k) s -= LU[(int64_t)i * d + k] * X[(int64_t)k * ldx + c];
      X[(int64_t)i * ldx + c] = s / LU[(int64_t)i * d + i];
    }
  }
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

__global__ __launch_bounds__(kCoreThreads) void core_kernel(int64_t n, int d, const double* __restrict__ F,
                                                            const double* __restrict__ R, double sigma2, double nu,
                                                            double* Flu, int32_t* piv, double* C, double* L,
                                                            double* logdet, int32_t* info) {
  __shared__ double redv[kCoreWaves];
  __shared__ int redi[kCoreWaves];
  __shared__ double red[kCoreWaves];
  const int t = threadIdx.x;
  const int64_t dd = (int64_t)d * d;
  for (int64_t e = t; e < dd; e += kCoreThreads) Flu[e] = F[e];
  __syncthreads();
  const int lu = lu_inplace(Flu, piv, d, redv, redi);
  if (lu != 0) {
    if (t == 0) {
      *info = lu;
      *logdet = __builtin_nan("");
    }
    return;
  }
  // C = F^{-1} R^T
  for (int64_t e = t; e < dd; e += kCoreThreads) {
    const int i = (int)(e / d), j = (int)(e % d);
    C[e] = R[(int64_t)j * d + i];
  }
  __syncthreads();
  lu_solve_cols(Flu, piv, d, C, d, d);
  __syncthreads();
  // symmetrise; S = C + (sigma2 - nu) I into the lower triangle of L
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
  if (t == 0) {
    *info = 0;
    *logdet = (double)(n - d) * log(sigma2) + 2.0 * s;
  }
}

hipError_t launch_core(hipStream_t st, int64_t n, int d, const double* F, const double* R, double sigma2, double nu,
                       double* Flu, int32_t* piv, double* C, double* L, double* logdet, int32_t* info) {
  hipLaunchKernelGGL(core_kernel, dim3(1), dim3(kCoreThreads), 0, st, n, d, F, R, sigma2, nu, Flu, piv, C, L, logdet,
                     info);
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

__global__ __launch_bounds__(256) void core_apply_kernel(int d, int m, const double* __restrict__ L,
                                                         const double* __restrict__ Z, double sigma2,
                                                         const int32_t* __restrict__ info, double* __restrict__ W) {
  extern __shared__ double ybuf[];  // 4 waves x d
  if (info != nullptr && *info != 0) return;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = blockIdx.x * 4 + w;
  if (c >= m) return;
  double* y = ybuf + (int64_t)w * d;
  // forward: L y = z
  for (int i = 0; i < d; ++i) {
    double part = 0.0;
    for (int k = lane; k < i; k += 64) part += L[(int64_t)i * d + k] * y[k];
    part = wave_sum(part);
    const double yi = (Z[(int64_t)i * m + c] - part) / L[(int64_t)i * d + i];
    if (lane == 0) y[i] = yi;
    __builtin_amdgcn_wave_barrier();
  }
  // backward: L^T x = y (x overwrites y from the end)
  for (int i = d - 1; i >= 0; --i) {
    double part = 0.0;
    for (int k = i + 1 + lane; k < d; k += 64) part += L[(int64_t)k * d + i] * y[k];
    part = wave_sum(part);
    const double xi = (y[i] - part) / L[(int64_t)i * d + i];
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) y[i] = xi;
    __builtin_amdgcn_wave_barrier();
  }
  for (int i = lane; i < d; i += 64) W[(int64_t)i * m + c] = y[i] - Z[(int64_t)i * m + c] / sigma2;
}

hipError_t launch_core_apply(hipStream_t st, int d, int m, const double* L, const double* Z, double sigma2,
                             const int32_t* info, double* Wout) {
  if (m <= 0) return hipSuccess;
  const size_t lds = (size_t)4 * d * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)core_apply_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(core_apply_kernel, dim3((unsigned)((m + 3) / 4)), dim3(256), lds, st, d, m, L, Z, sigma2, info,
                     Wout);
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
  double* Phi = b.scratch;            // F^{-1}
  double* Mq = b.scratch + dd;        // Q^T G Q
  double* T1 = b.scratch + 2 * dd;    // work
  double* T2 = b.scratch + 3 * dd;    // work

  // Phi = F^{-1}
  for (int64_t e = t; e < dd; e += kCoreThreads) Phi[e] = ((e / d) == (e % d)) ? 1.0 : 0.0;
  __syncthreads();
  lu_solve_cols(b.Flu, b.piv, d, Phi, d, d);
  __syncthreads();

  double dlogell_t1 = 0.0, trace_g = 0.0;
  if (b.mode == 0) {
    // S^{-1} into T1 (columns by forward/backward substitution with L)
    for (int64_t e = t; e < dd; e += kCoreThreads) T1[e] = ((e / d) == (e % d)) ? 1.0 : 0.0;
    __syncthreads();
    for (int c = t; c < d; c += kCoreThreads) {
      for (int i = 0; i < d; ++i) {
        double s = T1[(int64_t)i * d + c];
        for (int k = 0; k < i; ++k) s -= b.L[(int64_t)i * d + k] * T1[(int64_t)k * d + c];
        T1[(int64_t)i * d + c] = s / b.L[(int64_t)i * d + i];
      }
      for (int i = d - 1; i >= 0; --i) {
        double s = T1[(int64_t)i * d + c];
        for (int k = i + 1; k < d; ++k) s -= b.L[(int64_t)k * d + i] * T1[(int64_t)k * d + c];
        T1[(int64_t)i * d + c] = s / b.L[(int64_t)i * d + i];
      }
    }
    __syncthreads();
    // Mq = (a a^T - S^{-1}) / 2 ; tr S^{-1}
    double tr = 0.0;
    for (int64_t e = t; e < dd; e += kCoreThreads) {
      const int i = (int)(e / d), j = (int)(e % d);
      Mq[e] = 0.5 * (b.a[i] * b.a[j] - T1[e]);
      if (i == j) tr += T1[e];
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
    matmul_dd(T1, Phi, T2, d);
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
