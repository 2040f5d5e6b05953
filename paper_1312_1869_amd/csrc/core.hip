// The d x d float64 core of the Woodbury-form approximation and of its adjoint.
//
// Forward (d <= 1024):
//   blocked LU with partial pivoting of F = Omega^T Q (LAPACK getrf
//   convention: whole rows swapped, first index of the largest magnitude as
//   pivot); C = F^{-1} R^T by blocked forward/backward substitution; C <- (C + C^T)/2, S = C + (sigma2 - nu) I, blocked
//   Cholesky S = L L^T and log|K~| = (n - d) log sigma2 + 2 sum log L_jj.
//   info = -k for a zero LU pivot at step k, k for the k-th non-positive
//   Cholesky pivot (1-based), 0 on success.
// The solves with many right-hand sides (F^{-1} R^T, S^{-1} Z) are the blocked
// ones of dense.hip. The backward kernel adds up the contractions of the
// hyperparameter adjoint from the d x d and d x m products the host sequence
// forms with them.
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

// ---- blocked LU with partial pivoting (panels of kPanel columns).
// Panel kernel: one workgroup, row k0 + t of the panel in thread t's
// registers; per column a block arg-max (first index among equal magnitudes),
// an exchange of the pivot row through LDS, scaling and a rank-1 update of
// the remaining panel columns. Update kernel: one workgroup per 64 columns
// outside the panel applies the panel's row exchanges to its columns and, to
// the right of the panel, solves U12 = L11^{-1} A12 and updates
// A22 -= L21 U12 (L21 staged through LDS).
constexpr int kPanel = 32;

template <int CTRL>
__device__ __forceinline__ void argmax_dpp(double& a, int& i) {
  const double oa = dpp_move<CTRL>(a);
  const int oi = __builtin_amdgcn_update_dpp(0, i, CTRL, 0xF, 0xF, false);
  if (oa > a || (oa == a && oi < i)) {
    a = oa;
    i = oi;
  }
}

template <int NWV>
__device__ __forceinline__ int block_argmax_db(double v, int idx, double* redv, int* redi, int& parity) {
  double a = v;
  int i = idx;
  // inside each 16-lane row by DPP (xor 1, xor 2, half-row mirror, xor 8),
  // then across the 4 rows by two lane shuffles
  argmax_dpp<0xB1>(a, i);
  argmax_dpp<0x4E>(a, i);
  argmax_dpp<0x141>(a, i);
  argmax_dpp<0x128>(a, i);
#pragma unroll
  for (int off = 16; off <= 32; off <<= 1) {
    const double oa = __shfl_xor(a, off, 64);
    const int oi = __shfl_xor(i, off, 64);
    if (oa > a || (oa == a && oi < i)) {
      a = oa;
      i = oi;
    }
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* bv = redv + parity * NWV;
  int* bi = redi + parity * NWV;
  parity ^= 1;
  if (lane == 0) {
    bv[w] = a;
    bi[w] = i;
  }
  __syncthreads();
  double ba = -1.0;
  int best = 0x7fffffff;
  for (int k = 0; k < NWV; ++k) {
    if (bv[k] > ba || (bv[k] == ba && bi[k] < best)) {
      ba = bv[k];
      best = bi[k];
    }
  }
  return best;
}

// TPB >= d - k0 threads: one panel row each.
template <int TPB>
__global__ __launch_bounds__(TPB) void lu_panel_kernel(int d, double* A, int k0, int32_t* piv, int32_t* info,
                                                       double* logdet) {
  constexpr int NWV = TPB / 64;
  __shared__ double redv[2 * NWV];
  __shared__ int redi[2 * NWV];
  __shared__ double prow[2][kPanel];
  __shared__ double krow[2][kPanel];
  if (*info != 0) return;
  const int t = threadIdx.x;
  const int r = k0 + t;
  const int nb = min(kPanel, d - k0);
  const bool have = r < d;
  double a[kPanel];
#pragma unroll
  for (int c = 0; c < kPanel; ++c) a[c] = (have && c < nb) ? A[(int64_t)r * d + k0 + c] : 0.0;
  int par = 0;
  bool ok = true;  // uniform over the block
  // expanded at compile time so every register-array index is a constant
  static_for<0, kPanel>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    if (!ok || c >= nb) return;
    const int k = k0 + c;
    // candidate magnitude on rows >= k (NaN never wins)
    const double mag = (have && r >= k) ? fabs(a[c]) : -1.0;
    int p = block_argmax_db<NWV>(mag == mag ? mag : -1.0, have && r >= k ? r : 0x7fffffff, redv, redi, par);
    if (p < k || p >= d) p = k;
    const int buf = c & 1;
    if (r == p) {
#pragma unroll
      for (int q = 0; q < kPanel; ++q) prow[buf][q] = a[q];
    }
    if (r == k) {
#pragma unroll
      for (int q = 0; q < kPanel; ++q) krow[buf][q] = a[q];
    }
    __syncthreads();
    const double pv = prow[buf][c];
    if (!(fabs(pv) > 0.0)) {
      if (t == 0) {
        *info = -(k + 1);
        *logdet = __builtin_nan("");
      }
      ok = false;
      return;
    }
    if (t == 0) piv[k] = p;
    if (r == k && p != k) {
#pragma unroll
      for (int q = 0; q < kPanel; ++q) a[q] = prow[buf][q];
    } else if (r == p && p != k) {
#pragma unroll
      for (int q = 0; q < kPanel; ++q) a[q] = krow[buf][q];
    }
    if (have && r > k) {
      const double l = a[c] / pv;
      a[c] = l;
#pragma unroll
      for (int q = 0; q < kPanel; ++q)
        if (q > c) a[q] -= l * prow[buf][q];
    }
  });
  if (!ok) return;
  if (have) {
#pragma unroll
    for (int c = 0; c < kPanel; ++c)
      if (c < nb) A[(int64_t)r * d + k0 + c] = a[c];
  }
}

constexpr int kLuCols = 64;

// After the panel at k0: the panel's row exchanges on every other column
// block, and on the blocks right of the panel U12 = L11^{-1} A12 (unit lower,
// one column per thread, solved through LDS and written back). The rank-nb
// update of A22 follows in lu_gemm_kernel.
__global__ __launch_bounds__(256) void lu_swap_solve_kernel(int d, double* A, int k0, const int32_t* __restrict__ piv,
                                                            const int32_t* __restrict__ info) {
  __shared__ double L11[kPanel][kPanel];
  __shared__ double U12[kPanel][kLuCols];
  if (*info != 0) return;
  const int t = threadIdx.x;
  const int nb = min(kPanel, d - k0);
  const int kend = k0 + nb;
  // column blocks: left of the panel first, then right of it
  const int nleft = (k0 + kLuCols - 1) / kLuCols;
  int c0;
  bool right;
  if ((int)blockIdx.x < nleft) {
    c0 = blockIdx.x * kLuCols;
    right = false;
  } else {
    c0 = kend + (blockIdx.x - nleft) * kLuCols;
    right = true;
  }
  const int cend = right ? min(c0 + kLuCols, d) : min(c0 + kLuCols, k0);
  const int cl = t & (kLuCols - 1);
  const int col = c0 + cl;
  const bool col_ok = col < cend;
  // row exchanges of this panel, in order
  if (t < kLuCols && col_ok) {
    for (int k = k0; k < kend; ++k) {
      const int p = piv[k];
      if (p != k) {
        const double x = A[(int64_t)k * d + col];
        A[(int64_t)k * d + col] = A[(int64_t)p * d + col];
        A[(int64_t)p * d + col] = x;
      }
    }
  }
  if (!right) return;
  for (int e = t; e < kPanel * kPanel; e += 256) {
    const int i = e / kPanel, j = e % kPanel;
    L11[i][j] = (i < nb && j < nb) ? A[(int64_t)(k0 + i) * d + k0 + j] : 0.0;
  }
  __syncthreads();
  if (t < kLuCols) {
    for (int i = 0; i < kPanel; ++i) {
      double s = (col_ok && i < nb) ? A[(int64_t)(k0 + i) * d + col] : 0.0;
      for (int q = 0; q < i; ++q) s -= L11[i][q] * U12[q][t];
      U12[i][t] = s;
      if (col_ok && i < nb) A[(int64_t)(k0 + i) * d + col] = s;
    }
  }
}

// A22 -= L21 U12 for the trailing matrix right of and below the panel: one
// workgroup per 64 x 64 tile, L21 and U12 staged through LDS.
__global__ __launch_bounds__(256) void lu_gemm_kernel(int d, double* A, int k0, const int32_t* __restrict__ info) {
  __shared__ double L21[64][kPanel + 1];
  __shared__ double U12[kPanel][64];
  if (*info != 0) return;
  const int t = threadIdx.x;
  const int nb = min(kPanel, d - k0);
  const int kend = k0 + nb;
  const int c0 = kend + blockIdx.x * 64;
  const int r0 = kend + blockIdx.y * 64;
  for (int e = t; e < 64 * kPanel; e += 256) {
    const int i = e / kPanel, q = e % kPanel;
    L21[i][q] = (r0 + i < d && q < nb) ? A[(int64_t)(r0 + i) * d + k0 + q] : 0.0;
    const int qq = e / 64, j = e % 64;
    U12[qq][j] = (c0 + j < d && qq < nb) ? A[(int64_t)(k0 + qq) * d + c0 + j] : 0.0;
  }
  __syncthreads();
  const int cl = t & 63;
  const int col = c0 + cl;
  if (col >= d) return;
  for (int i = t >> 6; i < 64 && r0 + i < d; i += 4) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kPanel; ++q) s += L21[i][q] * U12[q][cl];
    A[(int64_t)(r0 + i) * d + col] -= s;
  }
}

// ---- blocked Cholesky of the lower triangle (panels of kPanel columns).
// TPB >= d - k0 - kPanel threads (one row below the diagonal block each), TPB >= 64.
template <int TPB>
__global__ __launch_bounds__(TPB) void chol_panel_kernel(int d, double* L, int k0, int32_t* info, double* logdet) {
  __shared__ double Lkk[kPanel][kPanel + 1];
  __shared__ int bad;
  if (*info != 0) return;
  const int t = threadIdx.x;
  const int nb = min(kPanel, d - k0);
  for (int e = t; e < kPanel * kPanel; e += TPB) {
    const int i = e / kPanel, j = e % kPanel;
    Lkk[i][j] = (i < nb && j < nb && j <= i) ? L[(int64_t)(k0 + i) * d + k0 + j] : 0.0;
  }
  if (t == 0) bad = 0;
  __syncthreads();
  // unblocked Cholesky of the diagonal block by the first wave
  if (t < 64) {
    for (int c = 0; c < nb; ++c) {
      double dc = Lkk[c][c];
      for (int q = 0; q < c; ++q) dc -= Lkk[c][q] * Lkk[c][q];
      if (!(dc > 0.0)) {
        if (t == 0) bad = k0 + c + 1;
        break;
      }
      const double lcc = sqrt(dc);
      __builtin_amdgcn_wave_barrier();
      if (t > c && t < nb) {
        double x = Lkk[t][c];
        for (int q = 0; q < c; ++q) x -= Lkk[t][q] * Lkk[c][q];
        Lkk[t][c] = x / lcc;
      }
      __builtin_amdgcn_wave_barrier();
      if (t == 0) Lkk[c][c] = lcc;
      __builtin_amdgcn_wave_barrier();
    }
  }
  __syncthreads();
  if (bad != 0) {
    if (t == 0) {
      *info = bad;
      *logdet = __builtin_nan("");
    }
    return;
  }
  for (int e = t; e < kPanel * kPanel; e += TPB) {
    const int i = e / kPanel, j = e % kPanel;
    if (i < nb && j < nb && j <= i) L[(int64_t)(k0 + i) * d + k0 + j] = Lkk[i][j];
  }
  // rows below: L[i, panel] = A[i, panel] Lkk^{-T} (one row per thread: d - k0 - nb <= TPB)
  const int i = k0 + nb + t;
  if (i < d) {
    double y[kPanel];
#pragma unroll
    for (int q = 0; q < kPanel; ++q) y[q] = (q < nb) ? L[(int64_t)i * d + k0 + q] : 0.0;
    static_for<0, kPanel>([&](auto qq) {
      constexpr int q = decltype(qq)::value;
      if (q < nb) {
        double x = y[q];
#pragma unroll
        for (int p = 0; p < q; ++p) x -= y[p] * Lkk[q][p];
        y[q] = x / Lkk[q][q];
      }
    });
#pragma unroll
    for (int q = 0; q < kPanel; ++q)
      if (q < nb) L[(int64_t)i * d + k0 + q] = y[q];
  }
}

// lower-triangle update A[i][j] -= sum_q L[i][k0+q] L[j][k0+q], k0+nb <= j <= i < d,
// one workgroup per 64 x 64 tile (tile row >= tile column).
__global__ __launch_bounds__(256) void chol_update_kernel(int d, double* L, int k0, const int32_t* __restrict__ info) {
  __shared__ double Li[64][kPanel + 1];
  __shared__ double Lj[64][kPanel + 1];
  if (*info != 0) return;
  const int nb = min(kPanel, d - k0);
  const int base = k0 + nb;
  // decode the lower-triangular tile index
  int ti = 0;
  int rem = blockIdx.x;
  while (rem > ti) {
    rem -= ti + 1;
    ++ti;
  }
  const int tj = rem;
  const int i0 = base + ti * 64, j0 = base + tj * 64;
  const int t = threadIdx.x;
  for (int e = t; e < 64 * kPanel; e += 256) {
    const int r = e / kPanel, q = e % kPanel;
    Li[r][q] = (i0 + r < d && q < nb) ? L[(int64_t)(i0 + r) * d + k0 + q] : 0.0;
    Lj[r][q] = (j0 + r < d && q < nb) ? L[(int64_t)(j0 + r) * d + k0 + q] : 0.0;
  }
  __syncthreads();
  const int cj = t & 63;
  const int j = j0 + cj;
  for (int r = t >> 6; r < 64; r += 4) {
    const int i = i0 + r;
    if (i < d && j < d && j <= i) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < kPanel; ++q) s += Li[r][q] * Lj[cj][q];
      L[(int64_t)i * d + j] -= s;
    }
  }
}

__global__ void shift_lower_kernel(int d, double sigma2, double nu, const double* C, double* L,
                                   const int32_t* __restrict__ info) {
  if (*info != 0) return;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)d * d) return;
  const int i = (int)(e / d), j = (int)(e % d);
  // symmetrise C (read both halves, each thread writes its own entry), lower part of S into L
  const double s = 0.5 * (C[e] + C[(int64_t)j * d + i]);
  L[e] = (j <= i) ? s + (i == j ? sigma2 - nu : 0.0) : 0.0;
}

// C <- (C + C^T) / 2 in place (one thread per pair i < j).
__global__ void sym_kernel(int d, double* C, const int32_t* __restrict__ info) {
  if (*info != 0) return;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)d * d) return;
  const int i = (int)(e / d), j = (int)(e % d);
  if (i < j) {
    const double s = 0.5 * (C[e] + C[(int64_t)j * d + i]);
    C[e] = s;
    C[(int64_t)j * d + i] = s;
  }
}

__global__ __launch_bounds__(kCoreThreads) void logdet_kernel(int64_t n, int d, double sigma2, const double* L,
                                                              double* logdet, const int32_t* __restrict__ info) {
  __shared__ double red[kCoreWaves];
  if (*info != 0) return;
  double part = 0.0;
  for (int k = threadIdx.x; k < d; k += kCoreThreads) part += log(L[(int64_t)k * d + k]);
  const double s = block_sum(part, red);
  if (threadIdx.x == 0) *logdet = (double)(n - d) * log(sigma2) + 2.0 * s;
}

__global__ void init_info_kernel(const double* __restrict__ F, double* Flu, int64_t count, int32_t* info) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < count) Flu[e] = F[e];
  if (e == 0) *info = 0;
}

static hipError_t chol_logdet(hipStream_t st, int64_t n, int d, double sigma2, double* L, double* logdet,
                              int32_t* info);

hipError_t launch_core(hipStream_t st, int64_t n, int d, const double* F, const double* R, double sigma2, double nu,
                       double* Flu, int32_t* piv, double* C, double* L, double* logdet, int32_t* info) {
  const int64_t dd = (int64_t)d * d;
  const unsigned ddb = (unsigned)((dd + 255) / 256);
  hipLaunchKernelGGL(init_info_kernel, dim3(ddb), dim3(256), 0, st, F, Flu, dd, info);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int k0 = 0; k0 < d; k0 += kPanel) {
    // the smallest workgroup with a thread for each of the d - k0 panel rows
    const int rows = d - k0;
    if (rows <= 64) {
      hipLaunchKernelGGL(lu_panel_kernel<64>, dim3(1), dim3(64), 0, st, d, Flu, k0, piv, info, logdet);
    } else if (rows <= 128) {
      hipLaunchKernelGGL(lu_panel_kernel<128>, dim3(1), dim3(128), 0, st, d, Flu, k0, piv, info, logdet);
    } else if (rows <= 256) {
      hipLaunchKernelGGL(lu_panel_kernel<256>, dim3(1), dim3(256), 0, st, d, Flu, k0, piv, info, logdet);
    } else if (rows <= 512) {
      hipLaunchKernelGGL(lu_panel_kernel<512>, dim3(1), dim3(512), 0, st, d, Flu, k0, piv, info, logdet);
    } else {
      hipLaunchKernelGGL(lu_panel_kernel<kCoreThreads>, dim3(1), dim3(kCoreThreads), 0, st, d, Flu, k0, piv, info,
                         logdet);
    }
    const int kend = min(k0 + kPanel, d);
    const int nright = (d - kend + kLuCols - 1) / kLuCols;
    const int nblk = (k0 + kLuCols - 1) / kLuCols + nright;
    if (nblk > 0) hipLaunchKernelGGL(lu_swap_solve_kernel, dim3(nblk), dim3(256), 0, st, d, Flu, k0, piv, info);
    const int ntile = (d - kend + 63) / 64;
    if (ntile > 0) hipLaunchKernelGGL(lu_gemm_kernel, dim3(ntile, ntile), dim3(256), 0, st, d, Flu, k0, info);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // C = F^{-1} R^T: column c of R^T is row c of R
  if ((e = launch_trsm_cols(st, false, d, d, Flu, piv, 1, R, C, d, info)) != hipSuccess) return e;
  hipLaunchKernelGGL(shift_lower_kernel, dim3(ddb), dim3(256), 0, st, d, sigma2, nu, C, L, info);
  hipLaunchKernelGGL(sym_kernel, dim3(ddb), dim3(256), 0, st, d, C, info);
  return chol_logdet(st, n, d, sigma2, L, logdet, info);
}

__global__ void zero_info_kernel(int32_t* info) { *info = 0; }

hipError_t launch_chol_core(hipStream_t st, int64_t n, int d, const double* B, double sigma2, double* L,
                            double* logdet, int32_t* info) {
  const int64_t dd = (int64_t)d * d;
  const unsigned ddb = (unsigned)((dd + 255) / 256);
  hipLaunchKernelGGL(zero_info_kernel, dim3(1), dim3(1), 0, st, info);
  hipLaunchKernelGGL(shift_lower_kernel, dim3(ddb), dim3(256), 0, st, d, sigma2, 0.0, B, L, info);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return chol_logdet(st, n, d, sigma2, L, logdet, info);
}

// Cholesky of the lower part of S held in L (blocked, in place) and the
// log-determinant (n - d) log sigma2 + 2 sum log L_kk; a non-positive pivot
// sets *info and every later kernel does nothing.
static hipError_t chol_logdet(hipStream_t st, int64_t n, int d, double sigma2, double* L, double* logdet,
                              int32_t* info) {
  for (int k0 = 0; k0 < d; k0 += kPanel) {
    // the smallest workgroup with a thread for each row below the diagonal block
    const int below = d - min(k0 + kPanel, d);
    if (below <= 64) {
      hipLaunchKernelGGL(chol_panel_kernel<64>, dim3(1), dim3(64), 0, st, d, L, k0, info, logdet);
    } else if (below <= 128) {
      hipLaunchKernelGGL(chol_panel_kernel<128>, dim3(1), dim3(128), 0, st, d, L, k0, info, logdet);
    } else if (below <= 256) {
      hipLaunchKernelGGL(chol_panel_kernel<256>, dim3(1), dim3(256), 0, st, d, L, k0, info, logdet);
    } else if (below <= 512) {
      hipLaunchKernelGGL(chol_panel_kernel<512>, dim3(1), dim3(512), 0, st, d, L, k0, info, logdet);
    } else {
      hipLaunchKernelGGL(chol_panel_kernel<kCoreThreads>, dim3(1), dim3(kCoreThreads), 0, st, d, L, k0, info, logdet);
    }
    const int base = min(k0 + kPanel, d);
    const int nt = (d - base + 63) / 64;
    if (nt > 0) hipLaunchKernelGGL(chol_update_kernel, dim3(nt * (nt + 1) / 2), dim3(256), 0, st, d, L, k0, info);
  }
  hipLaunchKernelGGL(logdet_kernel, dim3(1), dim3(kCoreThreads), 0, st, n, d, sigma2, L, logdet, info);
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

hipError_t launch_core_apply(hipStream_t st, int d, int m, const double* L, const double* Z, double sigma2,
                             const int32_t* info, double* Wfull, double* Wmix) {
  if (m <= 0) return hipSuccess;
  hipError_t e = launch_trsm_cols(st, true, d, m, L, nullptr, 3, Z, Wfull, m, info);
  if (e != hipSuccess) return e;
  return launch_wmix(st, (int64_t)d * m, Wfull, Z, sigma2, info, Wmix);
}

// ------------------------------------------------------------------ backward scalars

// Contractions of the adjoint from the d x d and d x m products (one workgroup):
//   log-likelihood: u = Phi^T a, T = S^{-1} Phi, G2 = Phi^T S^{-1} Phi,
//     d/dlog ell    = u.h - <T, P> - (u.E u - <G2, E>) / 2
//     d/dlog s      = a.C a - <S^{-1}, C>
//     d/dlog sigma2 = sigma2 (alpha^T alpha - (n - d) / sigma2 - tr S^{-1}) / 2
//   solve: U1 = Phi^T QX, U2 = Phi^T QB,
//     d/dlog ell    = -(<U2, XY^T> + <U1, BY^T>) + (<U1, E U2> + <U2, E U1>) / 2
//     d/dlog s      = -2 <QX, C QB>
//     d/dlog sigma2 = -sigma2 tr(X^T B)
//   with a shift nu (v1 = R^{-1} a, o = Omega^T alpha, OO = Omega^T Omega):
//     log-likelihood: d/dlog ell += -nu (h - P^T a).v1
//                     d/dlog s   += -2 nu (u.o - tr S^{-1}) + nu (u.OO u - <G2, OO>)
//                                   + 2 nu^2 (o - F a).v1
//     solve (M1 = XY - QX^T P, M2 = BY - QB^T P, Z1 = R^{-1} QB, Z2 = R^{-1} QX):
//                     d/dlog ell += nu (<M1^T, Z1> + <M2^T, Z2>)
//                     d/dlog s   += 2 nu (<U2, Omega^T X> + <U1, Omega^T B>) - 2 nu <U1, OO U2>
//                                   - 2 nu^2 (<Omega^T X - F QX, Z1> + <Omega^T B - F QB, Z2>)
__global__ __launch_bounds__(kCoreThreads) void backward_scalars_kernel(BackwardScalars b) {
  __shared__ double red[kCoreWaves];
  const int t = threadIdx.x;
  const int d = b.d;
  const int64_t dd = (int64_t)d * d;
  if (b.mode == 0) {
    double p_uh = 0.0, p_uEu = 0.0, p_aCa = 0.0, p_tr = 0.0;
    for (int i = t; i < d; i += kCoreThreads) {
      p_uh += b.u[i] * b.h[i];
      p_uEu += b.u[i] * b.Eu[i];
      p_aCa += b.a[i] * b.Ca[i];
      p_tr += b.Sinv[(int64_t)i * d + i];
    }
    double p_tp = 0.0, p_ge = 0.0, p_sc = 0.0;
    for (int64_t e = t; e < dd; e += kCoreThreads) {
      p_tp += b.T[e] * b.P[e];
      p_ge += b.G2[e] * b.E[e];
      p_sc += b.Sinv[e] * b.C[e];
    }
    const double uh = block_sum(p_uh, red);
    const double uEu = block_sum(p_uEu, red);
    const double aCa = block_sum(p_aCa, red);
    const double trs = block_sum(p_tr, red);
    const double tp = block_sum(p_tp, red);
    const double ge = block_sum(p_ge, red);
    const double sc = block_sum(p_sc, red);
    double x_ell = 0.0, x_s = 0.0;
    if (b.nu != 0.0) {
      double q_hv = 0.0, q_uo = 0.0, q_uu = 0.0, q_ov = 0.0, q_g = 0.0;
      for (int i = t; i < d; i += kCoreThreads) {
        q_hv += (b.h[i] - b.Pta[i]) * b.v1[i];
        q_uo += b.u[i] * b.oa[i];
        q_uu += b.u[i] * (b.OOu != nullptr ? b.OOu[i] : b.u[i]);
        q_ov += (b.oa[i] - b.Fa[i]) * b.v1[i];
        if (b.OO == nullptr) q_g += b.G2[(int64_t)i * d + i];
      }
      if (b.OO != nullptr)
        for (int64_t e = t; e < dd; e += kCoreThreads) q_g += b.G2[e] * b.OO[e];
      const double hv = block_sum(q_hv, red);
      const double uo = block_sum(q_uo, red);
      const double uu = block_sum(q_uu, red);
      const double ov = block_sum(q_ov, red);
      const double g2oo = block_sum(q_g, red);
      x_ell = -b.nu * hv;
      x_s = -2.0 * b.nu * (uo - trs) + b.nu * (uu - g2oo) + 2.0 * b.nu * b.nu * ov;
    }
    if (t == 0) {
      const double t2 = 0.5 * (uEu - ge);
      b.dtheta[0] = uh - tp - t2 + x_ell;
      b.dtheta[1] = aCa - sc + x_s;
      b.dtheta[2] = b.sigma2 * 0.5 * (b.aa[0] - ((double)(b.n - d) / b.sigma2 + trs));
    }
  } else {
    const int m = b.m;
    const int64_t dm = (int64_t)d * m;
    double p_t1 = 0.0, p_t2 = 0.0, p_mc = 0.0, p_xb = 0.0;
    for (int64_t e = t; e < dm; e += kCoreThreads) {
      const int i = (int)(e / m), c = (int)(e % m);
      p_t1 += b.U2[e] * b.XY[(int64_t)c * d + i] + b.U1[e] * b.BY[(int64_t)c * d + i];
      p_t2 += b.U1[e] * b.EU2[e] + b.U2[e] * b.EU1[e];
      p_mc += b.QX[e] * b.CQB[e];
    }
    for (int c = t; c < m; c += kCoreThreads) p_xb += b.XB[(int64_t)c * m + c];
    const double t1 = block_sum(p_t1, red);
    const double t2 = block_sum(p_t2, red);
    const double mc = block_sum(p_mc, red);
    const double xb = block_sum(p_xb, red);
    double x_ell = 0.0, x_s = 0.0;
    if (b.nu != 0.0) {
      double q_mz = 0.0, q_uo = 0.0, q_uu = 0.0, q_oz = 0.0;
      for (int64_t e = t; e < dm; e += kCoreThreads) {
        const int i = (int)(e / m), c = (int)(e % m);
        q_mz += b.M1[(int64_t)c * d + i] * b.Z1[e] + b.M2[(int64_t)c * d + i] * b.Z2[e];
        q_uo += b.U2[e] * b.OX[e] + b.U1[e] * b.OB[e];
        q_uu += b.U1[e] * (b.OOU2 != nullptr ? b.OOU2[e] : b.U2[e]);
        q_oz += (b.OX[e] - b.FQX[e]) * b.Z1[e] + (b.OB[e] - b.FQB[e]) * b.Z2[e];
      }
      const double mz = block_sum(q_mz, red);
      const double uo = block_sum(q_uo, red);
      const double uu = block_sum(q_uu, red);
      const double oz = block_sum(q_oz, red);
      x_ell = b.nu * mz;
      x_s = 2.0 * b.nu * uo - 2.0 * b.nu * uu - 2.0 * b.nu * b.nu * oz;
    }
    if (t == 0) {
      b.dtheta[0] = -t1 + 0.5 * t2 + x_ell;
      b.dtheta[1] = -2.0 * mc + x_s;
      b.dtheta[2] = -b.sigma2 * xb;
    }
  }
}

hipError_t launch_backward_scalars(hipStream_t st, const BackwardScalars& b) {
  hipLaunchKernelGGL(backward_scalars_kernel, dim3(1), dim3(kCoreThreads), 0, st, b);
  return hipGetLastError();
}

}  // namespace lr
