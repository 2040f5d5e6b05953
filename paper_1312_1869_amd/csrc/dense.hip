// Dense float64 building blocks of the d x d core and of the adjoint (d <= 1024).
//
//  * gemm_dd: out = alpha op(A) op(B) + beta out, row-major float64, op = identity
//    or transpose. One 256-thread workgroup per 64 x 64 output tile; the
//    operands pass through LDS in 16-deep slices and every wave runs 2 x 2
//    float64 16x16x4 matrix-core tiles.
//  * trsm_cols: solves with many right-hand sides. Each workgroup owns kTrNc
//    right-hand-side columns, keeps them whole in LDS (d x kTrNc doubles) and
//    sweeps the triangle in blocks of 64 rows: the rows of a block first take
//    the contribution of every solved block (factor tiles staged through LDS,
//    the next tile requested while the current one is used, two outputs per
//    thread), then one wave per two columns finishes the
//    64 x 64 diagonal triangle with the row held by its lane and the solved
//    entries broadcast lane to lane. Modes:
//      LU:       X <- U^{-1} L^{-1} P X for the getrf factors of F (row
//                exchanges in order, unit lower L, upper U, packed row-major);
//      Cholesky: X <- L^{-T} L^{-1} X for a lower factor L (S = L L^T).
//    Right-hand sides come from X itself, from another d x nrhs matrix, from
//    the rows of a matrix (column c is row c of src: F^{-1} R^T), or from the
//    identity (an inverse). A third mode applies only an upper triangle
//    (R^{-1} B for the TSQR factor).
//  * lu_apply: F B from the getrf factors of F.
//  * psd_part: the positive semidefinite part V max(Lambda, 0) V^T of a
//    symmetric matrix (the eig-clip core), without an eigendecomposition:
//    B+ = (B + B sign(B)) / 2 with sign(B) from the Newton-Schulz iteration
//    X <- X (3I - X^2) / 2 started at B / ||B||_F. Every eigenvalue of X stays
//    in [-1, 1] and moves towards its sign, by a factor 1.5 per step while
//    small and quadratically near +-1; an eigenvalue still unresolved when
//    the steps end is one below ~1e-13 ||B||, whose clipping cannot matter at
//    float64 precision. Two gemm_dd per step, all on float64 matrix cores.
#include "common.hpp"
#include "kernels.hpp"

namespace lr {

// ------------------------------------------------------------------ gemm_dd

constexpr int kGdTile = 64;
constexpr int kGdK = 16;

__global__ __launch_bounds__(256) void gemm_dd_kernel(int M, int N, int K, double alpha, const double* __restrict__ A,
                                                      int lda, bool ta, const double* __restrict__ B, int ldb, bool tb,
                                                      double beta, double* __restrict__ out, int ldo) {
  __shared__ double As[kGdTile][kGdK + 1];  // As[i][k] = op(A)[i0 + i][k0 + k]
  __shared__ double Bs[kGdK][kGdTile + 1];  // Bs[k][j] = op(B)[k0 + k][j0 + j]
  const int t = threadIdx.x;
  const int w = t >> 6, lane = t & 63;
  const int fl = lane & 15, fg = lane >> 4;
  const int i0 = blockIdx.x * kGdTile, j0 = blockIdx.y * kGdTile;
  const int wi = (w & 1) * 32, wj = (w >> 1) * 32;
  f64x4_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4_t{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += kGdK) {
    // 64 x 16 slice of op(A) and 16 x 64 slice of op(B), 4 elements per thread each
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = t + 256 * e;
      int i, k;
      if (ta) {  // A stored K x M: read along i
        i = idx & 63;
        k = idx >> 6;
      } else {   // A stored M x K: read along k
        i = idx >> 4;
        k = idx & 15;
      }
      const int gi = i0 + i, gk = k0 + k;
      double v = 0.0;
      if (gi < M && gk < K) v = ta ? A[(int64_t)gk * lda + gi] : A[(int64_t)gi * lda + gk];
      As[i][k] = v;
      int kk, j;
      if (tb) {  // B stored N x K: read along k
        j = idx >> 4;
        kk = idx & 15;
      } else {   // B stored K x N: read along j
        j = idx & 63;
        kk = idx >> 6;
      }
      const int gj = j0 + j, gkk = k0 + kk;
      double u = 0.0;
      if (gj < N && gkk < K) u = tb ? B[(int64_t)gj * ldb + gkk] : B[(int64_t)gkk * ldb + gj];
      Bs[kk][j] = u;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kGdK; ks += 4) {
      double av[2], bv[2];
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        av[f] = As[wi + 16 * f + fl][ks + fg];
        bv[f] = Bs[ks + fg][wj + 16 * f + fl];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = i0 + wi + 16 * a + acc_row<f64x4_t>(fg, q);
        const int col = j0 + wj + 16 * b + fl;
        if (row < M && col < N) {
          double* o = out + (int64_t)row * ldo + col;
          *o = alpha * acc[a][b][q] + (beta == 0.0 ? 0.0 : beta * *o);
        }
      }
}

hipError_t launch_gemm_dd(hipStream_t st, int M, int N, int K, double alpha, const double* A, int lda, bool ta,
                          const double* B, int ldb, bool tb, double beta, double* out, int ldo) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 grid((unsigned)((M + kGdTile - 1) / kGdTile), (unsigned)((N + kGdTile - 1) / kGdTile));
  hipLaunchKernelGGL(gemm_dd_kernel, grid, dim3(256), 0, st, M, N, K, alpha, A, lda, ta, B, ldb, tb, beta, out, ldo);
  return hipGetLastError();
}

// ------------------------------------------------------------------ trsm_cols

constexpr int kTrNc = 8;     // right-hand-side columns per workgroup
constexpr int kTrBlk = 64;   // rows per block
constexpr int kTrQ = 32;     // factor columns staged per update step
constexpr int kTrMaxD = 1024;
static_assert(kTrQ <= kTrBlk && (kTrQ * kTrBlk) % 256 == 0, "factor tiles fit the 64 x 65 LDS tile");

// Factor entry of the triangle being applied (row r, column q of the triangle).
//   LU lower:  F[r][q] (unit diagonal)    LU upper:  F[r][q]
//   Chol lower: L[r][q]                   Chol upper (L^T): L[q][r]
template <bool CHOL, bool UPPER>
__device__ __forceinline__ double tri_at(const double* __restrict__ Fm, int d, int r, int q) {
  if (CHOL && UPPER) return Fm[(int64_t)q * d + r];
  return Fm[(int64_t)r * d + q];
}

// One triangle sweep over the LDS columns xs (d x kTrNc, row-major).
template <bool CHOL, bool UPPER>
__device__ void trsm_sweep(const double* __restrict__ Fm, int d, double* xs, double (*tile)[kTrBlk + 1]) {
  constexpr bool UNIT = !CHOL && !UPPER;
  const int t = threadIdx.x;
  const int w = t >> 6, lane = t & 63;
  const int nblk = (d + kTrBlk - 1) / kTrBlk;
  // update mapping: rows 2 * (t / 8) and 2 * (t / 8) + 1 of the block, column t % 8
  const int ur = 2 * (t >> 3), uc = t & 7;
  for (int bi = 0; bi < nblk; ++bi) {
    const int blk = UPPER ? nblk - 1 - bi : bi;
    const int r0 = blk * kTrBlk;
    const int nb = min(kTrBlk, d - r0);
    // solved rows: [0, r0) for the lower triangle, [r0 + nb, d) for the upper one
    const int qbeg = UPPER ? r0 + nb : 0;
    const int qend = UPPER ? d : r0;
    double s0 = 0.0, s1 = 0.0;
    // the factor tile of step q0 + kTrQ is requested into registers before
    // the products of step q0, so its load latency overlaps them
    constexpr int kPer = kTrQ * kTrBlk / 256;
    auto fetch = [&](int q0, double (&dst)[kPer]) {
      const int nq = min(kTrQ, qend - q0);
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int e = t + 256 * u;
        int q, r;
        if (CHOL && UPPER) {  // contiguous along r
          r = e % kTrBlk;
          q = e / kTrBlk;
        } else {              // contiguous along q
          q = e % kTrQ;
          r = e / kTrQ;
        }
        dst[u] = (q < nq && r < nb) ? tri_at<CHOL, UPPER>(Fm, d, r0 + r, q0 + q) : 0.0;
      }
    };
    double pre[kPer];
    if (qbeg < qend) fetch(qbeg, pre);
    for (int q0 = qbeg; q0 < qend; q0 += kTrQ) {
      const int nq = min(kTrQ, qend - q0);
      // tile[q][r] = T(r0 + r, q0 + q)
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int e = t + 256 * u;
        if (CHOL && UPPER)
          tile[e / kTrBlk][e % kTrBlk] = pre[u];
        else
          tile[e % kTrQ][e / kTrQ] = pre[u];
      }
      __syncthreads();
      if (q0 + kTrQ < qend) fetch(q0 + kTrQ, pre);
      for (int q = 0; q < nq; ++q) {
        const double xq = xs[(q0 + q) * kTrNc + uc];
        s0 = fma(tile[q][ur], xq, s0);
        s1 = fma(tile[q][ur + 1], xq, s1);
      }
      __syncthreads();
    }
    if (ur < nb) xs[(r0 + ur) * kTrNc + uc] -= s0;
    if (ur + 1 < nb) xs[(r0 + ur + 1) * kTrNc + uc] -= s1;
    // diagonal block into the tile: tile[q][r] = T(r0 + r, r0 + q)
    for (int e = t; e < kTrBlk * kTrBlk; e += 256) {
      const int r = e >> 6, q = e & 63;
      tile[q][r] = (q < nb && r < nb) ? tri_at<CHOL, UPPER>(Fm, d, r0 + r, r0 + q) : 0.0;
    }
    __syncthreads();
    // wave w finishes columns 2w and 2w + 1; lane = row of the block
    {
      const int c0 = 2 * w;
      const bool row_ok = lane < nb;
      double x0 = row_ok ? xs[(r0 + lane) * kTrNc + c0] : 0.0;
      double x1 = row_ok ? xs[(r0 + lane) * kTrNc + c0 + 1] : 0.0;
      const double dinv = (UNIT || !row_ok) ? 1.0 : 1.0 / tile[lane][lane];
      for (int jj = 0; jj < nb; ++jj) {
        const int j = UPPER ? nb - 1 - jj : jj;
        if (lane == j) {
          x0 *= dinv;
          x1 *= dinv;
        }
        const double xj0 = __shfl(x0, j, 64);
        const double xj1 = __shfl(x1, j, 64);
        const bool after = UPPER ? lane < j : lane > j;
        if (after && row_ok) {
          const double f = tile[j][lane];
          x0 = fma(-f, xj0, x0);
          x1 = fma(-f, xj1, x1);
        }
      }
      if (row_ok) {
        xs[(r0 + lane) * kTrNc + c0] = x0;
        xs[(r0 + lane) * kTrNc + c0 + 1] = x1;
      }
    }
    __syncthreads();
  }
}

// src_kind: 0 = X itself, 1 = column c is row c of src (src d x d), 2 = identity,
// 3 = src (d x nrhs, leading dimension ldx).
// MODE: 0 = LU (getrf factors, piv may be NULL for none), 1 = Cholesky,
// 2 = upper triangle of Fm only (X <- U^{-1} B, e.g. U = R).
template <int MODE>
__global__ __launch_bounds__(256) void trsm_cols_kernel(int d, int nrhs, const double* __restrict__ Fm,
                                                        const int32_t* __restrict__ piv, int src_kind,
                                                        const double* __restrict__ src, double* X, int ldx,
                                                        const int32_t* __restrict__ info) {
  __shared__ double xs[kTrMaxD * kTrNc];
  __shared__ double tile[kTrBlk][kTrBlk + 1];
  if (info != nullptr && *info != 0) return;
  const int t = threadIdx.x;
  const int c0 = blockIdx.x * kTrNc;
  for (int e = t; e < d * kTrNc; e += 256) {
    const int i = e / kTrNc, c = e % kTrNc;
    const int col = c0 + c;
    double v = 0.0;
    if (col < nrhs) {
      if (src_kind == 0) v = X[(int64_t)i * ldx + col];
      else if (src_kind == 1) v = src[(int64_t)col * d + i];
      else if (src_kind == 2) v = (i == col) ? 1.0 : 0.0;
      else v = src[(int64_t)i * ldx + col];
    }
    xs[e] = v;
  }
  __syncthreads();
  constexpr bool CHOL = MODE == 1;
  if (MODE == 0 && piv != nullptr) {
    // row exchanges in factorisation order, one thread per column
    if (t < kTrNc) {
      for (int k = 0; k < d; ++k) {
        const int p = piv[k];
        if (p != k && p >= 0 && p < d) {
          const double a = xs[k * kTrNc + t];
          xs[k * kTrNc + t] = xs[p * kTrNc + t];
          xs[p * kTrNc + t] = a;
        }
      }
    }
    __syncthreads();
  }
  if (MODE != 2) trsm_sweep<CHOL, false>(Fm, d, xs, tile);
  trsm_sweep<CHOL, true>(Fm, d, xs, tile);
  for (int e = t; e < d * kTrNc; e += 256) {
    const int i = e / kTrNc, c = e % kTrNc;
    if (c0 + c < nrhs) X[(int64_t)i * ldx + c0 + c] = xs[e];
  }
}

hipError_t launch_trsm_cols(hipStream_t st, bool chol, int d, int nrhs, const double* Fm, const int32_t* piv,
                            int src_kind, const double* src, double* X, int ldx, const int32_t* info) {
  if (nrhs <= 0) return hipSuccess;
  if (d < 1 || d > kTrMaxD) return hipErrorInvalidValue;
  dim3 grid((unsigned)((nrhs + kTrNc - 1) / kTrNc));
  if (chol)
    hipLaunchKernelGGL(trsm_cols_kernel<1>, grid, dim3(256), 0, st, d, nrhs, Fm, piv, src_kind, src, X, ldx, info);
  else
    hipLaunchKernelGGL(trsm_cols_kernel<0>, grid, dim3(256), 0, st, d, nrhs, Fm, piv, src_kind, src, X, ldx, info);
  return hipGetLastError();
}

hipError_t launch_trsm_upper(hipStream_t st, int d, int nrhs, const double* U, const double* src, double* X,
                             int ldx) {
  if (nrhs <= 0) return hipSuccess;
  if (d < 1 || d > kTrMaxD) return hipErrorInvalidValue;
  dim3 grid((unsigned)((nrhs + kTrNc - 1) / kTrNc));
  hipLaunchKernelGGL(trsm_cols_kernel<2>, grid, dim3(256), 0, st, d, nrhs, U, nullptr, 3, src, X, ldx, nullptr);
  return hipGetLastError();
}

// ------------------------------------------------------------------ lu_apply

// out = F B for F = P^T L U given by its getrf factors (B, out d x nrhs with
// leading dimension ld; one workgroup per column, the column in LDS):
// t = U b, t = L t (unit lower), then the row exchanges undone last to first.
__global__ __launch_bounds__(256) void lu_apply_kernel(int d, int nrhs, const double* __restrict__ Flu,
                                                       const int32_t* __restrict__ piv, const double* __restrict__ B,
                                                       double* __restrict__ out, int ld) {
  __shared__ double b[kTrMaxD];
  __shared__ double t[kTrMaxD];
  const int c = blockIdx.x;
  for (int i = threadIdx.x; i < d; i += 256) b[i] = B[(int64_t)i * ld + c];
  __syncthreads();
  for (int i = threadIdx.x; i < d; i += 256) {  // (U b)_i = sum_{k >= i} U[i][k] b_k
    double s = 0.0;
    for (int k = i; k < d; ++k) s = fma(Flu[(int64_t)i * d + k], b[k], s);
    t[i] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < d; i += 256) {  // (L t)_i = t_i + sum_{k < i} L[i][k] t_k
    double s = t[i];
    for (int k = 0; k < i; ++k) s = fma(Flu[(int64_t)i * d + k], t[k], s);
    b[i] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = d - 1; k >= 0; --k) {
      const int p = piv[k];
      if (p != k && p >= 0 && p < d) {
        const double x = b[k];
        b[k] = b[p];
        b[p] = x;
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < d; i += 256) out[(int64_t)i * ld + c] = b[i];
}

hipError_t launch_lu_apply(hipStream_t st, int d, int nrhs, const double* Flu, const int32_t* piv, const double* B,
                           double* out, int ld) {
  if (nrhs <= 0) return hipSuccess;
  if (d < 1 || d > kTrMaxD) return hipErrorInvalidValue;
  hipLaunchKernelGGL(lu_apply_kernel, dim3((unsigned)nrhs), dim3(256), 0, st, d, nrhs, Flu, piv, B, out, ld);
  return hipGetLastError();
}

// ------------------------------------------------------------------ psd_part

// X0 = B / ||B||_F (one workgroup: the norm, then the scaled copy).
__global__ __launch_bounds__(1024) void frob_scale_kernel(int d, const double* __restrict__ B, double* __restrict__ X) {
  __shared__ double red[16];
  const int64_t dd = (int64_t)d * d;
  double part = 0.0;
  for (int64_t e = threadIdx.x; e < dd; e += blockDim.x) part += B[e] * B[e];
  for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
  __syncthreads();
  double tot = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += red[w];
  const double inv = tot > 0.0 ? 1.0 / sqrt(tot) : 0.0;
  for (int64_t e = threadIdx.x; e < dd; e += blockDim.x) X[e] = B[e] * inv;
}

// out = c I (d x d)
__global__ void scaled_identity_kernel(int d, double c, double* __restrict__ out) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < (int64_t)d * d) out[e] = (e / d == e % d) ? c : 0.0;
}

// M <- (M + M^T) / 2 in place (one thread per entry pair i < j).
__global__ void symmetrize_kernel(int d, double* __restrict__ M) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)d * d) return;
  const int i = (int)(e / d), j = (int)(e % d);
  if (i < j) {
    const double v = 0.5 * (M[e] + M[(int64_t)j * d + i]);
    M[e] = v;
    M[(int64_t)j * d + i] = v;
  }
}

hipError_t launch_symmetrize(hipStream_t st, int d, double* M) {
  const int64_t dd = (int64_t)d * d;
  hipLaunchKernelGGL(symmetrize_kernel, dim3((unsigned)((dd + 255) / 256)), dim3(256), 0, st, d, M);
  return hipGetLastError();
}

hipError_t launch_psd_part(hipStream_t st, int d, const double* B, double* Bplus, double* ws, int steps) {
  const int64_t dd = (int64_t)d * d;
  const unsigned ddb = (unsigned)((dd + 255) / 256);
  double* X = ws;
  double* Xn = ws + dd;
  double* T = ws + 2 * dd;
  hipLaunchKernelGGL(frob_scale_kernel, dim3(1), dim3(1024), 0, st, d, B, X);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int k = 0; k < steps; ++k) {
    hipLaunchKernelGGL(scaled_identity_kernel, dim3(ddb), dim3(256), 0, st, d, 3.0, T);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_gemm_dd(st, d, d, d, -1.0, X, d, false, X, d, false, 1.0, T, d)) != hipSuccess) return e;
    if ((e = launch_gemm_dd(st, d, d, d, 0.5, X, d, false, T, d, false, 0.0, Xn, d)) != hipSuccess) return e;
    double* t = X;
    X = Xn;
    Xn = t;
  }
  // B+ = B / 2 + B X / 2, then exact symmetry
  if ((e = hipMemcpyAsync(Bplus, B, dd * sizeof(double), hipMemcpyDeviceToDevice, st)) != hipSuccess) return e;
  if ((e = launch_gemm_dd(st, d, d, d, 0.5, B, d, false, X, d, false, 0.5, Bplus, d)) != hipSuccess) return e;
  return launch_symmetrize(st, d, Bplus);
}

}  // namespace lr
