// Tall-skinny products of the Woodbury stage and the backward pass.
//
//  * gemm_tn: out = sum_r X(r, :)^T Y(r, :) for n rows (F = Omega^T Q,
//    Z = Q^T A, Q^T Y', Omega^T Y', ...). Rows are split into chunks, one
//    workgroup per (64 x 64 output tile, chunk); a wave owns a 32 x 32 tile and
//    runs matrix-core FMAs over 32-row steps (lane group g holds rows 8g..8g+7,
//    so every lane reads 8 consecutive rows of a transposed Omega in one load).
//    float inputs accumulate in float32 for at most 512 rows and are then added
//    to a float64 accumulator; chunk partials are float64 and are summed in a
//    fixed order. The SRHT operand is generated from its sign/column
//    description: X(r, k) = signs[r] (-1)^popcount(r & cols[k]) (times c).
//  * rowmix: out = alpha A + Q W, W d x m (float64, staged in LDS as the
//    working precision), one wave per 16 rows x 16 columns.
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace lr {

constexpr int kTnFlushSteps = 16;  // 16 steps of 32 rows

template <typename R>
struct Frag8 {
  R v[8];
};

template <typename R>
__device__ __forceinline__ R load_as(const void* p, int dtype, int64_t idx) {
  if (dtype == 0) return (R) static_cast<const double*>(p)[idx];
  if (dtype == 1) return (R) static_cast<const float*>(p)[idx];
  uint32_t bits = (uint32_t) static_cast<const uint16_t*>(p)[idx] << 16;
  float f;
  __builtin_memcpy(&f, &bits, 4);
  return (R)f;
}

// X(r0 + e, col) for e = 0..7 (zero outside rows [.., rend) or col >= ncols).
template <typename R>
__device__ __forceinline__ void load_tn8(const TnOperand& op, int64_t r0, int64_t rend, int col, int ncols,
                                         int pk, Frag8<R>& f) {
  const bool col_ok = col < ncols;
  if (op.kind == 2) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t r = r0 + e;
      R v = 0;
      if (col_ok && r < rend) {
        const unsigned par = __popcll((unsigned long long)r & (unsigned long long)(unsigned)pk) & 1u;
        const R sg = op.signs[r] < 0 ? (R)-1 : (R)1;
        v = par ? -sg : sg;
      }
      f.v[e] = v;
    }
    return;
  }
  if (op.kind == 1) {
    // transposed: element (r, col) at col * ld + r, 8 consecutive r
    const int64_t base = (int64_t)(col_ok ? col : 0) * op.ld;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t r = r0 + e;
      f.v[e] = (col_ok && r < rend) ? load_as<R>(op.ptr, op.dtype, base + r) : (R)0;
    }
    return;
  }
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int64_t r = r0 + e;
    f.v[e] = (col_ok && r < rend) ? load_as<R>(op.ptr, op.dtype, r * op.ld + col) : (R)0;
  }
}

template <typename R>
__device__ __forceinline__ void mfma8(typename std::conditional<sizeof(R) == 4, f32x4_t, f64x4_t>::type& acc,
                                      const Frag8<R>& a, const Frag8<R>& b) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    if constexpr (sizeof(R) == 4)
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[e], b.v[e], acc, 0, 0, 0);
    else
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a.v[e], b.v[e], acc, 0, 0, 0);
  }
}

template <typename R>
__global__ __launch_bounds__(256) void gemm_tn_kernel(int64_t n, int64_t chunk, int M, int N, TnOperand X,
                                                      TnOperand Y, double* __restrict__ partial) {
  using Acc = typename std::conditional<sizeof(R) == 4, f32x4_t, f64x4_t>::type;
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int fl = lane & 15, fg = lane >> 4;
  const int i0 = blockIdx.x * 64 + (w & 1) * 32;
  const int j0 = blockIdx.y * 64 + (w >> 1) * 32;
  const int64_t rbeg = (int64_t)blockIdx.z * chunk;
  int64_t rend = rbeg + chunk;
  if (rend > n) rend = n;

  int pki[2] = {0, 0}, pkj[2] = {0, 0};
#pragma unroll
  for (int f = 0; f < 2; ++f) {
    const int ci = i0 + 16 * f + fl, cj = j0 + 16 * f + fl;
    if (X.kind == 2 && ci < M) pki[f] = X.cols[ci];
    if (Y.kind == 2 && cj < N) pkj[f] = Y.cols[cj];
  }

  Acc acc[2][2];
  double acc64[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        acc[a][b][i] = 0;
        acc64[a][b][i] = 0;
      }

  int step = 0;
  for (int64_t r0 = rbeg; r0 < rend; r0 += 32, ++step) {
    Frag8<R> xa[2], yb[2];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      load_tn8<R>(X, r0 + 8 * fg, rend, i0 + 16 * f + fl, M, pki[f], xa[f]);
      load_tn8<R>(Y, r0 + 8 * fg, rend, j0 + 16 * f + fl, N, pkj[f], yb[f]);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) mfma8<R>(acc[a][b], xa[a], yb[b]);
    if constexpr (sizeof(R) == 4) {
      if (step % kTnFlushSteps == kTnFlushSteps - 1) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              acc64[a][b][i] += (double)acc[a][b][i];
              acc[a][b][i] = 0;
            }
      }
    }
  }
  double* out = partial + (int64_t)blockIdx.z * M * N;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = i0 + 16 * a + acc_row<Acc>(fg, i);
        const int col = j0 + 16 * b + fl;
        if (row < M && col < N) out[(int64_t)row * N + col] = acc64[a][b][i] + (double)acc[a][b][i];
      }
}

__global__ void fill_kernel(double* __restrict__ out, int64_t count, double v) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx < count) out[idx] = v;
}

hipError_t launch_fill(hipStream_t st, double* out, int64_t count, double v) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, out, count, v);
  return hipGetLastError();
}

__global__ void identity_kernel(double* __restrict__ X, int d) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx < (int64_t)d * d) X[idx] = (idx / d == idx % d) ? 1.0 : 0.0;
}

hipError_t launch_identity(hipStream_t st, double* X, int d) {
  const int64_t count = (int64_t)d * d;
  hipLaunchKernelGGL(identity_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, X, d);
  return hipGetLastError();
}

__global__ void reduce_partials_kernel(const double* __restrict__ partial, int64_t nchunk, int64_t count,
                                       double scale, double* __restrict__ out) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= count) return;
  double s = 0;
  for (int64_t c = 0; c < nchunk; ++c) s += partial[c * count + idx];
  out[idx] = scale * s;
}

static int64_t tn_chunk(int64_t n) {
  int64_t chunk = 4096;
  while ((n + chunk - 1) / chunk > 64) chunk *= 2;
  return chunk;
}

size_t tn_workspace(int64_t n, int M, int N) {
  const int64_t chunk = tn_chunk(n);
  const int64_t nch = (n + chunk - 1) / chunk;
  return (size_t)(nch < 1 ? 1 : nch) * (size_t)M * (size_t)N * sizeof(double);
}

hipError_t launch_gemm_tn(hipStream_t st, int64_t n, int M, int N, const TnOperand& X, const TnOperand& Y,
                          double x_scale, double* out, void* ws, bool f64) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int64_t count = (int64_t)M * N;
  if (n <= 0) return launch_fill(st, out, count, 0.0);
  const int64_t chunk = tn_chunk(n);
  const int64_t nch = (n + chunk - 1) / chunk;
  double* partial = static_cast<double*>(ws);
  dim3 grid((M + 63) / 64, (N + 63) / 64, (unsigned)nch);
  if (f64)
    hipLaunchKernelGGL(gemm_tn_kernel<double>, grid, dim3(256), 0, st, n, chunk, M, N, X, Y, partial);
  else
    hipLaunchKernelGGL(gemm_tn_kernel<float>, grid, dim3(256), 0, st, n, chunk, M, N, X, Y, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, partial, nch,
                     count, x_scale, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ rowmix

template <typename R>
__global__ __launch_bounds__(256) void rowmix_kernel(int64_t n, int d, int m, const R* __restrict__ Q,
                                                     const double* __restrict__ W, R alpha,
                                                     const R* __restrict__ A, R* __restrict__ out,
                                                     const int32_t* __restrict__ info) {
  using Acc = typename std::conditional<sizeof(R) == 4, f32x4_t, f64x4_t>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* Ws = reinterpret_cast<R*>(smem_raw);  // d x 16
  if (info != nullptr && *info != 0) return;
  const int c0 = blockIdx.y * 16;
  for (int idx = threadIdx.x; idx < d * 16; idx += blockDim.x) {
    const int k = idx / 16, c = idx % 16;
    Ws[idx] = (c0 + c < m) ? (R)W[(int64_t)k * m + c0 + c] : (R)0;
  }
  __syncthreads();
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int fl = lane & 15, fg = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * 64 + w * 16;
  const int64_t arow = row0 + fl;
  const bool row_ok = arow < n;
  Acc acc;
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = 0;
  for (int k0 = 0; k0 < d; k0 += 32) {
    Frag8<R> a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = k0 + 8 * fg + e;
      a.v[e] = (row_ok && k < d) ? Q[arow * d + k] : (R)0;
      b.v[e] = (k < d) ? Ws[k * 16 + fl] : (R)0;
    }
    mfma8<R>(acc, a, b);
  }
  const int col = c0 + fl;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t row = row0 + acc_row<Acc>(fg, i);
    if (row < n && col < m) out[row * m + col] = alpha * A[row * m + col] + (R)acc[i];
  }
}

hipError_t launch_rowmix(hipStream_t st, int64_t n, int d, int m, const void* Q, const double* W, double alpha,
                         const void* A, void* out, bool f64) {
  return launch_rowmix_info(st, n, d, m, Q, W, alpha, A, out, f64, nullptr);
}

hipError_t launch_rowmix_info(hipStream_t st, int64_t n, int d, int m, const void* Q, const double* W, double alpha,
                              const void* A, void* out, bool f64, const int32_t* info) {
  if (m <= 0 || n <= 0) return hipSuccess;
  dim3 grid((unsigned)((n + 63) / 64), (unsigned)((m + 15) / 16));
  if (f64) {
    const size_t lds = (size_t)d * 16 * sizeof(double);
    hipError_t e = hipFuncSetAttribute((const void*)rowmix_kernel<double>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(rowmix_kernel<double>, grid, dim3(256), lds, st, n, d, m, (const double*)Q, W, alpha,
                       (const double*)A, (double*)out, info);
  } else {
    const size_t lds = (size_t)d * 16 * sizeof(float);
    hipError_t e = hipFuncSetAttribute((const void*)rowmix_kernel<float>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(rowmix_kernel<float>, grid, dim3(256), lds, st, n, d, m, (const float*)Q, W, (float)alpha,
                       (const float*)A, (float*)out, info);
  }
  return hipGetLastError();
}

}  // namespace lr
