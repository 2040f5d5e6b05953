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
//    description: X(r, k) = signs[r] (-1)^popcount(r & cols[k]) (times c);
//    against a row-major real matrix it takes the fast transform instead
//    (launch_srht_left, sketch.hip) whenever the workspace holds a slab.
//  * rowmix: out = alpha A + Q W, W d x m float64, one wave per 16 rows x 16
//    columns, products and sums in float64 with one rounding at the end.
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace lr {

constexpr int kTnFlushSteps = 16;  // 16 steps of 32 rows

// Output tile (bx, by) and row chunk bz of a transposed-product workgroup
// (grid: M tiles x N tiles x row chunks). Workgroups go to the 8 XCDs round
// robin by linear id, so in launch order the tiles of one row chunk would
// read its rows of X and Y into every L2. Here each XCD takes whole row
// chunks: its k-th workgroup is tile k mod (nx ny) of chunk xcd + 8 k / (nx ny).
// A bijection when the chunk count is a multiple of 8; otherwise the launch
// order is kept.
__device__ __forceinline__ void xcd_tile(int& bx, int& by, int& bz) {
  const int nx = (int)gridDim.x, ny = (int)gridDim.y, nz = (int)gridDim.z;
  if (nz % 8 != 0) {
    bx = (int)blockIdx.x;
    by = (int)blockIdx.y;
    bz = (int)blockIdx.z;
    return;
  }
  const int64_t lin = (int64_t)blockIdx.x + (int64_t)nx * ((int64_t)blockIdx.y + (int64_t)ny * blockIdx.z);
  const int64_t k = lin / 8;
  const int64_t t = k % ((int64_t)nx * ny);
  bz = (int)(lin % 8 + 8 * (k / ((int64_t)nx * ny)));
  bx = (int)(t % nx);
  by = (int)(t / nx);
}

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
  int bx, by, bz;
  xcd_tile(bx, by, bz);
  const int i0 = bx * 64 + (w & 1) * 32;
  const int j0 = by * 64 + (w >> 1) * 32;
  const int64_t rbeg = (int64_t)bz * chunk;
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
  double* out = partial + (int64_t)bz * M * N;
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

// Fast path of the same product for X a transposed dense Omega (float or bf16
// bits, 8 consecutive rows of a column in one 16-byte load) and Y a row-major
// float matrix (4 consecutive columns in one 16-byte load). A workgroup owns
// a 64 x 128 block of the output, each wave 32 x 64: its 4 column tiles take
// the columns j0 + 4 l + t (l = lane mod 16, t = tile), so every lane loads
// whole 16-byte rows of Y. Steps of 32 rows run in pairs with two register
// sets, the next step's loads issued before the current step's 64 products;
// float accumulators are added to float64 ones every kTnFlushSteps steps.
template <int XDT>
__global__ __launch_bounds__(256) void gemm_tn_xt_kernel(int64_t n, int64_t chunk, int M, int N,
                                                         const void* __restrict__ xptr, int64_t xld,
                                                         const float* __restrict__ Y, int64_t yld,
                                                         double* __restrict__ partial) {
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int fl = lane & 15, fg = lane >> 4;
  int bx, by, bz;
  xcd_tile(bx, by, bz);
  const int i0 = bx * 64 + (w & 1) * 32;
  const int j0 = by * 128 + (w >> 1) * 64;
  const int64_t rbeg = (int64_t)bz * chunk;
  int64_t rend = rbeg + chunk;
  if (rend > n) rend = n;

  f32x4_t acc[2][4];
  double acc64[2][4][4];
#pragma unroll
  for (int f = 0; f < 2; ++f)
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        acc[f][t][q] = 0.0f;
        acc64[f][t][q] = 0.0;
      }
  struct Step {
    float x[2][8];   // float Omega
    uint4 xr[2];     // bf16 Omega, 8 rows of a column as loaded
    float y[8][4];
  };
  // rows r0 + 8 fg + e; FULL: all 32 rows < rend
  auto load_step = [&](int64_t r0, Step& st, bool full) {
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      const int64_t col = i0 + 16 * f + fl;
      const int64_t rr = r0 + 8 * fg;
      // a group starting below rend ends inside the column (rr and ld are
      // multiples of 8 and ld >= n); a group starting at or past rend is zero
      if (!full && rr >= rend) {
#pragma unroll
        for (int e = 0; e < 8; ++e) st.x[f][e] = 0.0f;
        st.xr[f] = uint4{0u, 0u, 0u, 0u};
        continue;
      }
      if constexpr (XDT == 2) {
        const uint16_t* src = static_cast<const uint16_t*>(xptr) + col * xld + rr;
        uint4 raw = *reinterpret_cast<const uint4*>(src);
        if (!full) {  // rows past rend: element 2q is the low half of word q
          uint32_t wv[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            if (rr + 2 * q >= rend) wv[q] &= 0xffff0000u;
            if (rr + 2 * q + 1 >= rend) wv[q] &= 0x0000ffffu;
          }
          raw = uint4{wv[0], wv[1], wv[2], wv[3]};
        }
        st.xr[f] = raw;
        continue;
      } else {
        const float* src = static_cast<const float*>(xptr) + col * xld + rr;
        const float4 a = *reinterpret_cast<const float4*>(src);
        const float4 b = *reinterpret_cast<const float4*>(src + 4);
        st.x[f][0] = a.x; st.x[f][1] = a.y; st.x[f][2] = a.z; st.x[f][3] = a.w;
        st.x[f][4] = b.x; st.x[f][5] = b.y; st.x[f][6] = b.z; st.x[f][7] = b.w;
      }
      if (!full) {
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if (rr + e >= rend) st.x[f][e] = 0.0f;
      }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t r = r0 + 8 * fg + e;
      if (full || r < rend) {
        const float4 v = *reinterpret_cast<const float4*>(Y + r * yld + j0 + 4 * fl);
        st.y[e][0] = v.x; st.y[e][1] = v.y; st.y[e][2] = v.z; st.y[e][3] = v.w;
      } else {
        st.y[e][0] = st.y[e][1] = st.y[e][2] = st.y[e][3] = 0.0f;
      }
    }
  };
  auto mma_step = [&](const Step& st) {
    if constexpr (XDT == 2) {
      // bf16 Omega: each float of Y is the exact sum of three bf16 terms
      // (8 + 8 + 8 significand bits), and a bf16 x bf16 product is exact in
      // float, so three bf16 matrix-core products per tile give the float
      // product with float accumulation, at the bf16 rate
      bf16x8_t a[2];
#pragma unroll
      for (int f = 0; f < 2; ++f) __builtin_memcpy(&a[f], &st.xr[f], 16);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        bf16x8_t hi, mid, lo;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float v = st.y[e][t];
          const __bf16 h = (__bf16)v;
          const float r1 = v - (float)h;
          const __bf16 m = (__bf16)r1;
          hi[e] = h;
          mid[e] = m;
          lo[e] = (__bf16)(r1 - (float)m);
        }
#pragma unroll
        for (int f = 0; f < 2; ++f) {
          acc[f][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[f], hi, acc[f][t], 0, 0, 0);
          acc[f][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[f], mid, acc[f][t], 0, 0, 0);
          acc[f][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[f], lo, acc[f][t], 0, 0, 0);
        }
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e)
#pragma unroll
        for (int f = 0; f < 2; ++f)
#pragma unroll
          for (int t = 0; t < 4; ++t)
            acc[f][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(st.x[f][e], st.y[e][t], acc[f][t], 0, 0, 0);
    }
  };
  auto flush = [&]() {
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          acc64[f][t][q] += (double)acc[f][t][q];
          acc[f][t][q] = 0.0f;
        }
  };

  const int64_t nfull = (rend - rbeg) / 32;  // complete steps
  int64_t k = 0;
  if (nfull > 0) {
    Step s0, s1;
    // the load past the last complete step re-reads it and is unused
    auto rowk = [&](int64_t kk) { return rbeg + 32 * (kk < nfull ? kk : nfull - 1); };
    load_step(rowk(0), s0, true);
    for (; k + 1 < nfull; k += 2) {
      load_step(rowk(k + 1), s1, true);
      mma_step(s0);
      load_step(rowk(k + 2), s0, true);
      mma_step(s1);
      if ((k / 2) % (kTnFlushSteps / 2) == kTnFlushSteps / 2 - 1) flush();
    }
    if (k < nfull) {
      mma_step(s0);
      ++k;
    }
  }
  if (rbeg + 32 * k < rend) {  // ragged last step
    Step s2;
    load_step(rbeg + 32 * k, s2, false);
    mma_step(s2);
  }
  flush();
  double* out = partial + (int64_t)bz * M * N;
#pragma unroll
  for (int f = 0; f < 2; ++f)
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = i0 + 16 * f + acc_row<f32x4_t>(fg, q);
        const int col = j0 + 4 * fl + t;
        out[(int64_t)row * N + col] = acc64[f][t][q];
      }
}

__global__ void fill_kernel(double* __restrict__ out, int64_t count, double v) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx < count) out[idx] = v;
}

// out (d x ld, j contiguous) = Q^T for a row-major n x d Q, columns n .. ld-1
// zeroed: the transposed dense-Omega layout, so Q can stand in for Omega in
// a second sketch pass. 32 x 32 tiles through LDS keep both sides coalesced.
template <typename T>
__global__ void transpose_kernel(int64_t n, int d, const T* __restrict__ Q, int64_t ld, T* __restrict__ out) {
  __shared__ T tile[32][33];
  const int64_t j0 = (int64_t)blockIdx.x * 32;
  const int c0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 8 rows per pass
  for (int r = ty; r < 32; r += 8) {
    const int64_t j = j0 + r;
    const int c = c0 + tx;
    tile[r][tx] = (j < n && c < d) ? Q[j * d + c] : (T)0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int c = c0 + r;
    const int64_t j = j0 + tx;
    if (c < d && j < ld) out[(int64_t)c * ld + j] = tile[tx][r];
  }
}

hipError_t launch_transpose(hipStream_t st, int64_t n, int d, const void* Q, int64_t ld, void* out, bool f64) {
  const dim3 grid((unsigned)((ld + 31) / 32), (unsigned)((d + 31) / 32));
  if (f64)
    hipLaunchKernelGGL(transpose_kernel<double>, grid, dim3(256), 0, st, n, d, (const double*)Q, ld, (double*)out);
  else
    hipLaunchKernelGGL(transpose_kernel<float>, grid, dim3(256), 0, st, n, d, (const float*)Q, ld, (float*)out);
  return hipGetLastError();
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

// out[idx] = scale * sum_c partial[c * count + idx] with one wave per output:
// lane l sums partials l, l + 64, ... in order, then a fixed butterfly adds the
// lanes (the same order on every call).
__global__ __launch_bounds__(256) void reduce_partials_wave_kernel(const double* __restrict__ partial, int64_t nchunk,
                                                                   int64_t count, double scale,
                                                                   double* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (idx >= count) return;
  double s = 0.0;
  for (int64_t c = lane; c < nchunk; c += 64) s += partial[c * count + idx];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) out[idx] = scale * s;
}

static hipError_t launch_reduce_partials(hipStream_t st, const double* partial, int64_t nch, int64_t count,
                                         double scale, double* out) {
  if (nch >= 128 && count < 65536)
    hipLaunchKernelGGL(reduce_partials_wave_kernel, dim3((unsigned)((count + 3) / 4)), dim3(256), 0, st, partial, nch,
                       count, scale, out);
  else
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, partial, nch,
                       count, scale, out);
  return hipGetLastError();
}

// Rows per partial of the general product: 1024 or more, at most 64 partials
// (short products still spread over many workgroups).
static int64_t tn_chunk(int64_t n) {
  int64_t chunk = 1024;
  while ((n + chunk - 1) / chunk > 64) chunk *= 2;
  return chunk;
}

// Skinny products (row-major X n x M, M <= 1024, against row-major Y n x N,
// N <= 16: Z = Q^T A, Q^T y): one workgroup per chunk of rows, every thread
// owns the columns t, t + 256, ... of X against all N columns of Y, whose row
// is the same for the whole workgroup (scalar loads). Products of float inputs
// are exact in float64 (a float64 Y, as in Y'^T u, gives rounded float64
// products); all sums are float64.
constexpr int kSkinnyMaxM = 1024;
constexpr int kSkinnyMaxN = 16;
static int64_t skinny_chunk(int64_t n) {
  int64_t chunk = 256;
  while ((n + chunk - 1) / chunk > 1024) chunk *= 2;
  return chunk;
}

size_t tn_workspace(int64_t n, int M, int N) {
  const int64_t chunk = tn_chunk(n);
  const int64_t nch = (n + chunk - 1) / chunk;
  size_t b = (size_t)(nch < 1 ? 1 : nch) * (size_t)M * (size_t)N * sizeof(double);
  // room for a skinny product of any M' <= M, N' <= N as well
  const int ms = M < kSkinnyMaxM ? M : kSkinnyMaxM;
  const int nsk = N < kSkinnyMaxN ? N : kSkinnyMaxN;
  const int64_t ns = (n + skinny_chunk(n) - 1) / skinny_chunk(n);
  const size_t bs = (size_t)(ns < 1 ? 1 : ns) * (size_t)ms * (size_t)nsk * sizeof(double);
  return bs > b ? bs : b;
}

template <typename RX, typename RY, int CPM, int NN>
__global__ __launch_bounds__(256) void gemm_tn_skinny_kernel(int64_t n, int64_t chunk, int M, int N,
                                                             const RX* __restrict__ X, int64_t ldx,
                                                             const RY* __restrict__ Y, int64_t ldy,
                                                             double* __restrict__ partial) {
  // the Y rows of the current 256-row tile, converted to float64 once (thread
  // t converts row t); every thread then reads each row as a broadcast
  __shared__ double ytile[256][NN];
  const int t = threadIdx.x;
  const int64_t rbeg = (int64_t)blockIdx.x * chunk;
  const int64_t rend = rbeg + chunk < n ? rbeg + chunk : n;
  double acc[CPM][NN];
#pragma unroll
  for (int c = 0; c < CPM; ++c)
#pragma unroll
    for (int k = 0; k < NN; ++k) acc[c][k] = 0.0;
  for (int64_t r0 = rbeg; r0 < rend; r0 += 256) {
    const int rows = rend - r0 < 256 ? (int)(rend - r0) : 256;
    {
      const int64_t r = r0 + t;
#pragma unroll
      for (int k = 0; k < NN; ++k) ytile[t][k] = (t < rows && k < N) ? (double)Y[r * ldy + k] : 0.0;
    }
    __syncthreads();
    // eight rows of X per trip, all loads issued before the products
    constexpr int kRows = 8;
    for (int i0 = 0; i0 < rows; i0 += kRows) {
      RX qv[kRows][CPM];
#pragma unroll
      for (int u = 0; u < kRows; ++u) {
        const int64_t r = r0 + i0 + u;
#pragma unroll
        for (int c = 0; c < CPM; ++c) {
          const int col = t + 256 * c;
          qv[u][c] = (i0 + u < rows && col < M) ? X[r * ldx + col] : (RX)0;
        }
      }
#pragma unroll
      for (int u = 0; u < kRows; ++u) {
        const int i = i0 + u < rows ? i0 + u : rows - 1;  // rows past the tile add q = 0
#pragma unroll
        for (int c = 0; c < CPM; ++c) {
          const double q = (double)qv[u][c];
#pragma unroll
          for (int k = 0; k < NN; ++k) acc[c][k] = __builtin_fma(q, ytile[i][k], acc[c][k]);
        }
      }
    }
    __syncthreads();
  }
  double* out = partial + (int64_t)blockIdx.x * M * N;
#pragma unroll
  for (int c = 0; c < CPM; ++c) {
    const int col = t + 256 * c;
    if (col < M) {
#pragma unroll
      for (int k = 0; k < NN; ++k)
        if (k < N) out[(int64_t)col * N + k] = acc[c][k];
    }
  }
}

template <typename RX, typename RY, int CPM>
static hipError_t launch_skinny_cpm(hipStream_t st, int64_t n, int64_t chunk, int64_t nch, int M, int N,
                                    const RX* X, int64_t ldx, const RY* Y, int64_t ldy, double* partial) {
  const dim3 g((unsigned)nch), b(256);
  if (N <= 1)
    hipLaunchKernelGGL((gemm_tn_skinny_kernel<RX, RY, CPM, 1>), g, b, 0, st, n, chunk, M, N, X, ldx, Y, ldy,
                       partial);
  else if (N <= 4)
    hipLaunchKernelGGL((gemm_tn_skinny_kernel<RX, RY, CPM, 4>), g, b, 0, st, n, chunk, M, N, X, ldx, Y, ldy,
                       partial);
  else if (N <= 8)
    hipLaunchKernelGGL((gemm_tn_skinny_kernel<RX, RY, CPM, 8>), g, b, 0, st, n, chunk, M, N, X, ldx, Y, ldy,
                       partial);
  else
    hipLaunchKernelGGL((gemm_tn_skinny_kernel<RX, RY, CPM, 16>), g, b, 0, st, n, chunk, M, N, X, ldx, Y, ldy,
                       partial);
  return hipGetLastError();
}

template <typename RX, typename RY>
static hipError_t launch_skinny(hipStream_t st, int64_t n, int64_t chunk, int64_t nch, int M, int N, const RX* X,
                                int64_t ldx, const RY* Y, int64_t ldy, double* partial) {
  if (M <= 256) return launch_skinny_cpm<RX, RY, 1>(st, n, chunk, nch, M, N, X, ldx, Y, ldy, partial);
  if (M <= 512) return launch_skinny_cpm<RX, RY, 2>(st, n, chunk, nch, M, N, X, ldx, Y, ldy, partial);
  return launch_skinny_cpm<RX, RY, 4>(st, n, chunk, nch, M, N, X, ldx, Y, ldy, partial);
}

hipError_t launch_gemm_tn(hipStream_t st, int64_t n, int M, int N, const TnOperand& X, const TnOperand& Y,
                          double x_scale, double* out, void* ws, bool f64) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int64_t count = (int64_t)M * N;
  if (n <= 0) return launch_fill(st, out, count, 0.0);
  const int64_t chunk = tn_chunk(n);
  const int64_t nch = (n + chunk - 1) / chunk;
  double* partial = static_cast<double*>(ws);
  // an SRHT Omega against a row-major real matrix: the fast transform, column
  // by column, when a slab of at least one transform chunk fits the workspace
  if (X.kind == 2 && Y.kind == 0 && (Y.dtype == 0 || Y.dtype == 1) && Y.ld == N) {
    const size_t elem = Y.dtype == 0 ? sizeof(double) : sizeof(float);
    const int64_t S = srht_left_slab(n, M, N, elem, (size_t)nch * M * N * sizeof(double));
    if (S > 0) {
      if (Y.dtype == 0)
        return launch_srht_left<double>(st, n, M, X.signs, X.cols, static_cast<const double*>(Y.ptr), N, x_scale, out,
                                        ws, S);
      return launch_srht_left<float>(st, n, M, X.signs, X.cols, static_cast<const float*>(Y.ptr), N, x_scale, out, ws,
                                     S);
    }
  }
  // fast path: transposed float/bf16 Omega against a row-major float matrix
  const bool y16 = Y.kind == 0 && Y.dtype == 1 && Y.ld % 4 == 0 && reinterpret_cast<uintptr_t>(Y.ptr) % 16 == 0;
  const bool x16 = X.kind == 1 && (X.dtype == 1 || X.dtype == 2) && X.ld % 8 == 0 &&
                   reinterpret_cast<uintptr_t>(X.ptr) % 16 == 0;
  if (!f64 && x16 && y16 && M % 64 == 0 && N % 128 == 0) {
    dim3 g2(M / 64, N / 128, (unsigned)nch);
    if (X.dtype == 2)
      hipLaunchKernelGGL(gemm_tn_xt_kernel<2>, g2, dim3(256), 0, st, n, chunk, M, N, X.ptr, X.ld,
                         static_cast<const float*>(Y.ptr), Y.ld, partial);
    else
      hipLaunchKernelGGL(gemm_tn_xt_kernel<1>, g2, dim3(256), 0, st, n, chunk, M, N, X.ptr, X.ld,
                         static_cast<const float*>(Y.ptr), Y.ld, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, partial,
                       nch, count, x_scale, out);
    return hipGetLastError();
  }
  // skinny real x real products (float64 sums; products of float inputs are
  // exact, a float64 operand makes them rounded float64 products)
  const bool mixed = X.dtype == 1 && Y.dtype == 0;
  if (X.kind == 0 && Y.kind == 0 && (X.dtype == Y.dtype || mixed) && X.dtype != 2 && M <= kSkinnyMaxM &&
      N <= kSkinnyMaxN && (f64 || X.dtype == 1)) {
    const int64_t sc = skinny_chunk(n);
    const int64_t ns = (n + sc - 1) / sc;
    hipError_t e;
    if (X.dtype == 0)
      e = launch_skinny(st, n, sc, ns, M, N, static_cast<const double*>(X.ptr), X.ld,
                        static_cast<const double*>(Y.ptr), Y.ld, partial);
    else if (mixed)
      e = launch_skinny(st, n, sc, ns, M, N, static_cast<const float*>(X.ptr), X.ld, static_cast<const double*>(Y.ptr),
                        Y.ld, partial);
    else
      e = launch_skinny(st, n, sc, ns, M, N, static_cast<const float*>(X.ptr), X.ld, static_cast<const float*>(Y.ptr),
                        Y.ld, partial);
    if (e != hipSuccess) return e;
    return launch_reduce_partials(st, partial, ns, count, x_scale, out);
  }
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

// out = alpha A + Q W with the products and sums in float64 (float64 matrix
// cores; float inputs are exact in float64) and one rounding to RO at the
// end. W (d x m, float64) is read straight from L2: 16 lanes read 16
// consecutive entries of a row of W.
template <typename RI, typename RO>
__global__ __launch_bounds__(256) void rowmix_kernel(int64_t n, int d, int m, const RI* __restrict__ Q,
                                                     const double* __restrict__ W, double alpha,
                                                     const RI* __restrict__ A, RO* __restrict__ out,
                                                     const int32_t* __restrict__ info) {
  if (info != nullptr && *info != 0) return;
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int fl = lane & 15, fg = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * 64 + w * 16;
  const int64_t arow = row0 + fl;
  const bool row_ok = arow < n;
  const int col = blockIdx.y * 16 + fl;
  const bool col_ok = col < m;
  f64x4_t acc = f64x4_t{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < d; k0 += 32) {
    double a[8], b[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = k0 + 8 * fg + e;
      a[e] = (row_ok && k < d) ? (double)Q[arow * d + k] : 0.0;
      b[e] = (col_ok && k < d) ? W[(int64_t)k * m + col] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[e], b[e], acc, 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t row = row0 + acc_row<f64x4_t>(fg, i);
    if (row < n && col_ok) out[row * m + col] = (RO)(alpha * (double)A[row * m + col] + acc[i]);
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
  if (f64)
    hipLaunchKernelGGL((rowmix_kernel<double, double>), grid, dim3(256), 0, st, n, d, m, (const double*)Q, W, alpha,
                       (const double*)A, (double*)out, info);
  else
    hipLaunchKernelGGL((rowmix_kernel<float, float>), grid, dim3(256), 0, st, n, d, m, (const float*)Q, W, alpha,
                       (const float*)A, (float*)out, info);
  return hipGetLastError();
}

hipError_t launch_rowmix_f64out(hipStream_t st, int64_t n, int d, int m, const void* Q, const double* W,
                                double alpha, const void* A, double* out, bool in_f64) {
  if (m <= 0 || n <= 0) return hipSuccess;
  dim3 grid((unsigned)((n + 63) / 64), (unsigned)((m + 15) / 16));
  if (in_f64)
    hipLaunchKernelGGL((rowmix_kernel<double, double>), grid, dim3(256), 0, st, n, d, m, (const double*)Q, W, alpha,
                       (const double*)A, out, nullptr);
  else
    hipLaunchKernelGGL((rowmix_kernel<float, double>), grid, dim3(256), 0, st, n, d, m, (const float*)Q, W, alpha,
                       (const float*)A, out, nullptr);
  return hipGetLastError();
}

__global__ void narrow_kernel(int64_t count, const double* __restrict__ in, float* __restrict__ out) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx < count) out[idx] = (float)in[idx];
}

hipError_t launch_narrow(hipStream_t st, int64_t count, const double* in, float* out) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(narrow_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, count, in, out);
  return hipGetLastError();
}

__global__ void wmix_kernel(int64_t count, const double* __restrict__ W, const double* __restrict__ Z,
                            double inv_sigma2, const int32_t* __restrict__ info, double* __restrict__ out) {
  if (info != nullptr && *info != 0) return;
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx < count) out[idx] = W[idx] - Z[idx] * inv_sigma2;
}

hipError_t launch_wmix(hipStream_t st, int64_t count, const double* W, const double* Z, double sigma2,
                       const int32_t* info, double* out) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(wmix_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, count, W, Z, 1.0 / sigma2,
                     info, out);
  return hipGetLastError();
}

}  // namespace lr
