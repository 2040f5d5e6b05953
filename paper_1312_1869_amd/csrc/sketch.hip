// Sketch Y = (K_f + nu I) Omega with K_f evaluated on the fly (Sec. 3.1-3.2).
//
// This file: the points prescale and the SRHT kernel (sketch_dense.hip holds the
// dense-Omega kernel).
//  * sketch_srht_kernel: Omega = c D H P (Def. 1, Walsh-Hadamard T). Row i of
//    Y is c (H (D o k_i))[P]. With H_n = H_{n/2048} (x) H_2048, each 2048-long
//    chunk j1 of D o k_i is transformed in full (11 butterfly stages: 5 over
//    the register index, an LDS transpose, 5 more and one lane swap), and
//    every selected output P_k = p1 * 2048 + p2 adds (-1)^popcount(j1 & p1)
//    times entry p2 of the chunk transform. A wave owns two rows (float; they
//    share every point load) or one row with its value and derivative sketch
//    (the fused mode); lane l owns outputs l, l+64, ... Work per row:
//    n (11 + 1) butterflies/adds + d n / 2048 selections, against the 2 n d of
//    the dense product the structure avoids (Sec. 1, Sec. 3.2).
//  * sketch_srht_grid_kernel: the same transform for a batch of
//    hyperparameters sharing the points' loads and squared distances.
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace lr {

// ------------------------------------------------------------------ prescale

// Rows n .. n + kPointPad - 1 are written as zeros (padding for kernels that
// read whole steps of columns).
template <typename T>
__global__ void prep_points_kernel(const float* __restrict__ X, int64_t n, int D, int PD, T scale,
                                   const int8_t* __restrict__ signs, T* __restrict__ out) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n + kPointPad) return;
  if (j >= n) {
    for (int t = 0; t < PD; ++t) out[j * PD + t] = (T)0;
    return;
  }
  for (int t = 0; t < PD - 1; ++t) out[j * PD + t] = (t < D) ? (T)X[j * D + t] * scale : (T)0;
  out[j * PD + PD - 1] = (signs != nullptr && signs[j] < 0) ? (T)-1 : (T)1;
}

template <typename T>
hipError_t launch_prep_points(hipStream_t st, const float* X, int64_t n, int D, int PD, double scale,
                              const int8_t* signs, T* out) {
  const int threads = 256;
  const int64_t blocks = (n + kPointPad + threads - 1) / threads;
  hipLaunchKernelGGL(prep_points_kernel<T>, dim3((unsigned)blocks), dim3(threads), 0, st, X, n, D, PD,
                     (T)scale, signs, out);
  return hipGetLastError();
}
template hipError_t launch_prep_points<float>(hipStream_t, const float*, int64_t, int, int, double,
                                              const int8_t*, float*);
template hipError_t launch_prep_points<double>(hipStream_t, const float*, int64_t, int, int, double,
                                               const int8_t*, double*);

// ------------------------------------------------------------------ SRHT

constexpr int kChunk = 2048;        // chunk of j transformed at once
constexpr int kChunkRegs = kChunk / 64;
constexpr int kBufWords = 2112;     // per wave: 32 x 65 (transpose) and 64 x 33 (selection) layouts
constexpr int kLoadGroup = 8;       // point loads issued together
constexpr int kGridPass = 2;        // hyperparameters per pass of the grid kernel

template <typename T, int N>
__device__ __forceinline__ void fwht_regs(T (&v)[N]) {
#pragma unroll
  for (int h = 1; h < N; h <<= 1) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      if ((i & h) == 0) {
        T a = v[i], b = v[i + h];
        v[i] = a + b;
        v[i + h] = a - b;
      }
    }
  }
}

template <typename T, int PD>
struct PointLoad;
template <>
struct PointLoad<float, 4> {
  __device__ __forceinline__ static void get(const float* p, float (&o)[4]) {
    float4 v = *reinterpret_cast<const float4*>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  }
};
template <>
struct PointLoad<double, 4> {
  __device__ __forceinline__ static void get(const double* p, double (&o)[4]) {
    double2 a = *reinterpret_cast<const double2*>(p);
    double2 b = *reinterpret_cast<const double2*>(p + 2);
    o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
  }
};
template <typename T, int PD>
struct PointLoadGeneric {
  __device__ __forceinline__ static void get(const T* p, T (&o)[PD]) {
#pragma unroll
    for (int t = 0; t < PD; ++t) o[t] = p[t];
  }
};
template <> struct PointLoad<float, 8> : PointLoadGeneric<float, 8> {};
template <> struct PointLoad<float, 16> : PointLoadGeneric<float, 16> {};
template <> struct PointLoad<double, 8> : PointLoadGeneric<double, 8> {};
template <> struct PointLoad<double, 16> : PointLoadGeneric<double, 16> {};

// Walsh-Hadamard transform of one 2048-long chunk and accumulation of its
// selected entries. On entry register r of lane l holds chunk entry r*64 + l.
//   1. stages over entry bits 6..10: butterflies across the 32 registers;
//   2. LDS transpose (32 x 65 words): lane l then holds entries l*32 + t;
//   3. stages over bits 0..4 across the registers, and bit 5 (lane bit 0)
//      by a lane swap (DPP quad_perm [1,0,3,2]);
//   4. the transformed chunk goes to LDS (64 x 33 words) and each selected
//      output P_k = p1 * 2048 + p2 adds (-1)^popcount(chunk & p1) times entry p2.
template <typename T, int NQ>
__device__ __forceinline__ void srht_chunk_accumulate(T (&v)[kChunkRegs], T* buf, int lane, int64_t chunk,
                                                      const int (&pk)[NQ], int d, T (&acc)[NQ]) {
  fwht_regs(v);
#pragma unroll
  for (int r = 0; r < kChunkRegs; ++r) buf[r * 65 + lane] = v[r];
  __builtin_amdgcn_wave_barrier();
  const int rbase = (lane >> 1) * 65 + (lane & 1) * 32;
#pragma unroll
  for (int t = 0; t < kChunkRegs; ++t) v[t] = buf[rbase + t];
  __builtin_amdgcn_wave_barrier();
  fwht_regs(v);
  const T sgn = (lane & 1) ? (T)-1 : (T)1;
#pragma unroll
  for (int t = 0; t < kChunkRegs; ++t) {
    const T partner = dpp_move<0xB1>(v[t]);
    v[t] = __builtin_fma(sgn, v[t], partner);
  }
#pragma unroll
  for (int t = 0; t < kChunkRegs; ++t) buf[lane * 33 + t] = v[t];
  __builtin_amdgcn_wave_barrier();
  const unsigned hi = (unsigned)chunk;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int k = lane + 64 * q;
    if (k < d) {
      const int p2 = pk[q] & (kChunk - 1);
      const T val = buf[(p2 >> 5) * 33 + (p2 & 31)];
      const unsigned par = __popc(hi & (unsigned)(pk[q] >> 11)) & 1u;
      acc[q] += par ? -val : val;
    }
  }
  __builtin_amdgcn_wave_barrier();
}

// MODE: 0 = Y only, 1 = Yprime only, 2 = both (fused, one kernel evaluation).
// R rows per wave (they share every point load); NV = R value vectors, or 2
// (value and derivative) in the fused mode with R = 1.
template <typename T, int KERNEL, int PD, int ND, int NQ, int MODE, int R>
__global__ __launch_bounds__(256) void sketch_srht_kernel(const T* __restrict__ pts,
                                                          const int32_t* __restrict__ cols, int64_t n,
                                                          int d, T scale_out, T nu_c,
                                                          T* __restrict__ Y, T* __restrict__ Yp) {
  static_assert(MODE != 2 || R == 1, "the fused mode keeps two vectors of one row");
  constexpr int NV = MODE == 2 ? 2 : R;
  __shared__ __align__(16) T smem[4 * kBufWords];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  T* buf = smem + wave * kBufWords;
  using K = KernelT<T, KERNEL>;

  int pk[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int k = lane + 64 * q;
    pk[q] = (k < d) ? cols[k] : 0;
  }
  const int64_t nchunks = (n + kChunk - 1) / kChunk;
  const int64_t ngroups = (n + 4 * R - 1) / (4 * R);

  for (int64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
    const int64_t i0 = g * (4 * R) + (int64_t)wave * R;
    T xi[R][PD];
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      const int64_t i = i0 + rr < n ? i0 + rr : n - 1;
      PointLoad<T, PD>::get(pts + i * PD, xi[rr]);
    }
    T acc[NV][NQ];
#pragma unroll
    for (int u = 0; u < NV; ++u)
#pragma unroll
      for (int q = 0; q < NQ; ++q) acc[u][q] = 0;

    for (int64_t c = 0; c < nchunks; ++c) {
      const int64_t base = c * kChunk;
      // entries past n (a partial chunk when n < 2048) read row n of the
      // point array, a zero row whose sign slot is 0, so they contribute 0
      const int last = (int)(n - base < kChunk ? n - base : kChunk);
      const T* cpts = pts + base * PD;
      T v[NV][kChunkRegs];
#pragma unroll
      for (int r = 0; r < kChunkRegs; ++r) {
        // at most kLoadGroup point loads in flight per wave
        if (r % kLoadGroup == 0) __builtin_amdgcn_sched_barrier(0);
        int jl = r * 64 + lane;
        jl = jl < last ? jl : last;
        T pj[PD];
        PointLoad<T, PD>::get(cpts + jl * PD, pj);
        const T sg = pj[PD - 1];
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
          T r2 = 0;
#pragma unroll
          for (int t = 0; t < ND; ++t) {
            const T df = xi[rr][t] - pj[t];
            r2 = __builtin_fma(df, df, r2);
          }
          if constexpr (MODE == 0) {
            v[rr][r] = sg * K::value(r2);
          } else if constexpr (MODE == 1) {
            v[rr][r] = sg * K::deriv(r2);
          } else {
            T val, dval;
            K::both(r2, val, dval);
            v[0][r] = sg * val;
            v[1][r] = sg * dval;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < NV; ++u) srht_chunk_accumulate<T, NQ>(v[u], buf, lane, c, pk, d, acc[u]);
    }

#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int rr = MODE == 2 ? 0 : u;
      const int64_t i = i0 + rr;
      if (i >= n) continue;
      T* out = (MODE == 1 || (MODE == 2 && u == 1)) ? Yp : Y;
      const bool value = !(MODE == 1 || (MODE == 2 && u == 1));
      const T sgi = xi[rr][PD - 1];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int k = lane + 64 * q;
        if (k < d) {
          T y = scale_out * acc[u][q];
          if (value && nu_c != (T)0) {
            const unsigned par = __popcll((unsigned long long)i & (unsigned long long)pk[q]) & 1u;
            y += par ? -nu_c * sgi : nu_c * sgi;
          }
          out[i * d + k] = y;
        }
      }
    }
  }
}

// Grid mode (a batch of hyperparameters, Sec. 5.2's grids over the range
// parameter): the points are prescaled for ell = 1, so one squared distance
// per (i, j) serves every hyperparameter g of the pass; kernel g evaluates it
// at r2 * a_g (a_g = 1/ell_g^2) and runs its own transform accumulation. One
// row per wave, G hyperparameters per pass; outputs Y_g = Y + g * ystride
// scaled by so_g = c s_g^2.
template <typename T>
struct GridPass {
  T a[kGridPass];
  T so[kGridPass];
  int64_t yoff[kGridPass];
};

template <typename T, int KERNEL, int PD, int ND, int NQ, int G>
__global__ __launch_bounds__(256) void sketch_srht_grid_kernel(const T* __restrict__ pts,
                                                               const int32_t* __restrict__ cols, int64_t n, int d,
                                                               GridPass<T> gp, T nu_c, T* __restrict__ Y) {
  __shared__ __align__(16) T smem[4 * kBufWords];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  T* buf = smem + wave * kBufWords;
  using K = KernelT<T, KERNEL>;

  int pk[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int k = lane + 64 * q;
    pk[q] = (k < d) ? cols[k] : 0;
  }
  const int64_t nchunks = (n + kChunk - 1) / kChunk;
  const int64_t ngroups = (n + 3) / 4;

  for (int64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
    const int64_t i = grp * 4 + wave;
    T xi[PD];
    PointLoad<T, PD>::get(pts + (i < n ? i : n - 1) * PD, xi);
    T acc[G][NQ];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int q = 0; q < NQ; ++q) acc[g][q] = 0;

    for (int64_t c = 0; c < nchunks; ++c) {
      const int64_t base = c * kChunk;
      const int last = (int)(n - base < kChunk ? n - base : kChunk);
      const T* cpts = pts + base * PD;
      T v[G][kChunkRegs];
#pragma unroll
      for (int r = 0; r < kChunkRegs; ++r) {
        if (r % kLoadGroup == 0) __builtin_amdgcn_sched_barrier(0);
        int jl = r * 64 + lane;
        jl = jl < last ? jl : last;
        T pj[PD];
        PointLoad<T, PD>::get(cpts + jl * PD, pj);
        const T sg = pj[PD - 1];
        T r2 = 0;
#pragma unroll
        for (int t = 0; t < ND; ++t) {
          const T df = xi[t] - pj[t];
          r2 = __builtin_fma(df, df, r2);
        }
#pragma unroll
        for (int g = 0; g < G; ++g) v[g][r] = sg * K::value(r2 * gp.a[g]);
      }
#pragma unroll
      for (int g = 0; g < G; ++g) srht_chunk_accumulate<T, NQ>(v[g], buf, lane, c, pk, d, acc[g]);
    }
    if (i >= n) continue;
    const T sgi = xi[PD - 1];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      T* out = Y + gp.yoff[g];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int k = lane + 64 * q;
        if (k < d) {
          T y = gp.so[g] * acc[g][q];
          if (nu_c != (T)0) {
            const unsigned par = __popcll((unsigned long long)i & (unsigned long long)pk[q]) & 1u;
            y += par ? -nu_c * sgi : nu_c * sgi;
          }
          out[i * d + k] = y;
        }
      }
    }
  }
}

template <typename T, int KERNEL, int PD, int ND, int NQ, int G>
static hipError_t launch_srht_grid_impl(hipStream_t st, const T* pts, const int32_t* cols, int64_t n, int d,
                                        const GridPass<T>& gp, double nu_c, T* Y, int num_cu) {
  auto kfn = sketch_srht_grid_kernel<T, KERNEL, PD, ND, NQ, G>;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kfn, 256, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  int64_t blocks = (n + 3) / 4;
  const int64_t cap = (int64_t)num_cu * per_cu;
  if (blocks > cap) blocks = cap;
  hipLaunchKernelGGL(kfn, dim3((unsigned)blocks), dim3(256), 0, st, pts, cols, n, d, gp, (T)nu_c, Y);
  return hipGetLastError();
}

template <typename T, int KERNEL, int PD, int ND, int G>
static hipError_t launch_srht_grid_nq(hipStream_t st, const T* pts, const int32_t* cols, int64_t n, int d,
                                      const GridPass<T>& gp, double nc, T* Y, int num_cu) {
  const int nq = (d + 63) / 64;
  if (nq <= 1) return launch_srht_grid_impl<T, KERNEL, PD, ND, 1, G>(st, pts, cols, n, d, gp, nc, Y, num_cu);
  if (nq <= 2) return launch_srht_grid_impl<T, KERNEL, PD, ND, 2, G>(st, pts, cols, n, d, gp, nc, Y, num_cu);
  if (nq <= 4) return launch_srht_grid_impl<T, KERNEL, PD, ND, 4, G>(st, pts, cols, n, d, gp, nc, Y, num_cu);
  if (nq <= 8) return launch_srht_grid_impl<T, KERNEL, PD, ND, 8, G>(st, pts, cols, n, d, gp, nc, Y, num_cu);
  return launch_srht_grid_impl<T, KERNEL, PD, ND, 16, G>(st, pts, cols, n, d, gp, nc, Y, num_cu);
}

template <typename T, int KERNEL, int G>
static hipError_t launch_srht_grid_dim(hipStream_t st, int D, const T* pts, const int32_t* cols, int64_t n, int d,
                                       const GridPass<T>& gp, double nc, T* Y, int num_cu) {
  switch (D) {
    case 1: return launch_srht_grid_nq<T, KERNEL, 4, 1, G>(st, pts, cols, n, d, gp, nc, Y, num_cu);
    case 2: return launch_srht_grid_nq<T, KERNEL, 4, 2, G>(st, pts, cols, n, d, gp, nc, Y, num_cu);
    case 3: return launch_srht_grid_nq<T, KERNEL, 4, 3, G>(st, pts, cols, n, d, gp, nc, Y, num_cu);
    default:
      if (D <= 7) return launch_srht_grid_nq<T, KERNEL, 8, 7, G>(st, pts, cols, n, d, gp, nc, Y, num_cu);
      return launch_srht_grid_nq<T, KERNEL, 16, 15, G>(st, pts, cols, n, d, gp, nc, Y, num_cu);
  }
}

template <typename T>
hipError_t launch_sketch_srht_grid(hipStream_t st, int kernel, int D, const T* pts, const int32_t* cols, int64_t n,
                                   int d, int ntheta, const double* dist_scale, const double* scale_out, double nu_c,
                                   T* Y, int num_cu) {
  for (int g0 = 0; g0 < ntheta; g0 += kGridPass) {
    const int gn = ntheta - g0 < kGridPass ? ntheta - g0 : kGridPass;
    GridPass<T> gp{};
    for (int g = 0; g < kGridPass; ++g) {
      const int gg = g0 + (g < gn ? g : 0);
      gp.a[g] = (T)dist_scale[gg];
      gp.so[g] = (T)scale_out[gg];
      gp.yoff[g] = (int64_t)gg * n * d;
    }
    hipError_t e;
    if (gn == kGridPass) {
      e = kernel == LR_KERNEL_SE
              ? launch_srht_grid_dim<T, LR_KERNEL_SE, kGridPass>(st, D, pts, cols, n, d, gp, nu_c, Y, num_cu)
              : launch_srht_grid_dim<T, LR_KERNEL_MATERN32, kGridPass>(st, D, pts, cols, n, d, gp, nu_c, Y, num_cu);
    } else {
      e = kernel == LR_KERNEL_SE
              ? launch_srht_grid_dim<T, LR_KERNEL_SE, 1>(st, D, pts, cols, n, d, gp, nu_c, Y, num_cu)
              : launch_srht_grid_dim<T, LR_KERNEL_MATERN32, 1>(st, D, pts, cols, n, d, gp, nu_c, Y, num_cu);
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
template hipError_t launch_sketch_srht_grid<float>(hipStream_t, int, int, const float*, const int32_t*, int64_t, int,
                                                   int, const double*, const double*, double, float*, int);
template hipError_t launch_sketch_srht_grid<double>(hipStream_t, int, int, const double*, const int32_t*, int64_t,
                                                    int, int, const double*, const double*, double, double*, int);

template <typename T, int KERNEL, int PD, int ND, int NQ, int MODE>
static hipError_t launch_srht_impl(hipStream_t st, const T* pts, const int32_t* cols, int64_t n, int d,
                                   double scale_out, double nu_c, T* Y, T* Yp, int num_cu) {
  // two rows per wave share the point loads (float, separate passes); the
  // fused mode keeps value and derivative of one row; double keeps one row
  constexpr int R = (sizeof(T) == 4 && MODE != 2) ? 2 : 1;
  auto kfn = sketch_srht_kernel<T, KERNEL, PD, ND, NQ, MODE, R>;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kfn, 256, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  int64_t blocks = (n + 4 * R - 1) / (4 * R);
  const int64_t cap = (int64_t)num_cu * per_cu;
  if (blocks > cap) blocks = cap;
  hipLaunchKernelGGL(kfn, dim3((unsigned)blocks), dim3(256), 0, st, pts, cols, n, d, (T)scale_out, (T)nu_c, Y, Yp);
  return hipGetLastError();
}

template <typename T, int KERNEL, int PD, int ND, int MODE>
static hipError_t launch_srht_nq(hipStream_t st, const T* pts, const int32_t* cols, int64_t n, int d,
                                 double so, double nc, T* Y, T* Yp, int num_cu) {
  const int nq = (d + 63) / 64;
  if (nq <= 1) return launch_srht_impl<T, KERNEL, PD, ND, 1, MODE>(st, pts, cols, n, d, so, nc, Y, Yp, num_cu);
  if (nq <= 2) return launch_srht_impl<T, KERNEL, PD, ND, 2, MODE>(st, pts, cols, n, d, so, nc, Y, Yp, num_cu);
  if (nq <= 4) return launch_srht_impl<T, KERNEL, PD, ND, 4, MODE>(st, pts, cols, n, d, so, nc, Y, Yp, num_cu);
  if (nq <= 8) return launch_srht_impl<T, KERNEL, PD, ND, 8, MODE>(st, pts, cols, n, d, so, nc, Y, Yp, num_cu);
  return launch_srht_impl<T, KERNEL, PD, ND, 16, MODE>(st, pts, cols, n, d, so, nc, Y, Yp, num_cu);
}

template <typename T, int KERNEL, int MODE>
static hipError_t launch_srht_dim(hipStream_t st, int D, const T* pts, const int32_t* cols, int64_t n, int d,
                                  double so, double nc, T* Y, T* Yp, int num_cu) {
  switch (D) {
    case 1: return launch_srht_nq<T, KERNEL, 4, 1, MODE>(st, pts, cols, n, d, so, nc, Y, Yp, num_cu);
    case 2: return launch_srht_nq<T, KERNEL, 4, 2, MODE>(st, pts, cols, n, d, so, nc, Y, Yp, num_cu);
    case 3: return launch_srht_nq<T, KERNEL, 4, 3, MODE>(st, pts, cols, n, d, so, nc, Y, Yp, num_cu);
    default:
      if (D <= 7) return launch_srht_nq<T, KERNEL, 8, 7, MODE>(st, pts, cols, n, d, so, nc, Y, Yp, num_cu);
      return launch_srht_nq<T, KERNEL, 16, 15, MODE>(st, pts, cols, n, d, so, nc, Y, Yp, num_cu);
  }
}

template <typename T, int MODE>
static hipError_t launch_srht_mode(hipStream_t st, int kernel, int D, const T* pts, const int32_t* cols,
                                   int64_t n, int d, double so, double nc, T* Y, T* Yp, int num_cu) {
  if (kernel == LR_KERNEL_SE)
    return launch_srht_dim<T, LR_KERNEL_SE, MODE>(st, D, pts, cols, n, d, so, nc, Y, Yp, num_cu);
  return launch_srht_dim<T, LR_KERNEL_MATERN32, MODE>(st, D, pts, cols, n, d, so, nc, Y, Yp, num_cu);
}

template <typename T>
hipError_t launch_sketch_srht(hipStream_t st, int kernel, int D, const T* pts, const int32_t* cols, int64_t n,
                              int d, double scale_out, double nu_c, T* Y, T* Yp, int num_cu) {
  if (Y != nullptr && Yp != nullptr) {
    if constexpr (sizeof(T) == 4) {
      return launch_srht_mode<T, 2>(st, kernel, D, pts, cols, n, d, scale_out, nu_c, Y, Yp, num_cu);
    } else {
      hipError_t e = launch_srht_mode<T, 0>(st, kernel, D, pts, cols, n, d, scale_out, nu_c, Y, Yp, num_cu);
      if (e != hipSuccess) return e;
      return launch_srht_mode<T, 1>(st, kernel, D, pts, cols, n, d, scale_out, nu_c, Y, Yp, num_cu);
    }
  }
  if (Y != nullptr) return launch_srht_mode<T, 0>(st, kernel, D, pts, cols, n, d, scale_out, nu_c, Y, Yp, num_cu);
  return launch_srht_mode<T, 1>(st, kernel, D, pts, cols, n, d, scale_out, nu_c, Y, Yp, num_cu);
}
template hipError_t launch_sketch_srht<float>(hipStream_t, int, int, const float*, const int32_t*, int64_t, int,
                                              double, double, float*, float*, int);
template hipError_t launch_sketch_srht<double>(hipStream_t, int, int, const double*, const int32_t*, int64_t,
                                               int, double, double, double*, double*, int);


// ------------------------------------------------------------------ Omega^T M
//
// Omega^T M for an SRHT Omega and a real n x N matrix M (F = Omega^T Q and the
// adjoint's Omega^T Y'): column c of M is transformed like a row of K in the
// sketch (chunks of 2048, the same butterflies and selections), which costs
// n (11 + 1) adds per column instead of the 2 n d of a dense product. One
// wave per column, float64 throughout: the products D_j M[j, c] are exact and
// every sum is a float64 sum. M arrives in slabs of S rows, transposed (mt: N
// rows of S entries); the sums go to outT (N x d, one contiguous row per
// column). pass: 0 = first slab (store), 1 = later slab (add).
template <typename T, int NQ>
__global__ __launch_bounds__(256) void srht_left_kernel(const T* __restrict__ mt, int64_t S, int64_t row0, int N,
                                                        const int8_t* __restrict__ signs,
                                                        const int32_t* __restrict__ cols, int d, int pass,
                                                        double* __restrict__ outT) {
  __shared__ __align__(16) double smem[4 * kBufWords];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int c = blockIdx.x * 4 + wave;
  if (c >= N) return;  // whole waves; the transform synchronises within the wave only
  double* buf = smem + wave * kBufWords;
  int pk[NQ];
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int k = lane + 64 * q;
    pk[q] = (k < d) ? cols[k] : 0;
    acc[q] = 0.0;
  }
  const T* col = mt + (int64_t)c * S;
  const int64_t nchunks = (S + kChunk - 1) / kChunk;
  for (int64_t ch = 0; ch < nchunks; ++ch) {
    const int64_t base = ch * kChunk;
    double v[kChunkRegs];
#pragma unroll
    for (int r = 0; r < kChunkRegs; ++r) {
      const int64_t j = base + r * 64 + lane;
      double x = 0.0;
      if (j < S) {
        x = (double)col[j];
        if (signs[row0 + j] < 0) x = -x;
      }
      v[r] = x;
    }
    // chunk index within the whole of n: row0 is a multiple of the chunk, or 0
    srht_chunk_accumulate<double, NQ>(v, buf, lane, (row0 + base) / kChunk, pk, d, acc);
  }
  double* o = outT + (int64_t)c * d;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int k = lane + 64 * q;
    if (k < d) o[k] = pass == 0 ? acc[q] : o[k] + acc[q];
  }
}

// out[k][c] = scale * outT[c][k] (d x N from N x d) through 32 x 32 LDS tiles.
__global__ void scale_transpose_kernel(const double* __restrict__ outT, int N, int d, double scale,
                                       double* __restrict__ out) {
  __shared__ double tile[32][33];
  const int c0 = blockIdx.x * 32, k0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int c = c0 + r, k = k0 + tx;
    tile[r][tx] = (c < N && k < d) ? outT[(int64_t)c * d + k] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int k = k0 + r, c = c0 + tx;
    if (k < d && c < N) out[(int64_t)k * N + c] = scale * tile[tx][r];
  }
}

template <typename T, int NQ>
static hipError_t launch_srht_left_nq(hipStream_t st, int64_t n, int d, const int8_t* signs, const int32_t* cols,
                                      const T* M, int N, double scale, double* out, void* ws, int64_t S) {
  double* outT = static_cast<double*>(ws);
  T* slab = reinterpret_cast<T*>(static_cast<char*>(ws) + (((size_t)N * d * sizeof(double) + 255) & ~(size_t)255));
  const dim3 grid((unsigned)((N + 3) / 4));
  for (int64_t row0 = 0; row0 < n; row0 += S) {
    hipError_t e = launch_transpose(st, S, N, M + row0 * N, S, slab, sizeof(T) == 8);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((srht_left_kernel<T, NQ>), grid, dim3(256), 0, st, slab, S, row0, N, signs, cols, d,
                       row0 == 0 ? 0 : 1, outT);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(scale_transpose_kernel, dim3((unsigned)((N + 31) / 32), (unsigned)((d + 31) / 32)), dim3(256),
                     0, st, outT, N, d, scale, out);
  return hipGetLastError();
}

int64_t srht_left_slab(int64_t n, int d, int N, size_t elem, size_t ws_bytes) {
  const size_t head = ((size_t)N * d * sizeof(double) + 255) & ~(size_t)255;
  if (d > 16 * 64 || N < 1 || ws_bytes <= head || (n & (n - 1)) != 0) return 0;
  int64_t S = n;
  while (S > kChunk && (size_t)S * N * elem > ws_bytes - head) S >>= 1;
  return (size_t)S * N * elem <= ws_bytes - head ? S : 0;
}

template <typename T>
hipError_t launch_srht_left(hipStream_t st, int64_t n, int d, const int8_t* signs, const int32_t* cols, const T* M,
                            int N, double scale, double* out, void* ws, int64_t S) {
  const int nq = (d + 63) / 64;
  if (nq <= 1) return launch_srht_left_nq<T, 1>(st, n, d, signs, cols, M, N, scale, out, ws, S);
  if (nq <= 2) return launch_srht_left_nq<T, 2>(st, n, d, signs, cols, M, N, scale, out, ws, S);
  if (nq <= 4) return launch_srht_left_nq<T, 4>(st, n, d, signs, cols, M, N, scale, out, ws, S);
  if (nq <= 8) return launch_srht_left_nq<T, 8>(st, n, d, signs, cols, M, N, scale, out, ws, S);
  return launch_srht_left_nq<T, 16>(st, n, d, signs, cols, M, N, scale, out, ws, S);
}
template hipError_t launch_srht_left<float>(hipStream_t, int64_t, int, const int8_t*, const int32_t*, const float*,
                                            int, double, double*, void*, int64_t);
template hipError_t launch_srht_left<double>(hipStream_t, int64_t, int, const int8_t*, const int32_t*, const double*,
                                             int, double, double*, void*, int64_t);

}  // namespace lr
