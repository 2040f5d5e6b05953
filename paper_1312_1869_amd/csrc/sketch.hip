// Sketch Y = (K_f + nu I) Omega with K_f evaluated on the fly (Sec. 3.1-3.2).
//
// This file: the points prescale and the SRHT kernel (sketch_dense.hip holds the
// dense-Omega kernel).
//  * sketch_srht_kernel: Omega = c D H P (Def. 1, Walsh-Hadamard T). Row i of
//    Y is c (H (D o k_i))[P]. With H_n = H_{n/4096} (x) H_4096, each 4096-long
//    chunk j1 of D o k_i is transformed in full (12 butterfly stages: 6 over the
//    register index, an LDS transpose, 6 more), and every selected output
//    P_k = p1 * 4096 + p2 adds (-1)^popcount(j1 & p1) times entry p2 of the
//    chunk transform. One wave owns one row; lane l owns outputs l, l+64, ...
//    Work per row: n (12 + 1) butterflies/adds + d n / 4096 selections, against
//    the 2 n d of the dense product the structure avoids (Sec. 1, Sec. 3.2).
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

constexpr int kChunk = 4096;
constexpr int kChunkPad = kChunk + kChunk / 64;
__device__ __forceinline__ int padidx(int i) { return i + (i >> 6); }

template <typename T>
__device__ __forceinline__ void fwht64(T (&v)[64]) {
#pragma unroll
  for (int h = 1; h < 64; h <<= 1) {
#pragma unroll
    for (int i = 0; i < 64; ++i) {
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

// One chunk of values v (register r of lane l = chunk entry r*64 + l) is
// transformed and its selected entries accumulated into acc.
template <typename T, int NQ>
__device__ __forceinline__ void srht_chunk_accumulate(T (&v)[64], T* buf, int lane, int64_t chunk,
                                                      const int (&pk)[NQ], int d, T (&acc)[NQ]) {
  fwht64(v);  // stages over entry bits 6..11 (register index)
#pragma unroll
  for (int r = 0; r < 64; ++r) buf[r * 65 + lane] = v[r];
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int r = 0; r < 64; ++r) v[r] = buf[lane * 65 + r];
  fwht64(v);  // stages over entry bits 0..5
#pragma unroll
  for (int r = 0; r < 64; ++r) buf[lane * 65 + r] = v[r];
  __builtin_amdgcn_wave_barrier();
  const unsigned hi = (unsigned)chunk;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int k = lane + 64 * q;
    if (k < d) {
      const int p = pk[q];
      T val = buf[padidx(p & (kChunk - 1))];
      const unsigned par = __popc(hi & (unsigned)(p >> 12)) & 1u;
      acc[q] += par ? -val : val;
    }
  }
  __builtin_amdgcn_wave_barrier();
}

// MODE: 0 = Y only, 1 = Yprime only, 2 = both (fused, one kernel evaluation).
template <typename T, int KERNEL, int PD, int ND, int NQ, int MODE>
__global__ __launch_bounds__(256) void sketch_srht_kernel(const T* __restrict__ pts,
                                                          const int32_t* __restrict__ cols, int64_t n,
                                                          int d, T scale_out, T nu_c,
                                                          T* __restrict__ Y, T* __restrict__ Yp) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  T* buf = reinterpret_cast<T*>(smem_raw) + wave * kChunkPad;
  using K = KernelT<T, KERNEL>;

  int pk[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int k = lane + 64 * q;
    pk[q] = (k < d) ? cols[k] : 0;
  }
  const int64_t nchunks = (n + kChunk - 1) / kChunk;
  const int64_t stride = (int64_t)gridDim.x * 4;

  for (int64_t i = (int64_t)blockIdx.x * 4 + wave; i < n; i += stride) {
    T xi[PD];
    PointLoad<T, PD>::get(pts + i * PD, xi);
    T acc[NQ], accd[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) { acc[q] = 0; accd[q] = 0; }

    for (int64_t c = 0; c < nchunks; ++c) {
      const int64_t base = c * kChunk;
      const bool full = base + kChunk <= n;
      T v[64];
      T vd[MODE == 2 ? 64 : 1];
#pragma unroll
      for (int r = 0; r < 64; ++r) {
        const int64_t j = base + r * 64 + lane;
        T val = 0, dval = 0;
        if (full || j < n) {
          T pj[PD];
          PointLoad<T, PD>::get(pts + j * PD, pj);
          T r2 = 0;
#pragma unroll
          for (int t = 0; t < ND; ++t) {
            const T df = xi[t] - pj[t];
            r2 += df * df;
          }
          const T sg = pj[PD - 1];
          if constexpr (MODE == 0) {
            val = sg * K::value(r2);
          } else if constexpr (MODE == 1) {
            val = sg * K::deriv(r2);
          } else {
            K::both(r2, val, dval);
            val *= sg;
            dval *= sg;
          }
        }
        v[r] = val;
        if constexpr (MODE == 2) vd[r] = dval;
      }
      srht_chunk_accumulate<T, NQ>(v, buf, lane, c, pk, d, acc);
      if constexpr (MODE == 2) srht_chunk_accumulate<T, NQ>(vd, buf, lane, c, pk, d, accd);
    }

    const T sgi = xi[PD - 1];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int k = lane + 64 * q;
      if (k < d) {
        if constexpr (MODE != 1) {
          T y = scale_out * acc[q];
          if (nu_c != (T)0) {
            const unsigned par = __popcll((unsigned long long)i & (unsigned long long)pk[q]) & 1u;
            y += par ? -nu_c * sgi : nu_c * sgi;
          }
          Y[i * d + k] = y;
        }
        if constexpr (MODE == 1) Yp[i * d + k] = scale_out * acc[q];
        if constexpr (MODE == 2) Yp[i * d + k] = scale_out * accd[q];
      }
    }
  }
}

template <typename T, int KERNEL, int PD, int ND, int NQ, int MODE>
static hipError_t launch_srht_impl(hipStream_t st, const T* pts, const int32_t* cols, int64_t n, int d,
                                   double scale_out, double nu_c, T* Y, T* Yp, int num_cu) {
  const size_t lds = 4 * kChunkPad * sizeof(T);
  auto kfn = sketch_srht_kernel<T, KERNEL, PD, ND, NQ, MODE>;
  hipError_t e = hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int per_cu = sizeof(T) == 4 ? 2 : 1;
  int64_t blocks = (n + 3) / 4;
  const int64_t cap = (int64_t)num_cu * per_cu;
  if (blocks > cap) blocks = cap;
  hipLaunchKernelGGL(kfn, dim3((unsigned)blocks), dim3(256), lds, st, pts, cols, n, d, (T)scale_out, (T)nu_c,
                     Y, Yp);
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

}  // namespace lr
