// Sketch Y = (K_f + nu I) Omega with K_f evaluated on the fly (Sec. 3.1-3.2).
//
// Two kernels:
//  * sketch_srht_kernel: Omega = c D H P (Def. 1, Walsh-Hadamard T). Row i of
//    Y is c (H (D o k_i))[P]. With H_n = H_{n/4096} (x) H_4096, each 4096-long
//    chunk j1 of D o k_i is transformed in full (12 butterfly stages: 6 over the
//    register index, an LDS transpose, 6 more), and every selected output
//    P_k = p1 * 4096 + p2 adds (-1)^popcount(j1 & p1) times entry p2 of the
//    chunk transform. One wave owns one row; lane l owns outputs l, l+64, ...
//    Work per row: n (12 + 1) butterflies/adds + d n / 4096 selections, against
//    the 2 n d of the dense product the structure avoids (Sec. 1, Sec. 3.2).
//  * sketch_dense_kernel: dense Omega (e.g. Gaussian, Sec. 3.1) on matrix
//    cores. A 512-thread workgroup owns 128 rows x BN columns of Y; per step of
//    32 columns j of K it evaluates the 128 x 32 kernel tile once (each thread
//    8 entries), stores it in LDS in MFMA operand order, and each of the 8 waves
//    multiplies all 8 row fragments against its own 16*WN columns of Omega
//    (loaded straight from the transposed, j-contiguous Omega). Accumulation
//    stays in registers for the whole sweep over j; K is never written out.
//    Workgroups are persistent and sweep j in the same order, so the Omega
//    slice for a step is shared in L2 by every workgroup on an XCD.
#include "common.hpp"
#include "kernels.hpp"

namespace lr {

// ------------------------------------------------------------------ prescale

template <typename T>
__global__ void prep_points_kernel(const float* __restrict__ X, int64_t n, int D, int PD, T scale,
                                   const int8_t* __restrict__ signs, T* __restrict__ out) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  for (int t = 0; t < PD - 1; ++t) out[j * PD + t] = (t < D) ? (T)X[j * D + t] * scale : (T)0;
  out[j * PD + PD - 1] = (signs != nullptr && signs[j] < 0) ? (T)-1 : (T)1;
}

template <typename T>
hipError_t launch_prep_points(hipStream_t st, const float* X, int64_t n, int D, int PD, double scale,
                              const int8_t* signs, T* out) {
  const int threads = 256;
  const int64_t blocks = (n + threads - 1) / threads;
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
template <typename T, int KERNEL, int PD, int NQ, int MODE>
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
          for (int t = 0; t < PD - 1; ++t) {
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

template <typename T, int KERNEL, int PD, int NQ, int MODE>
static hipError_t launch_srht_impl(hipStream_t st, const T* pts, const int32_t* cols, int64_t n, int d,
                                   double scale_out, double nu_c, T* Y, T* Yp, int num_cu) {
  const size_t lds = 4 * kChunkPad * sizeof(T);
  auto kfn = sketch_srht_kernel<T, KERNEL, PD, NQ, MODE>;
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

template <typename T, int KERNEL, int PD, int MODE>
static hipError_t launch_srht_nq(hipStream_t st, const T* pts, const int32_t* cols, int64_t n, int d,
                                 double so, double nc, T* Y, T* Yp, int num_cu) {
  const int nq = (d + 63) / 64;
  if (nq <= 1) return launch_srht_impl<T, KERNEL, PD, 1, MODE>(st, pts, cols, n, d, so, nc, Y, Yp, num_cu);
  if (nq <= 2) return launch_srht_impl<T, KERNEL, PD, 2, MODE>(st, pts, cols, n, d, so, nc, Y, Yp, num_cu);
  if (nq <= 4) return launch_srht_impl<T, KERNEL, PD, 4, MODE>(st, pts, cols, n, d, so, nc, Y, Yp, num_cu);
  if (nq <= 8) return launch_srht_impl<T, KERNEL, PD, 8, MODE>(st, pts, cols, n, d, so, nc, Y, Yp, num_cu);
  return launch_srht_impl<T, KERNEL, PD, 16, MODE>(st, pts, cols, n, d, so, nc, Y, Yp, num_cu);
}

template <typename T, int MODE>
static hipError_t launch_srht_mode(hipStream_t st, int kernel, int PD, const T* pts, const int32_t* cols,
                                   int64_t n, int d, double so, double nc, T* Y, T* Yp, int num_cu) {
  if (kernel == LR_KERNEL_SE) {
    if (PD == 4) return launch_srht_nq<T, LR_KERNEL_SE, 4, MODE>(st, pts, cols, n, d, so, nc, Y, Yp, num_cu);
    if (PD == 8) return launch_srht_nq<T, LR_KERNEL_SE, 8, MODE>(st, pts, cols, n, d, so, nc, Y, Yp, num_cu);
    return launch_srht_nq<T, LR_KERNEL_SE, 16, MODE>(st, pts, cols, n, d, so, nc, Y, Yp, num_cu);
  }
  if (PD == 4) return launch_srht_nq<T, LR_KERNEL_MATERN32, 4, MODE>(st, pts, cols, n, d, so, nc, Y, Yp, num_cu);
  if (PD == 8) return launch_srht_nq<T, LR_KERNEL_MATERN32, 8, MODE>(st, pts, cols, n, d, so, nc, Y, Yp, num_cu);
  return launch_srht_nq<T, LR_KERNEL_MATERN32, 16, MODE>(st, pts, cols, n, d, so, nc, Y, Yp, num_cu);
}

template <typename T>
hipError_t launch_sketch_srht(hipStream_t st, int kernel, int PD, const T* pts, const int32_t* cols, int64_t n,
                              int d, double scale_out, double nu_c, T* Y, T* Yp, int num_cu) {
  if (Y != nullptr && Yp != nullptr) {
    if constexpr (sizeof(T) == 4) {
      return launch_srht_mode<T, 2>(st, kernel, PD, pts, cols, n, d, scale_out, nu_c, Y, Yp, num_cu);
    } else {
      hipError_t e = launch_srht_mode<T, 0>(st, kernel, PD, pts, cols, n, d, scale_out, nu_c, Y, Yp, num_cu);
      if (e != hipSuccess) return e;
      return launch_srht_mode<T, 1>(st, kernel, PD, pts, cols, n, d, scale_out, nu_c, Y, Yp, num_cu);
    }
  }
  if (Y != nullptr) return launch_srht_mode<T, 0>(st, kernel, PD, pts, cols, n, d, scale_out, nu_c, Y, Yp, num_cu);
  return launch_srht_mode<T, 1>(st, kernel, PD, pts, cols, n, d, scale_out, nu_c, Y, Yp, num_cu);
}
template hipError_t launch_sketch_srht<float>(hipStream_t, int, int, const float*, const int32_t*, int64_t, int,
                                              double, double, float*, float*, int);
template hipError_t launch_sketch_srht<double>(hipStream_t, int, int, const double*, const int32_t*, int64_t,
                                               int, double, double, double*, double*, int);

// ------------------------------------------------------------------ dense Omega (matrix cores)

// Per precision: element type of Omega and of the LDS kernel tile, the
// accumulator fragment, and the largest column-fragment count per wave.
template <int PREC>
struct DenseCfg;
template <>
struct DenseCfg<LR_PREC_BF16> {
  using Real = float;
  using OmegaElem = uint16_t;
  using TileElem = __bf16;
  using Acc = f32x4_t;
  static constexpr int kMaxWN = 4;
};
template <>
struct DenseCfg<LR_PREC_F32> {
  using Real = float;
  using OmegaElem = float;
  using TileElem = float;
  using Acc = f32x4_t;
  static constexpr int kMaxWN = 4;
};
template <>
struct DenseCfg<LR_PREC_F64> {
  using Real = double;
  using OmegaElem = double;
  using TileElem = double;
  using Acc = f64x4_t;
  static constexpr int kMaxWN = 2;
};

// 8 consecutive Omega entries (j0 .. j0+7 of one column), zero beyond n.
template <int PREC>
struct OmegaFrag {
  using Cfg = DenseCfg<PREC>;
  typename Cfg::TileElem v[8];
};

template <int PREC>
__device__ __forceinline__ void load_omega8(const typename DenseCfg<PREC>::OmegaElem* __restrict__ p,
                                            int64_t j0, int64_t n, bool col_ok, OmegaFrag<PREC>& f) {
  using E = typename DenseCfg<PREC>::OmegaElem;
  using TE = typename DenseCfg<PREC>::TileElem;
  if (col_ok && j0 + 8 <= n) {
    if constexpr (PREC == LR_PREC_BF16) {
      uint4 raw = *reinterpret_cast<const uint4*>(p + j0);
      __builtin_memcpy(&f.v[0], &raw, 16);
    } else if constexpr (PREC == LR_PREC_F32) {
      float4 a = *reinterpret_cast<const float4*>(p + j0);
      float4 b = *reinterpret_cast<const float4*>(p + j0 + 4);
      f.v[0] = a.x; f.v[1] = a.y; f.v[2] = a.z; f.v[3] = a.w;
      f.v[4] = b.x; f.v[5] = b.y; f.v[6] = b.z; f.v[7] = b.w;
    } else {
#pragma unroll
      for (int e = 0; e < 8; e += 2) {
        double2 a = *reinterpret_cast<const double2*>(p + j0 + e);
        f.v[e] = a.x;
        f.v[e + 1] = a.y;
      }
    }
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      if (col_ok && j0 + e < n) {
        if constexpr (PREC == LR_PREC_BF16) {
          uint16_t bits = p[j0 + e];
          __builtin_memcpy(&f.v[e], &bits, 2);
        } else {
          f.v[e] = (TE)p[j0 + e];
        }
      } else {
        f.v[e] = (TE)0.0f;
      }
    }
  }
  (void)sizeof(E);
}

template <int PREC>
__device__ __forceinline__ void mfma_step(typename DenseCfg<PREC>::Acc& acc, const OmegaFrag<PREC>& a,
                                          const OmegaFrag<PREC>& b) {
  if constexpr (PREC == LR_PREC_BF16) {
    bf16x8_t av, bv;
    __builtin_memcpy(&av, &a.v[0], 16);
    __builtin_memcpy(&bv, &b.v[0], 16);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
  } else if constexpr (PREC == LR_PREC_F32) {
#pragma unroll
    for (int e = 0; e < 8; ++e) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[e], b.v[e], acc, 0, 0, 0);
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a.v[e], b.v[e], acc, 0, 0, 0);
  }
}

template <int PREC>
__device__ __forceinline__ typename DenseCfg<PREC>::OmegaElem omega_scalar_zero() {
  return 0;
}

template <int PREC>
__device__ __forceinline__ typename DenseCfg<PREC>::Real omega_value(
    const typename DenseCfg<PREC>::OmegaElem* __restrict__ omt, int64_t ld, int col, int64_t row) {
  if constexpr (PREC == LR_PREC_BF16) {
    uint32_t bits = (uint32_t)omt[(int64_t)col * ld + row] << 16;
    float f;
    __builtin_memcpy(&f, &bits, 4);
    return f;
  } else {
    return omt[(int64_t)col * ld + row];
  }
}

constexpr int kDenseRows = 128;  // rows of Y per workgroup
constexpr int kDenseStep = 32;   // columns of K per step

template <int PREC, int KERNEL, int PD, int WN, bool DERIV>
__global__ __launch_bounds__(512, 1) void sketch_dense_kernel(
    const typename DenseCfg<PREC>::Real* __restrict__ pts,
    const typename DenseCfg<PREC>::OmegaElem* __restrict__ omt, int64_t ld, int64_t n, int d,
    typename DenseCfg<PREC>::Real scale_out, typename DenseCfg<PREC>::Real nu,
    typename DenseCfg<PREC>::Real* __restrict__ Y, int nrb, int ncb) {
  using Cfg = DenseCfg<PREC>;
  using Real = typename Cfg::Real;
  using TE = typename Cfg::TileElem;
  using Acc = typename Cfg::Acc;
  using K = KernelT<Real, KERNEL>;
  constexpr int BN = 8 * 16 * WN;
  constexpr int kUnits = kDenseRows * 4;  // (row, k-group) units of 8 entries

  __shared__ __align__(16) TE tile[2][kUnits * 8];

  const int tid = threadIdx.x;
  const int w = tid >> 6;
  const int lane = tid & 63;
  const int grow = (w & 1) * 64 + lane;   // generation: row of the tile
  const int gg = wave_uniform(w >> 1);    // generation: k-group (wave-uniform)
  const int fl = lane & 15;               // fragment row/column
  const int fg = lane >> 4;               // fragment k-group
  const int64_t nsteps = (n + kDenseStep - 1) / kDenseStep;
  const int nblk = nrb * ncb;

  for (int blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int rb = blk % nrb;
    const int cb = blk / nrb;
    const int64_t row0 = (int64_t)rb * kDenseRows;
    const int colw = cb * BN + w * 16 * WN;  // first column owned by this wave

    Real xi[PD];
    {
      int64_t r = row0 + grow;
      if (r >= n) r = n - 1;
#pragma unroll
      for (int t = 0; t < PD; ++t) xi[t] = pts[r * PD + t];
    }

    Acc acc[8][WN];
#pragma unroll
    for (int f = 0; f < 8; ++f)
#pragma unroll
      for (int c = 0; c < WN; ++c)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[f][c][i] = 0;

    TE gen[8];
    auto generate = [&](int64_t step) {
      const int64_t j0 = step * kDenseStep + 8 * gg;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t j = j0 + e;
        Real val = 0;
        if (j < n) {
          Real r2 = 0;
#pragma unroll
          for (int t = 0; t < PD - 1; ++t) {
            const Real df = xi[t] - pts[j * PD + t];
            r2 += df * df;
          }
          val = DERIV ? K::deriv(r2) : K::value(r2);
        }
        gen[e] = (TE)val;
      }
    };
    auto store_gen = [&](int buf) {
      TE* dst = &tile[buf][(gg * kDenseRows + grow) * 8];
#pragma unroll
      for (int e = 0; e < 8; ++e) dst[e] = gen[e];
    };

    generate(0);
    store_gen(0);
    __syncthreads();

    const bool wave_active = colw < d;
    for (int64_t s = 0; s < nsteps; ++s) {
      const int cur = (int)(s & 1);
      OmegaFrag<PREC> b[WN];
      const int64_t jb = s * kDenseStep + 8 * fg;
#pragma unroll
      for (int c = 0; c < WN; ++c) {
        const int col = colw + 16 * c + fl;
        load_omega8<PREC>(omt + (int64_t)(col < d ? col : 0) * ld, jb, n, wave_active && col < d, b[c]);
      }
      if (s + 1 < nsteps) generate(s + 1);
      if (wave_active) {
#pragma unroll
        for (int f = 0; f < 8; ++f) {
          OmegaFrag<PREC> a;
          const TE* src = &tile[cur][(fg * kDenseRows + 16 * f + fl) * 8];
#pragma unroll
          for (int e = 0; e < 8; ++e) a.v[e] = src[e];
#pragma unroll
          for (int c = 0; c < WN; ++c) mfma_step<PREC>(acc[f][c], a, b[c]);
        }
      }
      if (s + 1 < nsteps) store_gen(cur ^ 1);
      __syncthreads();
    }

    if (wave_active) {
#pragma unroll
      for (int f = 0; f < 8; ++f) {
#pragma unroll
        for (int c = 0; c < WN; ++c) {
          const int col = colw + 16 * c + fl;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int64_t row = row0 + 16 * f + acc_row<Acc>(fg, i);
            if (row < n && col < d) {
              Real y = scale_out * (Real)acc[f][c][i];
              if (!DERIV && nu != (Real)0) y += nu * omega_value<PREC>(omt, ld, col, row);
              Y[row * d + col] = y;
            }
          }
        }
      }
    }
  }
}

template <int PREC, int KERNEL, int PD, int WN, bool DERIV>
static hipError_t launch_dense_impl(hipStream_t st, const void* pts, const void* omt, int64_t ld, int64_t n,
                                    int d, double scale_out, double nu, void* Y, int num_cu) {
  using Cfg = DenseCfg<PREC>;
  using Real = typename Cfg::Real;
  constexpr int BN = 8 * 16 * WN;
  const int nrb = (int)((n + kDenseRows - 1) / kDenseRows);
  const int ncb = (d + BN - 1) / BN;
  int64_t blocks = (int64_t)nrb * ncb;
  if (blocks > num_cu) blocks = num_cu;
  hipLaunchKernelGGL((sketch_dense_kernel<PREC, KERNEL, PD, WN, DERIV>), dim3((unsigned)blocks), dim3(512), 0, st,
                     (const Real*)pts, (const typename Cfg::OmegaElem*)omt, ld, n, d, (Real)scale_out, (Real)nu,
                     (Real*)Y, nrb, ncb);
  return hipGetLastError();
}

template <int PREC, int KERNEL, int PD, bool DERIV>
static hipError_t launch_dense_wn(hipStream_t st, const void* pts, const void* omt, int64_t ld, int64_t n, int d,
                                  double so, double nu, void* Y, int num_cu) {
  constexpr int maxwn = DenseCfg<PREC>::kMaxWN;
  if (d <= 128) return launch_dense_impl<PREC, KERNEL, PD, 1, DERIV>(st, pts, omt, ld, n, d, so, nu, Y, num_cu);
  if (d <= 256 || maxwn == 2)
    return launch_dense_impl<PREC, KERNEL, PD, 2, DERIV>(st, pts, omt, ld, n, d, so, nu, Y, num_cu);
  if constexpr (maxwn >= 4)
    return launch_dense_impl<PREC, KERNEL, PD, 4, DERIV>(st, pts, omt, ld, n, d, so, nu, Y, num_cu);
  return hipErrorInvalidValue;
}

template <int PREC, bool DERIV>
static hipError_t launch_dense_prec(hipStream_t st, int kernel, int PD, const void* pts, const void* omt,
                                   int64_t ld, int64_t n, int d, double so, double nu, void* Y, int num_cu) {
  if (kernel == LR_KERNEL_SE) {
    if (PD == 4) return launch_dense_wn<PREC, LR_KERNEL_SE, 4, DERIV>(st, pts, omt, ld, n, d, so, nu, Y, num_cu);
    if (PD == 8) return launch_dense_wn<PREC, LR_KERNEL_SE, 8, DERIV>(st, pts, omt, ld, n, d, so, nu, Y, num_cu);
    return launch_dense_wn<PREC, LR_KERNEL_SE, 16, DERIV>(st, pts, omt, ld, n, d, so, nu, Y, num_cu);
  }
  if (PD == 4) return launch_dense_wn<PREC, LR_KERNEL_MATERN32, 4, DERIV>(st, pts, omt, ld, n, d, so, nu, Y, num_cu);
  if (PD == 8) return launch_dense_wn<PREC, LR_KERNEL_MATERN32, 8, DERIV>(st, pts, omt, ld, n, d, so, nu, Y, num_cu);
  return launch_dense_wn<PREC, LR_KERNEL_MATERN32, 16, DERIV>(st, pts, omt, ld, n, d, so, nu, Y, num_cu);
}

hipError_t launch_sketch_dense(hipStream_t st, int prec, int kernel, int PD, const void* pts, const void* omt,
                               int64_t ld, int64_t n, int d, double scale_out, double nu, void* Y, bool deriv,
                               int num_cu) {
  if (prec == LR_PREC_BF16) {
    return deriv ? launch_dense_prec<LR_PREC_BF16, true>(st, kernel, PD, pts, omt, ld, n, d, scale_out, nu, Y, num_cu)
                 : launch_dense_prec<LR_PREC_BF16, false>(st, kernel, PD, pts, omt, ld, n, d, scale_out, nu, Y, num_cu);
  }
  if (prec == LR_PREC_F32) {
    return deriv ? launch_dense_prec<LR_PREC_F32, true>(st, kernel, PD, pts, omt, ld, n, d, scale_out, nu, Y, num_cu)
                 : launch_dense_prec<LR_PREC_F32, false>(st, kernel, PD, pts, omt, ld, n, d, scale_out, nu, Y, num_cu);
  }
  return deriv ? launch_dense_prec<LR_PREC_F64, true>(st, kernel, PD, pts, omt, ld, n, d, scale_out, nu, Y, num_cu)
               : launch_dense_prec<LR_PREC_F64, false>(st, kernel, PD, pts, omt, ld, n, d, scale_out, nu, Y, num_cu);
}

}  // namespace lr
