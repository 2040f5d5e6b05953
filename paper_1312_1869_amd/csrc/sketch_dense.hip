// Sketch Y = (K_f + nu I) Omega for a dense Omega (Sec. 3.1), on matrix cores.
//
// sketch_dense_kernel: dense Omega (e.g. Gaussian, Sec. 3.1) on matrix
//    cores. A 512-thread workgroup owns 128 rows x BN columns of Y; per step of
//    32 columns j of K it evaluates the 128 x 32 kernel tile once (each thread
//    8 entries), stores it in LDS in MFMA operand order, and each of the 8 waves
//    multiplies all 8 row fragments against its own 16*WN columns of Omega
//    (loaded straight from the transposed, j-contiguous Omega). Accumulation
//    stays in registers for the whole sweep over j; K is never written out.
//    Workgroups are persistent and sweep j in the same order, so the Omega
//    slice for a step is shared in L2 by every workgroup on an XCD.
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace lr {

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

template <int PREC, int KERNEL, int PD, int ND, int WN, bool DERIV>
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
    // Kernel values K[row0 + grow, j0 + e], j0 = step * 32 + 8 gg (FULL: j < n known).
    auto generate = [&](int64_t step, auto full_tag) {
      constexpr bool FULL = decltype(full_tag)::value;
      const int64_t j0 = step * kDenseStep + 8 * gg;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t j = j0 + e;
        Real val = 0;
        if (FULL || j < n) {
          Real r2 = 0;
#pragma unroll
          for (int t = 0; t < ND; ++t) {
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
    // Omega columns of this wave; columns >= d read column 0 and are zeroed.
    const typename Cfg::OmegaElem* ocol[WN];
    bool cok[WN];
#pragma unroll
    for (int c = 0; c < WN; ++c) {
      const int col = colw + 16 * c + fl;
      cok[c] = col < d;
      ocol[c] = omt + (int64_t)(cok[c] ? col : 0) * ld;
    }
    // One step: the 8 A fragments of step s come from LDS, the Omega fragments
    // of step s were loaded during the previous step (those of step s + 1 are
    // requested now), and the kernel tile of step s + 1 is evaluated on the
    // vector ALUs interleaved with the 8 x WN matrix-core products of step s.
    OmegaFrag<PREC> b[WN];
    auto load_b = [&](int64_t s, OmegaFrag<PREC> (&dst)[WN], auto full_tag) {
      constexpr bool FULL = decltype(full_tag)::value;
      const int64_t jb = s * kDenseStep + 8 * fg;
#pragma unroll
      for (int c = 0; c < WN; ++c) {
        if (FULL) {
          // columns >= d read column 0: their products land only in
          // accumulator columns that are never stored
          load_omega8<PREC>(ocol[c], jb, jb + 8, true, dst[c]);
        } else {
          load_omega8<PREC>(ocol[c], jb, n, cok[c], dst[c]);
        }
      }
    };
    auto step_body = [&](int64_t s, auto full_tag) {
      constexpr bool FULL = decltype(full_tag)::value;
      const int cur = (int)(s & 1);
      OmegaFrag<PREC> a[8];
#pragma unroll
      for (int f = 0; f < 8; ++f) {
        const TE* src = &tile[cur][(fg * kDenseRows + 16 * f + fl) * 8];
#pragma unroll
        for (int e = 0; e < 8; ++e) a[f].v[e] = src[e];
      }
      const bool has_next = FULL || s + 1 < nsteps;
      OmegaFrag<PREC> bn[WN];
      if (has_next) load_b(s + 1, bn, full_tag);
      if (has_next) generate(s + 1, full_tag);
#pragma unroll
      for (int f = 0; f < 8; ++f)
#pragma unroll
        for (int c = 0; c < WN; ++c) mfma_step<PREC>(acc[f][c], a[f], b[c]);
      if constexpr (PREC == LR_PREC_BF16 && FULL) {
        // interleave: one matrix-core op, then up to four vector ALU ops
#pragma unroll
        for (int i = 0; i < 8 * WN; ++i) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);
        }
      }
      if (has_next) store_gen(cur ^ 1);
#pragma unroll
      for (int c = 0; c < WN; ++c) b[c] = bn[c];
      __syncthreads();
    };

    generate(0, std::false_type{});
    store_gen(0);
    load_b(0, b, std::false_type{});
    __syncthreads();

    // steps s with s + 1 < nfull have both tiles s and s + 1 inside [0, n)
    const int64_t nfull = n / kDenseStep;
    int64_t s = 0;
    for (; s + 1 < nfull; ++s) step_body(s, std::true_type{});
    for (; s < nsteps; ++s) step_body(s, std::false_type{});

    const bool wave_active = colw < d;
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

template <int PREC, int KERNEL, int PD, int ND, int WN, bool DERIV>
static hipError_t launch_dense_impl(hipStream_t st, const void* pts, const void* omt, int64_t ld, int64_t n,
                                    int d, double scale_out, double nu, void* Y, int num_cu) {
  using Cfg = DenseCfg<PREC>;
  using Real = typename Cfg::Real;
  constexpr int BN = 8 * 16 * WN;
  const int nrb = (int)((n + kDenseRows - 1) / kDenseRows);
  const int ncb = (d + BN - 1) / BN;
  int64_t blocks = (int64_t)nrb * ncb;
  if (blocks > num_cu) blocks = num_cu;
  hipLaunchKernelGGL((sketch_dense_kernel<PREC, KERNEL, PD, ND, WN, DERIV>), dim3((unsigned)blocks), dim3(512), 0, st,
                     (const Real*)pts, (const typename Cfg::OmegaElem*)omt, ld, n, d, (Real)scale_out, (Real)nu,
                     (Real*)Y, nrb, ncb);
  return hipGetLastError();
}

template <int PREC, int KERNEL, int PD, int ND, bool DERIV>
static hipError_t launch_dense_wn(hipStream_t st, const void* pts, const void* omt, int64_t ld, int64_t n, int d,
                                  double so, double nu, void* Y, int num_cu) {
  constexpr int maxwn = DenseCfg<PREC>::kMaxWN;
  if (d <= 128) return launch_dense_impl<PREC, KERNEL, PD, ND, 1, DERIV>(st, pts, omt, ld, n, d, so, nu, Y, num_cu);
  if (d <= 256 || maxwn == 2)
    return launch_dense_impl<PREC, KERNEL, PD, ND, 2, DERIV>(st, pts, omt, ld, n, d, so, nu, Y, num_cu);
  if constexpr (maxwn >= 4)
    return launch_dense_impl<PREC, KERNEL, PD, ND, 4, DERIV>(st, pts, omt, ld, n, d, so, nu, Y, num_cu);
  return hipErrorInvalidValue;
}

// Coordinates used: D itself for D <= 3 (stride 4), else every slot but the sign.
template <int PREC, int KERNEL, bool DERIV>
static hipError_t launch_dense_dim(hipStream_t st, int D, const void* pts, const void* omt, int64_t ld, int64_t n,
                                   int d, double so, double nu, void* Y, int num_cu) {
  switch (D) {
    case 1: return launch_dense_wn<PREC, KERNEL, 4, 1, DERIV>(st, pts, omt, ld, n, d, so, nu, Y, num_cu);
    case 2: return launch_dense_wn<PREC, KERNEL, 4, 2, DERIV>(st, pts, omt, ld, n, d, so, nu, Y, num_cu);
    case 3: return launch_dense_wn<PREC, KERNEL, 4, 3, DERIV>(st, pts, omt, ld, n, d, so, nu, Y, num_cu);
    default:
      if (D <= 7) return launch_dense_wn<PREC, KERNEL, 8, 7, DERIV>(st, pts, omt, ld, n, d, so, nu, Y, num_cu);
      return launch_dense_wn<PREC, KERNEL, 16, 15, DERIV>(st, pts, omt, ld, n, d, so, nu, Y, num_cu);
  }
}

template <int PREC, bool DERIV>
static hipError_t launch_dense_prec(hipStream_t st, int kernel, int D, const void* pts, const void* omt,
                                   int64_t ld, int64_t n, int d, double so, double nu, void* Y, int num_cu) {
  if (kernel == LR_KERNEL_SE)
    return launch_dense_dim<PREC, LR_KERNEL_SE, DERIV>(st, D, pts, omt, ld, n, d, so, nu, Y, num_cu);
  return launch_dense_dim<PREC, LR_KERNEL_MATERN32, DERIV>(st, D, pts, omt, ld, n, d, so, nu, Y, num_cu);
}

hipError_t launch_sketch_dense(hipStream_t st, int prec, int kernel, int D, const void* pts, const void* omt,
                               int64_t ld, int64_t n, int d, double scale_out, double nu, void* Y, bool deriv,
                               int num_cu) {
  if (prec == LR_PREC_BF16) {
    return deriv ? launch_dense_prec<LR_PREC_BF16, true>(st, kernel, D, pts, omt, ld, n, d, scale_out, nu, Y, num_cu)
                 : launch_dense_prec<LR_PREC_BF16, false>(st, kernel, D, pts, omt, ld, n, d, scale_out, nu, Y, num_cu);
  }
  if (prec == LR_PREC_F32) {
    return deriv ? launch_dense_prec<LR_PREC_F32, true>(st, kernel, D, pts, omt, ld, n, d, scale_out, nu, Y, num_cu)
                 : launch_dense_prec<LR_PREC_F32, false>(st, kernel, D, pts, omt, ld, n, d, scale_out, nu, Y, num_cu);
  }
  return deriv ? launch_dense_prec<LR_PREC_F64, true>(st, kernel, D, pts, omt, ld, n, d, scale_out, nu, Y, num_cu)
               : launch_dense_prec<LR_PREC_F64, false>(st, kernel, D, pts, omt, ld, n, d, scale_out, nu, Y, num_cu);
}

}  // namespace lr
