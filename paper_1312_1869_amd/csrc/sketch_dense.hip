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

    // Points x_j of the 8 columns of K a wave evaluates in a step (wave
    // uniform, so they live in scalar registers). Indices past n are clamped;
    // those kernel values are masked in the ragged tail.
    using PtsStep = Real[8][ND];
    auto load_pts = [&](int64_t step, PtsStep& xj) {
      const int64_t j0 = step * kDenseStep + 8 * gg;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t j = (j0 + e < n) ? j0 + e : n - 1;
#pragma unroll
        for (int t = 0; t < ND; ++t) xj[e][t] = pts[j * PD + t];
      }
    };
    TE gen[8];
    // Kernel values K[row0 + grow, j0 + e], j0 = step * 32 + 8 gg (FULL: j < n known).
    auto generate = [&](int64_t step, const PtsStep& xj, auto full_tag) {
      constexpr bool FULL = decltype(full_tag)::value;
      const int64_t j0 = step * kDenseStep + 8 * gg;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        Real val = 0;
        if (FULL || j0 + e < n) {
          Real r2 = 0;
#pragma unroll
          for (int t = 0; t < ND; ++t) {
            const Real df = xi[t] - xj[e][t];
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
    // Omega columns of this wave: a wave-uniform base (column colw) and 32-bit
    // per-lane element offsets of the WN fragments' columns. Columns >= d read
    // column 0 and only feed accumulator columns that are never stored.
    const typename Cfg::OmegaElem* obase = omt + (int64_t)(colw < d ? colw : 0) * ld;
    uint32_t coff[WN];
    bool cok[WN];
#pragma unroll
    for (int c = 0; c < WN; ++c) {
      const int col = colw + 16 * c + fl;
      cok[c] = col < d;
      coff[c] = cok[c] ? (uint32_t)((int64_t)(16 * c + fl) * ld) : 0u;
    }
    auto load_b = [&](int64_t s, OmegaFrag<PREC> (&dst)[WN], auto full_tag) {
      constexpr bool FULL = decltype(full_tag)::value;
      const int64_t jb = s * kDenseStep + 8 * fg;
#pragma unroll
      for (int c = 0; c < WN; ++c) {
        if (FULL) {
          load_omega8<PREC>(obase + coff[c], jb, jb + 8, true, dst[c]);
        } else {
          load_omega8<PREC>(obase + coff[c], jb, n, cok[c], dst[c]);
        }
      }
    };
    // One step s: the 8 A fragments come from LDS tile s, the Omega fragments
    // b were requested during step s - 1 (those of step s + 1 go to bn now),
    // the points of step s + 1 were loaded during step s - 1 (those of step
    // s + 2 go to xjn now), and the kernel tile of step s + 1 is evaluated on
    // the vector ALUs interleaved with the 8 x WN matrix-core products.
    auto step_body = [&](int64_t s, OmegaFrag<PREC> (&b)[WN], OmegaFrag<PREC> (&bn)[WN], const PtsStep& xj,
                         PtsStep& xjn, auto full_tag) {
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
      if (has_next) {
        load_b(s + 1, bn, full_tag);
        generate(s + 1, xj, full_tag);
      }
#pragma unroll
      for (int f = 0; f < 8; ++f)
#pragma unroll
        for (int c = 0; c < WN; ++c) mfma_step<PREC>(acc[f][c], a[f], b[c]);
      if constexpr (PREC == LR_PREC_BF16 && FULL) {
        // interleave: one matrix-core op, then up to two vector ALU ops
#pragma unroll
        for (int i = 0; i < 8 * WN; ++i) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);
        }
      }
      if (has_next) store_gen(cur ^ 1);
      __syncthreads();
      // requested after the barrier's wait, so the step's LDS waits do not
      // also wait for these scalar loads
      if (s + 2 < nsteps) load_pts(s + 2, xjn);
    };

    OmegaFrag<PREC> bA[WN], bB[WN];
    PtsStep xA, xB;
    load_pts(0, xA);
    generate(0, xA, std::false_type{});
    store_gen(0);
    load_b(0, bA, std::false_type{});
    if (nsteps > 1) load_pts(1, xA);
    __syncthreads();

    // Steps in pairs with the operand registers alternating roles. A step s
    // runs FULL when the tile it evaluates (s + 1) lies inside [0, n).
    const int64_t nfull = n / kDenseStep;
    int64_t s = 0;
    for (; s + 2 < nfull; s += 2) {
      step_body(s, bA, bB, xA, xB, std::true_type{});
      step_body(s + 1, bB, bA, xB, xA, std::true_type{});
    }
    for (; s < nsteps; s += 2) {
      step_body(s, bA, bB, xA, xB, std::false_type{});
      if (s + 1 < nsteps) step_body(s + 1, bB, bA, xB, xA, std::false_type{});
    }

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

// ------------------------------------------------------------------ bf16 on matrix cores
//
// Omega is first copied into matrix-core operand order (omega_frag_kernel):
// for every 16-column group c16 and step s of 32 rows j, one 1 KB fragment
// whose lane l = fl + 16 fg holds Omega[32 s + 8 fg .. + 7][16 c16 + fl] as 8
// bf16. Rows j >= n and columns >= the padded width are zero, so the sketch
// kernel reads every operand with one contiguous, unmasked 16-byte load per
// lane and needs no ragged-tail handling (kernel values at j >= n meet zero
// Omega rows).
//
// sketch_bf16_kernel: NW waves (NW * 64 threads, 8 waves = 2 per SIMD) own 128
// rows x NW*16*WC columns of Y; each wave keeps the accumulators of the 128
// rows x its 16*WC columns. Per step of 32 columns j of K:
//   * every thread evaluates GPT = 64/NW kernel entries (one row, GPT
//     consecutive j); its x_i is in registers, and x_j comes from one vector
//     load per step (lane fl of each 16-lane row holds point fl mod GPT) read
//     back with a DPP row broadcast;
//   * the entries are rounded to bf16 and written to a double-buffered LDS
//     tile in operand order; each wave reads the 8 row fragments of the tile
//     and multiplies them with its WC Omega fragments (8 x WC products);
//   * the Omega fragments of step s + 2 (three rotating register sets) and
//     the points of step s + 3 (three rotating sets) are requested at the
//     start of step s.

#ifndef LR_B16_WAVES
#define LR_B16_WAVES 8
#endif
constexpr int kB16Waves = LR_B16_WAVES;

__global__ void omega_frag_kernel(const uint16_t* __restrict__ omt, int64_t ld, int64_t n, int d, int64_t nst,
                                  int64_t total, uint4* __restrict__ frag) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;  // (c16 * nst + s) * 64 + lane
  if (q >= total) return;
  const int lane = (int)(q & 63);
  const int64_t fs = q >> 6;
  const int64_t c16 = fs / nst;
  const int64_t step = fs - c16 * nst;
  const int64_t col = c16 * 16 + (lane & 15);
  const int64_t j0 = step * kDenseStep + 8 * (lane >> 4);
  uint4 v = {0u, 0u, 0u, 0u};
  if (col < d && j0 < n) {
    const uint16_t* src = omt + col * ld + j0;
    if (j0 + 8 <= n) {
      v = *reinterpret_cast<const uint4*>(src);  // j0 and ld are multiples of 8
    } else {
      uint16_t t[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) t[e] = (j0 + e < n) ? src[e] : (uint16_t)0;
      __builtin_memcpy(&v, t, 16);
    }
  }
  frag[q] = v;
}

// steps by which the bf16 sketch fetches its Omega fragments ahead
#ifndef LR_B16_AHEAD
#define LR_B16_AHEAD 2
#endif
constexpr int kB16Ahead = LR_B16_AHEAD;
// interleave the kernel evaluation with the matrix-core operations
#ifndef LR_B16_INTERLEAVE
#define LR_B16_INTERLEAVE 1
#endif
constexpr bool kB16Interleave = LR_B16_INTERLEAVE != 0;

// largest n of the bf16 matrix-core sketch (31-bit buffer extents)
constexpr int64_t kBf16MaxRows = int64_t(1) << 25;

// A raw buffer view of global memory: reads beyond `bytes` return zero.
// The base is wave-uniform, so the view lives in scalar registers and each
// load takes a 32-bit lane offset plus a scalar offset.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_view(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

template <int E>
__device__ __forceinline__ float row_bcast(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x150 + E, 0xF, 0xF,
                                                               false));
}

template <int NW, int KERNEL, int PD, int ND, int WC, bool DERIV, bool X2>
__global__ __launch_bounds__(NW * 64, 1) void sketch_bf16_kernel(const float* __restrict__ pts,
                                                                 const uint4* __restrict__ frag, int64_t nst,
                                                                 const uint16_t* __restrict__ omt, int64_t ld,
                                                                 int64_t n, int d, float scale_out, float nu,
                                                                 float* __restrict__ Y, int nrb, int ncb) {
  using K = KernelT<float, KERNEL>;
  using Frag = OmegaFrag<LR_PREC_BF16>;
  constexpr int BN = NW * 16 * WC;
  constexpr int GPT = 64 / NW;  // kernel entries per thread per step (8 or 16)
  // X2: every entry k is split into k_hi = bf16(k) and k_lo = bf16(k - k_hi),
  // two tiles and two products per fragment (NFR fragment reads per step)
  constexpr int NFR = X2 ? 16 : 8;
  constexpr int NMF = NFR * WC;
  constexpr int kTileHalf = 4 * kDenseRows * 8;
#ifdef LR_B16_VALU_PER_MFMA
  constexpr int kValuPerMfma = LR_B16_VALU_PER_MFMA;
#else
  constexpr int kValuPerMfma = X2 ? ((11 * GPT / (16 * WC)) > 1 ? (11 * GPT / (16 * WC)) : 1)
                                  : ((9 * GPT / (8 * WC)) > 2 ? (9 * GPT / (8 * WC)) : 2);
#endif
  static_assert(NW == 4 || NW == 8, "4 or 8 waves");

  __shared__ __align__(16) __bf16 tile[2][(X2 ? 2 : 1) * kTileHalf];  // [buf][hi/lo][k-group][row][8]

  const int tid = threadIdx.x;
  const int w = wave_uniform(tid >> 6);
  const int lane = tid & 63;
  const int grow = (w & 1) * 64 + lane;  // generation: row of the tile
  const int gg = wave_uniform(w >> 1);   // generation: j = GPT gg .. GPT gg + GPT - 1 of the step
  const int fl = lane & 15;
  const int fg = lane >> 4;
  const int nblk = nrb * ncb;

  for (int blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int rb = blk % nrb;
    const int cb = blk / nrb;
    const int64_t row0 = (int64_t)rb * kDenseRows;
    const int colw = cb * BN + w * 16 * WC;

    float xi[ND];
    {
      int64_t r = row0 + grow;
      if (r >= n) r = n - 1;
#pragma unroll
      for (int t = 0; t < ND; ++t) xi[t] = pts[r * PD + t];
    }

    f32x4_t acc[8][WC];
#pragma unroll
    for (int f = 0; f < 8; ++f)
#pragma unroll
      for (int c = 0; c < WC; ++c)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[f][c][i] = 0.0f;

    // x_j of j = 32 step + GPT gg + (fl mod GPT); the point array has
    // kPointPad zero rows past n (steps up to nst + 2 are read), and kernel
    // values there meet zero Omega rows
    using Pts = float[ND];
    const __amdgpu_buffer_rsrc_t pview = buffer_view(pts, (uint32_t)((n + kPointPad) * PD * sizeof(float)));
    const uint32_t poff = (uint32_t)((GPT * gg + (fl & (GPT - 1))) * PD * sizeof(float));
    auto load_pts = [&](int64_t step, Pts& p) {
      const int soff = (int)(step * (kDenseStep * PD * sizeof(float)));
      // (the builtins return plain vector_size vectors: copy them out bytewise)
      if constexpr (ND == 1) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b32(pview, poff, soff, 0);
        static_assert(sizeof(v) >= 4, "load width");
        __builtin_memcpy(&p[0], &v, 4);
      } else if constexpr (ND == 2) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(pview, poff, soff, 0);
        static_assert(sizeof(v) >= 8, "load width");
        __builtin_memcpy(&p[0], &v, 8);
      } else {
        const auto v = __builtin_amdgcn_raw_buffer_load_b96(pview, poff, soff, 0);
        static_assert(sizeof(v) >= 12, "load width");
        __builtin_memcpy(&p[0], &v, 12);
      }
    };
    __bf16 gen[GPT];
    __bf16 genlo[X2 ? GPT : 1];
    auto generate = [&](const Pts& p) {
      static_for<0, GPT>([&](auto ee) {
        constexpr int e = decltype(ee)::value;
        float r2 = 0.0f;
#pragma unroll
        for (int t = 0; t < ND; ++t) {
          const float df = row_bcast<e>(p[t]) - xi[t];
          r2 = __builtin_fmaf(df, df, r2);
        }
        const float kv = DERIV ? K::deriv(r2) : K::value(r2);
        gen[e] = (__bf16)kv;
        if constexpr (X2) genlo[e] = (__bf16)(kv - (float)gen[e]);
      });
    };
    auto store_gen = [&](int buf) {
#pragma unroll
      for (int u = 0; u < GPT / 8; ++u) {
        __bf16* dst = &tile[buf][((GPT / 8 * gg + u) * kDenseRows + grow) * 8];
#pragma unroll
        for (int e = 0; e < 8; ++e) dst[e] = gen[8 * u + e];
        if constexpr (X2) {
#pragma unroll
          for (int e = 0; e < 8; ++e) dst[kTileHalf + e] = genlo[8 * u + e];
        }
      }
    };
    // this wave's fragments: one buffer view per 16-column group (nst steps
    // of 1 KB; the prefetch past the last step reads zeros), lane offset
    // 16 lane bytes
    __amdgpu_buffer_rsrc_t fview[WC];
#pragma unroll
    for (int c = 0; c < WC; ++c)
      fview[c] = buffer_view(frag + (int64_t)(colw / 16 + c) * nst * 64, (uint32_t)(nst * 64 * sizeof(uint4)));
    const uint32_t foff = (uint32_t)lane * sizeof(uint4);
    auto load_b = [&](int64_t s, Frag (&dst)[WC]) {
      const int soff = (int)(s * (64 * sizeof(uint4)));
#pragma unroll
      for (int c = 0; c < WC; ++c) {
        const auto raw = __builtin_amdgcn_raw_buffer_load_b128(fview[c], foff, soff, 0);
        static_assert(sizeof(raw) == 16, "load width");
        __builtin_memcpy(&dst[c].v[0], &raw, 16);
      }
    };
    // Step s: b holds Omega of step s, bl receives Omega of step
    // s + kB16Ahead, pg holds the points of step s + 1, pl receives those of
    // step s + 3. The
    // loads, the evaluation and the tile store are unconditional (the last
    // steps read the zero padding past the data and their tiles are never
    // used), so no branch hides from the compiler how many loads are in flight.
    auto step_body = [&](int64_t s, Frag (&b)[WC], Frag (&bl)[WC], const Pts& pg, Pts& pl) {
      const int cur = (int)(s & 1);
      load_b(s + kB16Ahead, bl);
      load_pts(s + 3, pl);
      Frag a[NFR];
#pragma unroll
      for (int f = 0; f < NFR; ++f) {
        const __bf16* src = &tile[cur][(f / 8) * kTileHalf + (fg * kDenseRows + 16 * (f % 8) + fl) * 8];
#pragma unroll
        for (int e = 0; e < 8; ++e) a[f].v[e] = src[e];
      }
      generate(pg);
#pragma unroll
      for (int f = 0; f < NFR; ++f)
#pragma unroll
        for (int c = 0; c < WC; ++c) mfma_step<LR_PREC_BF16>(acc[f % 8][c], a[f], b[c]);
      store_gen(cur ^ 1);
      // issue order: the tile reads and operand loads, then every
      // matrix-core operation followed by a few vector instructions of the
      // evaluation, so the vector work runs while the matrix cores are busy
      if constexpr (kB16Interleave) {
        __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
        __builtin_amdgcn_sched_group_barrier(0x020, WC + 1, 0);
        static_for<0, NMF>([&](auto ii) {
          constexpr int i = decltype(ii)::value;
          if constexpr (i % WC == 0 && i / WC < NFR - 2) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x002, kValuPerMfma, 0);
        });
        __builtin_amdgcn_sched_group_barrier(0x200, (X2 ? 2 : 1) * GPT / 8, 0);
      }
      __syncthreads();
      // keep each step's instructions inside the step, so loads issued at its
      // start are not sunk towards their uses one or two steps later
      __builtin_amdgcn_sched_barrier(0);
    };

    // Omega in kB16Ahead + 1 rotating register sets, points in 3 rotating
    // sets (two steps ahead): six steps per loop trip.
    constexpr int NB = kB16Ahead + 1;
    static_assert(6 % NB == 0, "register sets rotate within a loop trip");
    Frag bs[NB][WC];
    Pts ps[3];
    // prologue: the loads in the order the steps issue them ([Omega, points]
    // per step), so the waits of the first loop step match the later ones
    load_pts(0, ps[0]);
    constexpr int kPro = kB16Ahead > 2 ? kB16Ahead : 2;
    static_for<0, kPro>([&](auto kk) {
      constexpr int k = decltype(kk)::value;
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (k < kB16Ahead) load_b(k, bs[k]);
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (k < 2) load_pts(k + 1, ps[k + 1]);
    });
    __builtin_amdgcn_sched_barrier(0);
    generate(ps[0]);
    store_gen(0);
    __syncthreads();

    int64_t s = 0;
    for (; s + 6 <= nst; s += 6) {
      static_for<0, 6>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        step_body(s + k, bs[k % NB], bs[(k + kB16Ahead) % NB], ps[(k + 1) % 3], ps[k % 3]);
      });
    }
    static_for<0, 5>([&](auto kk) {
      constexpr int k = decltype(kk)::value;
      if (s + k < nst) step_body(s + k, bs[k % NB], bs[(k + kB16Ahead) % NB], ps[(k + 1) % 3], ps[k % 3]);
    });

#pragma unroll
    for (int f = 0; f < 8; ++f) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t row = row0 + 16 * f + acc_row<f32x4_t>(fg, i);
        if (row < n) {
          float* yr = Y + row * d + colw + fl;
#pragma unroll
          for (int c = 0; c < WC; ++c)
            if (colw + 16 * c + fl < d) yr[16 * c] = scale_out * acc[f][c][i];
        }
      }
    }
    if (!DERIV && nu != 0.0f) {  // + nu Omega (Y written by this thread above)
      for (int c = 0; c < WC; ++c) {
        const int col = colw + 16 * c + fl;
        if (col >= d) continue;
        for (int f = 0; f < 8; ++f)
          for (int i = 0; i < 4; ++i) {
            const int64_t row = row0 + 16 * f + acc_row<f32x4_t>(fg, i);
            if (row < n) Y[row * d + col] += nu * omega_value<LR_PREC_BF16>(omt, ld, col, row);
          }
      }
    }
  }
}

// Columns of the fragment copy: d rounded up to the widest column block.
int64_t omega_frag_cols(int d) {
  const int bn = kB16Waves * 16 * 4;
  return d <= kB16Waves * 16 ? kB16Waves * 16 : (d <= 2 * kB16Waves * 16 ? 2 * kB16Waves * 16 : (d + bn - 1) / bn * bn);
}

// plus kB16Ahead zero steps of padding, read by the last steps' (unused)
// prefetches
size_t omega_frag_bytes(int64_t n, int d) {
  const int64_t nst = (n + kDenseStep - 1) / kDenseStep;
  return ((size_t)(omega_frag_cols(d) / 16) * nst + kB16Ahead) * 64 * 16;
}

template <int KERNEL, int PD, int ND, int WC, bool DERIV, bool X2>
static hipError_t launch_bf16_impl(hipStream_t st, const void* pts, const uint4* frag, const void* omt, int64_t ld,
                                   int64_t n, int d, double scale_out, double nu, void* Y, int num_cu) {
  constexpr int NW = kB16Waves;
  constexpr int BN = NW * 16 * WC;
  const int nrb = (int)((n + kDenseRows - 1) / kDenseRows);
  const int ncb = (d + BN - 1) / BN;
  const int64_t nst = (n + kDenseStep - 1) / kDenseStep;
  // buffer views take 31-bit byte extents: 1 KB per step of a column group
  if (n > kBf16MaxRows) return hipErrorInvalidValue;
  int64_t blocks = (int64_t)nrb * ncb;
  if (blocks > num_cu) blocks = num_cu;
  hipLaunchKernelGGL((sketch_bf16_kernel<NW, KERNEL, PD, ND, WC, DERIV, X2>), dim3((unsigned)blocks), dim3(NW * 64), 0,
                     st, (const float*)pts, frag, nst, (const uint16_t*)omt, ld, n, d, (float)scale_out, (float)nu,
                     (float*)Y, nrb, ncb);
  return hipGetLastError();
}

template <int KERNEL, int PD, int ND, bool DERIV, bool X2>
static hipError_t launch_bf16_wc(hipStream_t st, const void* pts, const uint4* frag, const void* omt, int64_t ld,
                                 int64_t n, int d, double so, double nu, void* Y, int num_cu) {
  constexpr int cols_per_wc = kB16Waves * 16;
  if (d <= cols_per_wc)
    return launch_bf16_impl<KERNEL, PD, ND, 1, DERIV, X2>(st, pts, frag, omt, ld, n, d, so, nu, Y, num_cu);
  if (d <= 2 * cols_per_wc)
    return launch_bf16_impl<KERNEL, PD, ND, 2, DERIV, X2>(st, pts, frag, omt, ld, n, d, so, nu, Y, num_cu);
  // wider column blocks do not fit the register file with the operands;
  // larger d takes several column blocks
  return launch_bf16_impl<KERNEL, PD, ND, 4, DERIV, X2>(st, pts, frag, omt, ld, n, d, so, nu, Y, num_cu);
}

hipError_t launch_omega_frag(hipStream_t st, const void* omt, int64_t ld, int64_t n, int d, void* frag) {
  const int64_t nst = (n + kDenseStep - 1) / kDenseStep;
  const int64_t total = (omega_frag_cols(d) / 16 * nst + kB16Ahead) * 64;  // the last steps are the zero pad
  const int threads = 256;
  hipLaunchKernelGGL(omega_frag_kernel, dim3((unsigned)((total + threads - 1) / threads)), dim3(threads), 0, st,
                     (const uint16_t*)omt, ld, n, d, nst, total, (uint4*)frag);
  return hipGetLastError();
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
                                   int d, double so, double nu, void* Y, const void* frag, int num_cu) {
  if constexpr (PREC == LR_PREC_BF16X2) {
    // the split product runs on the matrix-core kernel only (D <= 3)
    if (D > 3 || frag == nullptr) return hipErrorInvalidValue;
    const uint4* f = static_cast<const uint4*>(frag);
    switch (D) {
      case 1: return launch_bf16_wc<KERNEL, 4, 1, DERIV, true>(st, pts, f, omt, ld, n, d, so, nu, Y, num_cu);
      case 2: return launch_bf16_wc<KERNEL, 4, 2, DERIV, true>(st, pts, f, omt, ld, n, d, so, nu, Y, num_cu);
      default: return launch_bf16_wc<KERNEL, 4, 3, DERIV, true>(st, pts, f, omt, ld, n, d, so, nu, Y, num_cu);
    }
  } else if constexpr (PREC == LR_PREC_BF16) {
    // D <= 3 (point stride 4): the matrix-core kernel on the fragment copy
    if (D <= 3) {
      if (frag == nullptr) return hipErrorInvalidValue;
      const uint4* f = static_cast<const uint4*>(frag);
      switch (D) {
        case 1: return launch_bf16_wc<KERNEL, 4, 1, DERIV, false>(st, pts, f, omt, ld, n, d, so, nu, Y, num_cu);
        case 2: return launch_bf16_wc<KERNEL, 4, 2, DERIV, false>(st, pts, f, omt, ld, n, d, so, nu, Y, num_cu);
        default: return launch_bf16_wc<KERNEL, 4, 3, DERIV, false>(st, pts, f, omt, ld, n, d, so, nu, Y, num_cu);
      }
    }
    if (D <= 7) return launch_dense_wn<PREC, KERNEL, 8, 7, DERIV>(st, pts, omt, ld, n, d, so, nu, Y, num_cu);
    return launch_dense_wn<PREC, KERNEL, 16, 15, DERIV>(st, pts, omt, ld, n, d, so, nu, Y, num_cu);
  } else {
    (void)frag;
    // Coordinates used: D itself for D <= 3 (stride 4), else every slot but the sign.
    switch (D) {
      case 1: return launch_dense_wn<PREC, KERNEL, 4, 1, DERIV>(st, pts, omt, ld, n, d, so, nu, Y, num_cu);
      case 2: return launch_dense_wn<PREC, KERNEL, 4, 2, DERIV>(st, pts, omt, ld, n, d, so, nu, Y, num_cu);
      case 3: return launch_dense_wn<PREC, KERNEL, 4, 3, DERIV>(st, pts, omt, ld, n, d, so, nu, Y, num_cu);
      default:
        if (D <= 7) return launch_dense_wn<PREC, KERNEL, 8, 7, DERIV>(st, pts, omt, ld, n, d, so, nu, Y, num_cu);
        return launch_dense_wn<PREC, KERNEL, 16, 15, DERIV>(st, pts, omt, ld, n, d, so, nu, Y, num_cu);
    }
  }
}

template <int PREC, bool DERIV>
static hipError_t launch_dense_prec(hipStream_t st, int kernel, int D, const void* pts, const void* omt,
                                    int64_t ld, int64_t n, int d, double so, double nu, void* Y, const void* frag,
                                    int num_cu) {
  if (kernel == LR_KERNEL_SE)
    return launch_dense_dim<PREC, LR_KERNEL_SE, DERIV>(st, D, pts, omt, ld, n, d, so, nu, Y, frag, num_cu);
  return launch_dense_dim<PREC, LR_KERNEL_MATERN32, DERIV>(st, D, pts, omt, ld, n, d, so, nu, Y, frag, num_cu);
}

hipError_t launch_sketch_dense(hipStream_t st, int prec, int kernel, int D, const void* pts, const void* omt,
                               int64_t ld, int64_t n, int d, double so, double nu, void* Y, bool deriv,
                               const void* frag, int num_cu) {
  if (prec == LR_PREC_BF16) {
    return deriv ? launch_dense_prec<LR_PREC_BF16, true>(st, kernel, D, pts, omt, ld, n, d, so, nu, Y, frag, num_cu)
                 : launch_dense_prec<LR_PREC_BF16, false>(st, kernel, D, pts, omt, ld, n, d, so, nu, Y, frag, num_cu);
  }
  if (prec == LR_PREC_BF16X2) {
    return deriv ? launch_dense_prec<LR_PREC_BF16X2, true>(st, kernel, D, pts, omt, ld, n, d, so, nu, Y, frag, num_cu)
                 : launch_dense_prec<LR_PREC_BF16X2, false>(st, kernel, D, pts, omt, ld, n, d, so, nu, Y, frag,
                                                            num_cu);
  }
  if (prec == LR_PREC_F32) {
    return deriv ? launch_dense_prec<LR_PREC_F32, true>(st, kernel, D, pts, omt, ld, n, d, so, nu, Y, frag, num_cu)
                 : launch_dense_prec<LR_PREC_F32, false>(st, kernel, D, pts, omt, ld, n, d, so, nu, Y, frag, num_cu);
  }
  return deriv ? launch_dense_prec<LR_PREC_F64, true>(st, kernel, D, pts, omt, ld, n, d, so, nu, Y, frag, num_cu)
               : launch_dense_prec<LR_PREC_F64, false>(st, kernel, D, pts, omt, ld, n, d, so, nu, Y, frag, num_cu);
}

}  // namespace lr
