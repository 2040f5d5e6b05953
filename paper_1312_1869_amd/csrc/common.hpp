// Shared device definitions for the lrinv HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "lrinv.h"

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x4_t __attribute__((ext_vector_type(4)));

namespace lr {

// zero rows appended to the prescaled point array
constexpr int kPointPad = 128;

constexpr double kLog2e = 1.4426950408889634074;
constexpr double kLn2 = 0.69314718055994530942;
constexpr int kWave = 64;

// Padded stride (in elements) of the prescaled point array: the coordinates in
// slots [0, D), zeros up to PD-1, and the SRHT sign (+-1) in slot PD-1.
__host__ __device__ inline int point_stride(int D) { return D <= 3 ? 4 : (D <= 7 ? 8 : 16); }

// Coordinates are prescaled so the kernels need only exp2 and sqrt:
//   SE:        x^ = x sqrt(log2(e) / 2) / ell,  k/s^2 = exp2(-r^2),
//              (dk/dlog ell)/s^2 = exp2(-r^2) * r^2 * 2 ln2       (r^ = |x^_i - x^_j|)
//   Matern32:  x^ = x sqrt(3) log2(e) / ell,     u^ = r^ = u log2(e),
//              k/s^2 = (1 + u^ ln2) exp2(-u^),  (dk/dlog ell)/s^2 = (u^ ln2)^2 exp2(-u^)
inline double coord_scale(int kernel, double ell) {
  if (kernel == LR_KERNEL_SE) return sqrt(0.5 * kLog2e) / ell;
  return sqrt(3.0) * kLog2e / ell;
}

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

template <int KERNEL>
struct KernelF32 {
  // value / s^2 from the prescaled squared distance
  __device__ __forceinline__ static float value(float r2) {
    if constexpr (KERNEL == LR_KERNEL_SE) {
      return fast_exp2(-r2);
    } else {
      float u = fast_sqrt(r2);
      return __builtin_fmaf(u, (float)kLn2, 1.0f) * fast_exp2(-u);
    }
  }
  __device__ __forceinline__ static float deriv(float r2) {
    if constexpr (KERNEL == LR_KERNEL_SE) {
      return fast_exp2(-r2) * (r2 * (float)(2.0 * kLn2));
    } else {
      float u = fast_sqrt(r2);
      float ul = u * (float)kLn2;
      return ul * ul * fast_exp2(-u);
    }
  }
  // both at once (shares the exponential)
  __device__ __forceinline__ static void both(float r2, float& v, float& dv) {
    if constexpr (KERNEL == LR_KERNEL_SE) {
      float e = fast_exp2(-r2);
      v = e;
      dv = e * (r2 * (float)(2.0 * kLn2));
    } else {
      float u = fast_sqrt(r2);
      float e = fast_exp2(-u);
      float ul = u * (float)kLn2;
      v = (1.0f + ul) * e;
      dv = ul * ul * e;
    }
  }
};

template <int KERNEL>
struct KernelF64 {
  __device__ __forceinline__ static double value(double r2) {
    if constexpr (KERNEL == LR_KERNEL_SE) {
      return exp2(-r2);
    } else {
      double u = sqrt(r2);
      return fma(u, kLn2, 1.0) * exp2(-u);
    }
  }
  __device__ __forceinline__ static double deriv(double r2) {
    if constexpr (KERNEL == LR_KERNEL_SE) {
      return exp2(-r2) * (r2 * (2.0 * kLn2));
    } else {
      double u = sqrt(r2);
      double ul = u * kLn2;
      return ul * ul * exp2(-u);
    }
  }
  __device__ __forceinline__ static void both(double r2, double& v, double& dv) {
    if constexpr (KERNEL == LR_KERNEL_SE) {
      double e = exp2(-r2);
      v = e;
      dv = e * (r2 * (2.0 * kLn2));
    } else {
      double u = sqrt(r2);
      double e = exp2(-u);
      double ul = u * kLn2;
      v = (1.0 + ul) * e;
      dv = ul * ul * e;
    }
  }
};

template <typename T, int KERNEL>
struct KernelT;
template <int KERNEL>
struct KernelT<float, KERNEL> : KernelF32<KERNEL> {};
template <int KERNEL>
struct KernelT<double, KERNEL> : KernelF64<KERNEL> {};

// DPP lane moves (GFX9 encodings): quad_perm [1,0,3,2] and [2,3,0,1] swap
// lanes xor 1 and xor 2; row_ror:4 and row_ror:8 rotate within 16-lane rows.
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Wave-wide sum (64 lanes), every lane gets the total: four DPP steps give each
// 16-lane row its sum, two xor shuffles combine the rows. Fixed order, so the
// result is the same on every call.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  v += dpp_move<0xB1>(v);
  v += dpp_move<0x4E>(v);
  v += dpp_move<0x124>(v);
  v += dpp_move<0x128>(v);
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Calls f(std::integral_constant<int, I>{}) for I = B .. E-1, expanded at
// compile time, so register arrays indexed by I inside f stay in registers.
// (#pragma unroll may be declined for large bodies, and a register array
// indexed by a loop variable then lives in scratch memory.)
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(static_cast<F&&>(f));
  }
}

// Row (within a 16 x 16 output fragment) of accumulator register i for a lane
// in k-group g = lane / 16 (the column is lane % 16). The float32 16x16x4 and
// bf16 16x16x32 instructions give row 4g + i; the float64 16x16x4 instruction
// gives row g + 4i (measured on gfx950).
template <typename Acc>
__device__ __forceinline__ int acc_row(int g, int i) {
  if constexpr (sizeof(Acc) == 4 * sizeof(double)) return g + 4 * i;
  return 4 * g + i;
}

}  // namespace lr
