// Structured random matrices written out densely: Omega[j,k] = D_j T[j, P_k]
// with T the orthonormal DCT-II, the discrete Hartley transform or the
// Walsh-Hadamard matrix (Def. 1 of Sec. 3.2; Sec. 5 uses the cosine and
// Hartley forms). The output is the transposed Omega (d rows of leading
// dimension ld, j contiguous) that the dense sketch, F = Omega^T Q and the
// backward read; one thread per entry, consecutive threads along j, so every
// store of a wave is contiguous.
//
// Accuracy: the angle is reduced exactly in 64-bit integers to the first octant
// before the float64 cospi/sinpi, so large j p never lose digits and zeros of
// the transform are exact; the float64 value is then
// rounded once to the output type (nearest even). For bf16 the float64 value
// is first cut to float with round-to-odd (truncate, then set the last bit if
// anything was cut), which makes the following float-to-bf16 rounding equal to
// a direct rounding of the float64 value.
#include "common.hpp"
#include "kernels.hpp"
#include "lrinv.h"

namespace lr {
namespace {

// cos(pi k / N) for an integer k: the quadrant is removed in integers
// (cos is even and 2N-periodic, cos(pi - a) = -cos a, cos a = sin(pi/2 - a)),
// so cospi / sinpi only see arguments in [0, 1/4] and the zeros are exact.
__device__ __forceinline__ double cos_pi_over(int64_t k, int64_t big_n) {
  const int64_t period = 2 * big_n;
  k %= period;
  if (k < 0) k += period;
  if (k > big_n) k = period - k;  // [0, N]
  double sign = 1.0;
  if (2 * k > big_n) {  // second quadrant
    k = big_n - k;
    sign = -1.0;
  }
  if (4 * k > big_n) return sign * sinpi((double)(big_n - 2 * k) / (2.0 * (double)big_n));
  return sign * cospi((double)k / (double)big_n);
}

__device__ __forceinline__ double structured_entry(int transform, int64_t n, int64_t j, int64_t p) {
  const int64_t pm = ((p % n) + n) % n;  // any index value stays in range
  if (transform == LR_TRANSFORM_DCT) {
    // a_p cos(pi (2j+1) p / (2n)); (2j+1) p < 2 n^2 fits in 64 bits for n <= 2^30
    const double a = pm == 0 ? sqrt(1.0 / (double)n) : sqrt(2.0 / (double)n);
    return a * cos_pi_over((2 * j + 1) * pm, 2 * n);
  }
  if (transform == LR_TRANSFORM_DHT) {
    // cas(2 pi m / n) = sqrt(2) cos(2 pi m / n - pi / 4) = sqrt(2) cos(pi (8m - n) / (4n))
    const int64_t m = (j * pm) % n;
    return sqrt(2.0) * cos_pi_over(8 * m - n, 4 * n) / sqrt((double)n);
  }
  // Walsh-Hadamard (n a power of two, checked on the host)
  return (__popcll((unsigned long long)(j & pm)) & 1 ? -1.0 : 1.0) / sqrt((double)n);
}

__device__ __forceinline__ uint16_t bf16_bits_rne(double v) {
  float f = __double2float_rz(v);
  unsigned int b = __float_as_uint(f);
  if ((double)f != v) b |= 1u;  // round to odd: keeps the cut part visible
  const unsigned int r = b + 0x7FFFu + ((b >> 16) & 1u);  // float -> bf16, nearest even
  return (uint16_t)(r >> 16);
}

template <typename T>
__device__ __forceinline__ T store_value(double v);
template <>
__device__ __forceinline__ double store_value<double>(double v) {
  return v;
}
template <>
__device__ __forceinline__ float store_value<float>(double v) {
  return (float)v;
}
template <>
__device__ __forceinline__ uint16_t store_value<uint16_t>(double v) {
  return bf16_bits_rne(v);
}

template <typename T>
__global__ void structured_omega_kernel(int transform, int64_t n, int64_t ld, int64_t total,
                                        const int8_t* __restrict__ signs, const int32_t* __restrict__ cols,
                                        T* __restrict__ out) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = q / ld;
    const int64_t j = q - k * ld;
    double v = 0.0;
    if (j < n) {
      v = structured_entry(transform, n, j, (int64_t)cols[k]);
      if (signs[j] < 0) v = -v;
    }
    out[q] = store_value<T>(v);
  }
}

}  // namespace

hipError_t launch_structured_omega(hipStream_t st, int transform, int64_t n, int d, const int8_t* signs,
                                   const int32_t* cols, int prec, void* out, int64_t ld, int num_cu) {
  const int64_t total = (int64_t)d * ld;
  const int threads = 256;
  int64_t blocks = (total + threads - 1) / threads;
  if (blocks > (int64_t)num_cu * 32) blocks = (int64_t)num_cu * 32;
  const dim3 g((unsigned)blocks), b(threads);
  if (prec == LR_PREC_F64)
    hipLaunchKernelGGL(structured_omega_kernel<double>, g, b, 0, st, transform, n, ld, total, signs, cols,
                       (double*)out);
  else if (prec == LR_PREC_F32)
    hipLaunchKernelGGL(structured_omega_kernel<float>, g, b, 0, st, transform, n, ld, total, signs, cols,
                       (float*)out);
  else
    hipLaunchKernelGGL(structured_omega_kernel<uint16_t>, g, b, 0, st, transform, n, ld, total, signs, cols,
                       (uint16_t*)out);
  return hipGetLastError();
}

}  // namespace lr
