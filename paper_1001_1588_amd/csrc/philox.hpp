// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As Easy
// as 1, 2, 3", SC'11) and Box-Muller, for the spectral perturbations e_k ~ N(0, R).
//
// Round: (hi0, lo0) = M0 * x0, (hi1, lo1) = M1 * x2,
//        x <- (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0);
// key bumped by the Weyl constants between rounds.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fftenkf {

struct u32x4 {
  uint32_t x0, x1, x2, x3;
};

// a ^ b ^ c in one instruction (v_bitop3_b32 with the truth table of XOR3)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c.x0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c.x2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c = u32x4{xor3(hi1, c.x1, k0), lo1, xor3(hi0, c.x3, k1), lo0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// Uniform in (0, 1): (2 * (w >> 9) + 1) * 2^-24, exact in binary32 and binary64.
template <typename T>
__device__ __forceinline__ T uniform_open(uint32_t w) {
  return T((int)(((w >> 9) << 1) | 1u)) * T(5.9604644775390625e-08);
}
// The same value in binary32 with one fewer instruction: the float with
// exponent 0 and mantissa w >> 9 is 1 + (w >> 9) 2^-23, and subtracting
// 1 - 2^-24 from it is exact (the operands are within a factor of two), which
// leaves (w >> 9) 2^-23 + 2^-24.
template <>
__device__ __forceinline__ float uniform_open<float>(uint32_t w) {
  return __builtin_bit_cast(float, (w >> 9) | 0x3F800000u) - 0.999999940395355224609375f;
}

// Box-Muller in parts: rho = sqrt(-2 ln u1), and cos, sin of 2 pi u2; the two
// standard normals are rho cos and rho sin.
template <typename T> __device__ __forceinline__ void box_muller_parts(uint32_t wa, uint32_t wb, T& rho, T& c, T& s);

// Two standard normals from two words (Box-Muller): rho (cos 2 pi u2, sin 2 pi u2).
template <typename T> __device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, T& a, T& b);

// float32: hardware log2, square root, and sine/cosine of 2 pi x (v_log_f32,
// v_sqrt_f32, v_sin_f32 and v_cos_f32 take their argument in revolutions);
// u1 >= 2^-24 keeps the logarithm finite and u2 < 1 stays in the hardware range.
template <>
__device__ __forceinline__ void box_muller_parts<float>(uint32_t wa, uint32_t wb, float& rho, float& c, float& s) {
  const float u1 = uniform_open<float>(wa);
  const float u2 = uniform_open<float>(wb);
  rho = __builtin_amdgcn_sqrtf(-1.38629436111989061883f * __builtin_amdgcn_logf(u1));  // -2 ln 2 log2(u1)
  c = __builtin_amdgcn_cosf(u2);
  s = __builtin_amdgcn_sinf(u2);
}

template <>
__device__ __forceinline__ void box_muller_parts<double>(uint32_t wa, uint32_t wb, double& rho, double& c,
                                                         double& s) {
  const double u1 = uniform_open<double>(wa);
  const double u2 = uniform_open<double>(wb);
  rho = sqrt(-2.0 * log(u1));
  sincospi(2.0 * u2, &s, &c);
}

template <typename T>
__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, T& a, T& b) {
  T rho, c, s;
  box_muller_parts<T>(wa, wb, rho, c, s);
  a = rho * c;
  b = rho * s;
}

}  // namespace fftenkf
