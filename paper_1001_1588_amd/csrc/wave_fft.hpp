// Length-64 and length-128 transforms of the spectral sweep with one block
// exchange.
//
// The sweep's thread (c, t2) = (tid % C, tid / C) of a 256-thread block holds
// elements n = t2 + (L/4) i (i < 4) of a column, C = 1024 / L columns (8 at
// L = 128, 16 at L = 64): the two top bits of n are the register index i, the
// next two the wave (t2 / (64 / C)), and the low bits (three at L = 128, two at
// L = 64) lane bits 3..5 or 4..5.  The forward transform is a decimation in
// frequency, digit by digit, each radix-4 (or 2) step on the digit that sits in
// registers:
//   1. radix 4 over i, twiddle W_L^(t2 p);
//   2. LDS transpose of the register digit with the wave digit, radix 4, twiddle
//      W_(L/4)^(l p) with l the lane part of t2;
//   3. v_permlane16_swap / v_permlane32_swap exchange the register digit with
//      lane bits 4 and 5, radix 4 (at L = 128 with twiddle W_8^(n0 p), n0 =
//      lane bit 3);
//   4. (L = 128) radix 2 across lane bit 3, the partner's value by a DPP row
//      rotation.
// X[k] then sits at k = p1 + 4 p2 + 16 p3 (+ 64 s at L = 128): p1 the wave, p2
// lane bits 4 and 5, p3 the register index and s lane bit 3 (wave_fft_bin).
// The inverse runs the same steps backwards with conjugate twiddles and returns
// x * L in the natural order, so loads and stores stay those of the Stockham
// form.  One block synchronisation per transform instead of three (L = 128) or
// two (L = 64).
#pragma once

#include "fft_core.hpp"

namespace fftenkf {

// Lengths served, and the frequency held by register i of the thread with row
// index t2.
template <int L>
constexpr bool wave_fft_length() { return L == 64 || L == 128; }
template <int L>
__host__ __device__ __forceinline__ int wave_fft_bin(int t2, int i) {
  if constexpr (L == 128) return (t2 >> 3) + 4 * ((t2 >> 1) & 3) + 16 * i + 64 * (t2 & 1);
  else return (t2 >> 2) + 4 * (t2 & 3) + 16 * i;
}

namespace wfft {

__device__ __forceinline__ void idft4(cx<float>& v0, cx<float>& v1, cx<float>& v2, cx<float>& v3) {
  const cx<float> t0 = v0 + v2, t1 = v0 - v2, t2 = v1 + v3, t3 = mul_pi(v1 - v3);
  v0 = t0 + t2;
  v2 = t0 - t2;
  v1 = t1 + t3;
  v3 = t1 - t3;
}

// Exchange register bit 0 with lane bit 4 (pairs 0-1 and 2-3) and register bit
// 1 with lane bit 5 (pairs 0-2 and 1-3): afterwards the value at lane bits
// (b4, b5), register (r0, r1) is the one that was at lane bits (r0, r1),
// register (b4, b5).  v_permlane16_swap_b32 a, b exchanges the odd rows of 16
// lanes of a with the even rows of b, v_permlane32_swap_b32 the upper 32 lanes
// of a with the lower 32 of b, both registers in place.  They are written as
// inline assembly with every operand read and written (the compiler's builtin
// for them has folded the second result into the first), and the s_nop
// instructions give the wait states at each dependence: after the VALU writes
// of the operands, between the two swap steps (the second reads the first's
// results) and before the VALU reads that follow.
__device__ __forceinline__ void swap_lane45(cx<float> (&v)[4]) {
  asm volatile(
      "s_nop 1\n\t"
      "v_permlane16_swap_b32 %0, %2\n\t"
      "v_permlane16_swap_b32 %1, %3\n\t"
      "v_permlane16_swap_b32 %4, %6\n\t"
      "v_permlane16_swap_b32 %5, %7\n\t"
      "s_nop 1\n\t"
      "v_permlane32_swap_b32 %0, %4\n\t"
      "v_permlane32_swap_b32 %1, %5\n\t"
      "v_permlane32_swap_b32 %2, %6\n\t"
      "v_permlane32_swap_b32 %3, %7\n\t"
      "s_nop 1"
      : "+v"(v[0].re), "+v"(v[0].im), "+v"(v[1].re), "+v"(v[1].im), "+v"(v[2].re), "+v"(v[2].im), "+v"(v[3].re),
        "+v"(v[3].im));
}

// The value of lane l ^ 8 (a rotation by 8 within each row of 16 lanes).
__device__ __forceinline__ float xor8(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x128, 0xF, 0xF, false));
}

// Radix 2 across lane bit 3, the forward and the (unnormalised) inverse alike:
// lane bit 3 = 0 takes own + partner, 1 takes partner - own.
__device__ __forceinline__ cx<float> radix2_lane8(cx<float> v, float sgn) {
  const cx<float> p{xor8(v.re), xor8(v.im)};
  return cx<float>{fma_t(sgn, v.re, p.re), fma_t(sgn, v.im, p.im)};
}

// Twiddle products with W_8^p (forward) or its conjugate, p = 1, 2, 3, applied
// where lane bit 3 is set.
template <bool INV>
__device__ __forceinline__ void twiddle8(cx<float> (&v)[4], bool odd) {
  constexpr float h = 0.70710678118654752440f;
  // forward W_8^1 = (1 - i) h, W_8^2 = -i, W_8^3 = -(1 + i) h; inverse conjugates
  const cx<float> a = v[1], b = v[2], c = v[3];
  const cx<float> ta = INV ? cx<float>{(a.re - a.im) * h, (a.re + a.im) * h} : cx<float>{(a.re + a.im) * h, (a.im - a.re) * h};
  const cx<float> tb = INV ? mul_pi(b) : mul_mi(b);
  const cx<float> tc = INV ? cx<float>{-(c.re + c.im) * h, (c.re - c.im) * h} : cx<float>{(c.im - c.re) * h, -(c.re + c.im) * h};
  v[1] = odd ? ta : a;
  v[2] = odd ? tb : b;
  v[3] = odd ? tc : c;
}

}  // namespace wfft

// The thread's twiddles, read from the block's LDS copy tw of W_L^k (k < L) at
// each transform rather than held across the sweep: W_L^t2, W_L^(2 t2) (step 1)
// and W_(L/4)^l, W_(L/4)^(2 l) (step 2); the third power of each is their
// product.
template <int L>
struct WaveTw {
  static constexpr int LB = L / 16;  // values of the lane part l of t2
  cx<float> w1a, w2a, w3a, w1b, w2b, w3b;
  float sgn;  // L = 128: +1 where lane bit 3 is clear, else -1
  bool odd;
  __device__ __forceinline__ WaveTw(const V2<float>* tw, int t2) {
    w1a = from2<float>(tw[t2]);
    w2a = from2<float>(tw[2 * t2]);
    const int l = t2 & (LB - 1);
    w1b = from2<float>(tw[4 * l]);
    w2b = from2<float>(tw[8 * l]);
    w3a = w1a * w2a;
    w3b = w1b * w2b;
    odd = (t2 & 1) != 0;
    sgn = odd ? -1.0f : 1.0f;
  }
};

// NB sequences, v[s][i] = element t2 + (L/4) i of sequence s in, frequency
// wave_fft_bin<L>(t2, i) out.  xbuf: NB x 4 x (L/4) x C elements of LDS, the
// thread's column c; tw: the block's W_L^k, visible to every thread (written
// before an earlier block synchronisation).  Every thread of the block calls
// it (one LDS barrier).
template <int L, int NB>
__device__ __forceinline__ void wave_fft_forward(cx<float> (&v)[NB][4], const V2<float>* tw, V2<float>* xbuf, int t2,
                                                 int c) {
  static_assert(wave_fft_length<L>(), "wave-level transform lengths: 64 and 128");
  constexpr int C = 1024 / L, Q = L / 4, LB = L / 16;
  const WaveTw<L> w(tw, t2);
#pragma unroll
  for (int s = 0; s < NB; ++s) {
    dft4(v[s][0], v[s][1], v[s][2], v[s][3]);
    v[s][1] = v[s][1] * w.w1a;
    v[s][2] = v[s][2] * w.w2a;
    v[s][3] = v[s][3] * w.w3a;
  }
  // register digit p to the wave: slot (p, n') of sequence s
#pragma unroll
  for (int s = 0; s < NB; ++s)
#pragma unroll
    for (int p = 0; p < 4; ++p) xbuf[((s * 4 + p) * Q + t2) * C + c] = to2<float>(v[s][p]);
  lds_barrier();
  const int wv = t2 / LB, l = t2 & (LB - 1);
#pragma unroll
  for (int s = 0; s < NB; ++s)
#pragma unroll
    for (int q = 0; q < 4; ++q) v[s][q] = from2<float>(xbuf[((s * 4 + wv) * Q + l + LB * q) * C + c]);
#pragma unroll
  for (int s = 0; s < NB; ++s) {
    dft4(v[s][0], v[s][1], v[s][2], v[s][3]);
    v[s][1] = v[s][1] * w.w1b;
    v[s][2] = v[s][2] * w.w2b;
    v[s][3] = v[s][3] * w.w3b;
    wfft::swap_lane45(v[s]);
    dft4(v[s][0], v[s][1], v[s][2], v[s][3]);
    if constexpr (L == 128) {
      wfft::twiddle8<false>(v[s], w.odd);
#pragma unroll
      for (int i = 0; i < 4; ++i) v[s][i] = wfft::radix2_lane8(v[s][i], w.sgn);
    }
  }
}

// The inverse: frequencies wave_fft_bin<L>(t2, i) in, L x element t2 + (L/4) i out.
template <int L, int NB>
__device__ __forceinline__ void wave_fft_inverse(cx<float> (&v)[NB][4], const V2<float>* tw, V2<float>* xbuf, int t2,
                                                 int c) {
  static_assert(wave_fft_length<L>(), "wave-level transform lengths: 64 and 128");
  constexpr int C = 1024 / L, Q = L / 4, LB = L / 16;
  const WaveTw<L> w(tw, t2);
#pragma unroll
  for (int s = 0; s < NB; ++s) {
    if constexpr (L == 128) {
#pragma unroll
      for (int i = 0; i < 4; ++i) v[s][i] = wfft::radix2_lane8(v[s][i], w.sgn);
      wfft::twiddle8<true>(v[s], w.odd);
    }
    wfft::idft4(v[s][0], v[s][1], v[s][2], v[s][3]);
    wfft::swap_lane45(v[s]);
    v[s][1] = v[s][1] * conj(w.w1b);
    v[s][2] = v[s][2] * conj(w.w2b);
    v[s][3] = v[s][3] * conj(w.w3b);
    wfft::idft4(v[s][0], v[s][1], v[s][2], v[s][3]);
  }
  const int wv = t2 / LB, l = t2 & (LB - 1);
#pragma unroll
  for (int s = 0; s < NB; ++s)
#pragma unroll
    for (int q = 0; q < 4; ++q) xbuf[((s * 4 + wv) * Q + l + LB * q) * C + c] = to2<float>(v[s][q]);
  lds_barrier();
#pragma unroll
  for (int s = 0; s < NB; ++s)
#pragma unroll
    for (int p = 0; p < 4; ++p) v[s][p] = from2<float>(xbuf[((s * 4 + p) * Q + t2) * C + c]);
#pragma unroll
  for (int s = 0; s < NB; ++s) {
    v[s][1] = v[s][1] * conj(w.w1a);
    v[s][2] = v[s][2] * conj(w.w2a);
    v[s][3] = v[s][3] * conj(w.w3a);
    wfft::idft4(v[s][0], v[s][1], v[s][2], v[s][3]);
  }
}

}  // namespace fftenkf
