// Register/LDS FFT building blocks for gfx950 (wave64, 64 KiB-class LDS budgets).
//
// Conventions: forward transforms use W_m = exp(-2 pi i / m) and are
// unnormalised; an inverse transform is computed as swap(FFT(swap(x))), where
// swap exchanges real and imaginary parts (a register renaming, no arithmetic).
//
// A length-NFFT transform is spread over TF = NFFT / P threads holding P points
// each.  Thread t always holds the elements {t + TF * i : 0 <= i < P}: that is
// the input set of the first Stockham pass and the output set of the last, so
// loads and stores of whole sequences are coalesced across threads, and between
// passes the data is exchanged through LDS.  Pass s has radix RAD = min(P,
// NFFT / NS), NS the product of the earlier radices (Stockham autosort, no bit
// reversal).  Twiddles come from one table of W_4096^k (k < 4096) computed in
// float64 on the host and rounded once; W_M^j = W_4096^(j * 4096 / M).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace fftenkf {

// Compile-time loop: f(std::integral_constant<int, I>) for I = B, B+S, ... < E.
// Used wherever a register array is indexed, so the index is always constant.
template <int B, int E, int S = 1, typename F>
__host__ __device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + S, E, S>(f);
  }
}

constexpr int kTwiddleN = 4096;

template <typename T> struct vec2;
template <> struct vec2<float> { using type = float2; };
template <> struct vec2<double> { using type = double2; };
template <typename T> using V2 = typename vec2<T>::type;

template <typename T> struct cx {
  T re, im;
};

template <typename T> __host__ __device__ __forceinline__ cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <typename T> __host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __host__ __device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return {a.re * s, a.im * s}; }
template <typename T> __host__ __device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
template <typename T> __host__ __device__ __forceinline__ cx<T> swapri(cx<T> a) { return {a.im, a.re}; }
// a * (-i)
template <typename T> __host__ __device__ __forceinline__ cx<T> mul_mi(cx<T> a) { return {a.im, -a.re}; }
// a * (+i)
template <typename T> __host__ __device__ __forceinline__ cx<T> mul_pi(cx<T> a) { return {-a.im, a.re}; }

// a * b + c with one rounding
__host__ __device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__host__ __device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T> __host__ __device__ __forceinline__ cx<T> from2(V2<T> v) { return {v.x, v.y}; }
template <typename T> __host__ __device__ __forceinline__ V2<T> to2(cx<T> a) {
  V2<T> v;
  v.x = a.re;
  v.y = a.im;
  return v;
}

// cos and sin of 2 pi k / 16, k = 0..15 (forward twiddle W_16^k = c - i s).
__host__ __device__ constexpr double kCos16(int k) {
  return k == 0 ? 1.0 : k == 1 ? 0.92387953251128675613 : k == 2 ? 0.70710678118654752440
       : k == 3 ? 0.38268343236508977173 : k == 4 ? 0.0 : k == 5 ? -0.38268343236508977173
       : k == 6 ? -0.70710678118654752440 : k == 7 ? -0.92387953251128675613 : k == 8 ? -1.0
       : k == 9 ? -0.92387953251128675613 : k == 10 ? -0.70710678118654752440
       : k == 11 ? -0.38268343236508977173 : k == 12 ? 0.0 : k == 13 ? 0.38268343236508977173
       : k == 14 ? 0.70710678118654752440 : 0.92387953251128675613;
}
__host__ __device__ constexpr double kSin16(int k) { return kCos16((k + 12) & 15); }  // sin x = cos(x - pi/2)

// Forward twiddle W_R^k for R dividing 16, as a constant.
template <typename T, int R>
__host__ __device__ __forceinline__ cx<T> w_const(int k) {
  const int j = ((k % R) + R) % R * (16 / R);
  return cx<T>{T(kCos16(j)), T(-kSin16(j))};
}

// Multiply by the constant W_16^k, using the cheapest form for the special angles.
template <typename T, int K>
__host__ __device__ __forceinline__ cx<T> mul_w16(cx<T> a) {
  constexpr int k = K & 15;
  if constexpr (k == 0) return a;
  else if constexpr (k == 4) return mul_mi(a);
  else if constexpr (k == 8) return cx<T>{-a.re, -a.im};
  else if constexpr (k == 12) return mul_pi(a);
  else if constexpr (k == 2 || k == 6 || k == 10 || k == 14) {
    constexpr T h = T(0.70710678118654752440);
    cx<T> b = k == 2 ? a : k == 6 ? mul_mi(a) : k == 10 ? cx<T>{-a.re, -a.im} : mul_pi(a);
    // b * (1 - i) / sqrt(2)
    return cx<T>{(b.re + b.im) * h, (b.im - b.re) * h};
  } else {
    return a * cx<T>{T(kCos16(k)), T(-kSin16(k))};
  }
}

// ---------------------------------------------------------------- small DFTs
// In-place forward DFT of R points in natural order.
template <typename T>
__host__ __device__ __forceinline__ void dft2(cx<T>& a, cx<T>& b) {
  cx<T> s = a + b, d = a - b;
  a = s;
  b = d;
}

template <typename T>
__host__ __device__ __forceinline__ void dft4(cx<T>& v0, cx<T>& v1, cx<T>& v2, cx<T>& v3) {
  cx<T> t0 = v0 + v2, t1 = v0 - v2, t2 = v1 + v3, t3 = mul_mi(v1 - v3);
  v0 = t0 + t2;
  v2 = t0 - t2;
  v1 = t1 + t3;
  v3 = t1 - t3;
}

template <typename T, int R>
__host__ __device__ __forceinline__ void dft(cx<T>* v) {
  if constexpr (R == 1) {
  } else if constexpr (R == 2) {
    dft2(v[0], v[1]);
  } else if constexpr (R == 4) {
    dft4(v[0], v[1], v[2], v[3]);
  } else if constexpr (R == 8) {
    cx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    cx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    o1 = mul_w16<T, 2>(o1);
    o2 = mul_w16<T, 4>(o2);
    o3 = mul_w16<T, 6>(o3);
    v[0] = e0 + o0; v[4] = e0 - o0;
    v[1] = e1 + o1; v[5] = e1 - o1;
    v[2] = e2 + o2; v[6] = e2 - o2;
    v[3] = e3 + o3; v[7] = e3 - o3;
  } else if constexpr (R == 16) {
    // n = n1 + 4 n2, k = k2 + 4 k1
    cx<T> y[4][4];
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) {
      y[n1][0] = v[n1]; y[n1][1] = v[n1 + 4]; y[n1][2] = v[n1 + 8]; y[n1][3] = v[n1 + 12];
      dft4(y[n1][0], y[n1][1], y[n1][2], y[n1][3]);
    }
    y[1][1] = mul_w16<T, 1>(y[1][1]); y[1][2] = mul_w16<T, 2>(y[1][2]); y[1][3] = mul_w16<T, 3>(y[1][3]);
    y[2][1] = mul_w16<T, 2>(y[2][1]); y[2][2] = mul_w16<T, 4>(y[2][2]); y[2][3] = mul_w16<T, 6>(y[2][3]);
    y[3][1] = mul_w16<T, 3>(y[3][1]); y[3][2] = mul_w16<T, 6>(y[3][2]); y[3][3] = mul_w16<T, 9>(y[3][3]);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) {
      cx<T> a = y[0][k2], b = y[1][k2], c = y[2][k2], d = y[3][k2];
      dft4(a, b, c, d);
      v[k2] = a; v[k2 + 4] = b; v[k2 + 8] = c; v[k2 + 12] = d;
    }
  } else {
    static_assert(R == 1, "unsupported radix");
  }
}

// Forward DFT of R real samples a[0..R-1]: V[k], k = 0..R/2 (V[0], V[R/2] real).
// Uses one complex DFT of length R/2 on z[m] = a[2m] + i a[2m+1].
template <typename T, int R>
__host__ __device__ __forceinline__ void rdft(const T* a, cx<T>* V) {
  constexpr int H = R / 2;
  cx<T> z[H];
#pragma unroll
  for (int m = 0; m < H; ++m) z[m] = cx<T>{a[2 * m], a[2 * m + 1]};
  dft<T, H>(z);
#pragma unroll
  for (int k = 0; k <= H; ++k) {
    cx<T> zk = z[k % H], zc = conj(z[(H - k) % H]);
    cx<T> e = scale(zk + zc, T(0.5));
    cx<T> o = scale(mul_mi(zk - zc), T(0.5));
    V[k] = e + w_const<T, R>(k) * o;
  }
  V[0].im = T(0);
  V[H].im = T(0);
}

// Unnormalised inverse of rdft: a[y] = sum over the Hermitian extension of V of
// V_k W_R^(-y k), i.e. V0 + (-1)^y V_{R/2} + 2 Re sum_{k=1}^{R/2-1} V_k W_R^(-y k).
// Only the real parts of V[0] and V[R/2] are used.
template <typename T, int R>
__host__ __device__ __forceinline__ void irdft(const cx<T>* V, T* a) {
  constexpr int H = R / 2;
  cx<T> Z[H];
#pragma unroll
  for (int k = 0; k < H; ++k) {
    cx<T> vk = V[k], vc = conj(V[H - k]);
    if (k == 0) {
      vk = cx<T>{V[0].re, T(0)};
      vc = cx<T>{V[H].re, T(0)};
    }
    cx<T> e = vk + vc;
    cx<T> o = (vk - vc) * conj(w_const<T, R>(k));
    Z[k] = e + mul_pi(o);
  }
  // unnormalised inverse DFT of length H by the swap trick
#pragma unroll
  for (int k = 0; k < H; ++k) Z[k] = swapri(Z[k]);
  dft<T, H>(Z);
#pragma unroll
  for (int m = 0; m < H; ++m) {
    cx<T> z = swapri(Z[m]);
    a[2 * m] = z.re;
    a[2 * m + 1] = z.im;
  }
}

// ------------------------------------------------------------ Stockham passes
// Twiddles W_M^(j m), m = 0..RAD-1, from the table; three table loads per radix-8
// butterfly (W^j, W^2j, W^4j), the rest by products of at most two levels.
// `tab` holds W_TWN^k for k < TWN (the 4096-entry device table, or a block's
// own copy of the TWN = NFFT twiddles in LDS); M divides TWN.
template <typename T, int RAD, int TWN = kTwiddleN>
__device__ __forceinline__ void load_twiddles(cx<T>* w, int j, int M, const V2<T>* __restrict__ tab) {
  const int s = TWN / M;
  w[0] = cx<T>{T(1), T(0)};
  if constexpr (RAD >= 2) w[1] = from2<T>(tab[j * s]);
  if constexpr (RAD >= 4) {
    w[2] = from2<T>(tab[2 * j * s]);
    w[3] = w[1] * w[2];
  }
  if constexpr (RAD >= 8) {
    w[4] = from2<T>(tab[4 * j * s]);
    w[5] = w[4] * w[1];
    w[6] = w[4] * w[2];
    w[7] = w[4] * w[3];
  }
  if constexpr (RAD >= 16) {
    w[8] = from2<T>(tab[8 * j * s]);
#pragma unroll
    for (int m = 9; m < 16; ++m) w[m] = w[8] * w[m - 8];
  }
}

// LDS index with one padding element after every 8: the strided writes of the
// Stockham passes then spread over the banks instead of piling on a few.
__device__ __forceinline__ int lds_pad(int idx) { return idx + (idx >> 3); }
// Elements to allocate for n logical elements.
__host__ __device__ constexpr int lds_padded_size(int n) { return n + (n >> 3) + 1; }

// LDS index of element e of the sequence held in column `off` of `stride`
// columns, relative to the sequence's block: the padded layout above.
struct PadLayout {
  static __device__ __forceinline__ int index(int e, int stride, int off) { return lds_pad(e * stride + off); }
};

// Rows of W columns of B-byte elements, unpadded.  The G = 256 / (W B) rows
// sharing one 256-byte line of banks are permuted: row e takes slot
// (e xor (e >> 2)) mod G of its group.  After a radix-4 pass a half-wave
// writes rows 4t + m for G consecutive t and reads rows t + const, and both
// sets then fall on distinct banks.
template <int W, int B>
struct SwizzleLayout {
  static constexpr int G = W * B >= 256 ? 1 : 256 / (W * B);
  static constexpr int elems(int rows) { return rows * W; }
  static __device__ __forceinline__ int index(int e, int, int off) {
    if constexpr (G == 1)
      return e * W + off;
    else
      return ((e & ~(G - 1)) + ((e ^ (e >> 2)) & (G - 1))) * W + off;
  }
};

// All passes of a length-NFFT transform for NB sequences held in registers,
// v[s][i] = element (t + TF i) of sequence s.  In LDS, sequence s occupies the
// block [s * SEQP, (s + 1) * SEQP) and its element e sits at
// Layout::index(e, elem_stride, lp.off) inside it (SEQP above the largest
// index), so the per-sequence part of every address is a constant.
// Every thread of the block must call this (it synchronises the block).
//
// LDS exchange: with buf1 == nullptr each exchange writes buf0, synchronises,
// reads, and synchronises again before the buffer can be rewritten.  With a
// second buffer the exchanges alternate between buf0 and buf1 (`parity`, kept
// by the caller across calls) and need one synchronisation each: a buffer is
// rewritten only after the next exchange's synchronisation.
struct LdsPair {
  void* buf0;
  void* buf1;
  int parity;
  int off;  // per-thread element offset added to every index (e.g. a column)
};

// Block barrier that orders LDS only: every wave's earlier LDS accesses
// complete before any wave passes it.  Unlike __syncthreads it does not wait
// for the wave's outstanding global loads and stores, which the exchanges do
// not need (every thread reads and writes its own global addresses).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Order a wave's own LDS writes before its later reads (and reads before later
// writes) without a block-wide barrier: LDS instructions of one wave execute in
// order, so only the compiler has to be kept from moving them.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// WAVE = true: all TF threads of a sequence belong to one wave and the LDS
// region they exchange through is private to that wave, so exchanges need no
// block synchronisation (buf1 is then ignored).
template <typename T, int NFFT, int P, int NS, int NB, int SEQP, bool WAVE = false, typename Layout = PadLayout,
          int TWN = kTwiddleN>
__device__ __forceinline__ void fft_passes(cx<T> (&v)[NB][P], int t, LdsPair& lp, int elem_stride,
                                           const V2<T>* __restrict__ tab) {
  if constexpr (NS < NFFT) {
    constexpr int RAD = (P < NFFT / NS) ? P : NFFT / NS;
    constexpr int Q = P / RAD;
    constexpr int TF = NFFT / P;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int b = t + TF * q;
      cx<T> w[RAD];
      if constexpr (NS > 1) load_twiddles<T, RAD, TWN>(w, b % NS, NS * RAD, tab);
#pragma unroll
      for (int s = 0; s < NB; ++s) {
        cx<T> a[RAD];
#pragma unroll
        for (int m = 0; m < RAD; ++m) a[m] = v[s][q + m * Q];
        if constexpr (NS > 1) {
#pragma unroll
          for (int m = 1; m < RAD; ++m) a[m] = a[m] * w[m];
        }
        dft<T, RAD>(a);
#pragma unroll
        for (int m = 0; m < RAD; ++m) v[s][q + m * Q] = a[m];
      }
    }
    if constexpr (NS * RAD < NFFT) {
      V2<T>* lds = static_cast<V2<T>*>((!WAVE && lp.buf1 != nullptr && lp.parity) ? lp.buf1 : lp.buf0);
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int b = t + TF * q;
        const int o = (b / NS) * NS * RAD + (b % NS);
#pragma unroll
        for (int m = 0; m < RAD; ++m) {
          V2<T>* dst = lds + Layout::index(o + m * NS, elem_stride, lp.off);
#pragma unroll
          for (int s = 0; s < NB; ++s) dst[s * SEQP] = to2<T>(v[s][q + m * Q]);
        }
      }
      if constexpr (WAVE) wave_lds_sync(); else lds_barrier();
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const V2<T>* src = lds + Layout::index(t + TF * i, elem_stride, lp.off);
#pragma unroll
        for (int s = 0; s < NB; ++s) v[s][i] = from2<T>(src[s * SEQP]);
      }
      if constexpr (WAVE)
        wave_lds_sync();
      else if (lp.buf1 == nullptr)
        lds_barrier();
      else
        lp.parity ^= 1;
      fft_passes<T, NFFT, P, NS * RAD, NB, SEQP, WAVE, Layout, TWN>(v, t, lp, elem_stride, tab);
    }
  }
}

template <typename T, int NFFT, int P, int NB, int SEQP, bool WAVE = false, typename Layout = PadLayout,
          int TWN = kTwiddleN>
__device__ __forceinline__ void fft_forward(cx<T> (&v)[NB][P], int t, LdsPair& lp, int elem_stride,
                                            const V2<T>* __restrict__ tab) {
  fft_passes<T, NFFT, P, 1, NB, SEQP, WAVE, Layout, TWN>(v, t, lp, elem_stride, tab);
}

template <typename T, int NFFT, int P, int NB, int SEQP, bool WAVE = false, typename Layout = PadLayout,
          int TWN = kTwiddleN>
__device__ __forceinline__ void fft_inverse(cx<T> (&v)[NB][P], int t, LdsPair& lp, int elem_stride,
                                            const V2<T>* __restrict__ tab) {
#pragma unroll
  for (int s = 0; s < NB; ++s)
#pragma unroll
    for (int i = 0; i < P; ++i) v[s][i] = swapri(v[s][i]);
  fft_passes<T, NFFT, P, 1, NB, SEQP, WAVE, Layout, TWN>(v, t, lp, elem_stride, tab);
#pragma unroll
  for (int s = 0; s < NB; ++s)
#pragma unroll
    for (int i = 0; i < P; ++i) v[s][i] = swapri(v[s][i]);
}

// Global memory access as uniform base + 32-bit unsigned byte offset, so the
// compiler can use the scalar-base addressing form and keep one 32-bit offset
// per element instead of a 64-bit address.
template <typename V>
__device__ __forceinline__ V ld_off(const V* base, uint32_t byte_off) {
  return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + byte_off);
}
template <typename V>
__device__ __forceinline__ void st_off(V* base, uint32_t byte_off, V v) {
  *reinterpret_cast<V*>(reinterpret_cast<char*>(base) + byte_off) = v;
}

// Raw buffer access: a resource over [base, base + bytes) (bytes < 2^32), with
// a per-thread 32-bit offset and a uniform 32-bit offset per access that the
// hardware adds; an access beyond `bytes` reads zero and writes nothing.  The
// per-thread offsets of a unit are computed once and reused for every field,
// whose offset travels in a scalar register, so no 64-bit vector address is
// formed per access.
struct Buf {
  __amdgpu_buffer_rsrc_t r;
};
__device__ __forceinline__ Buf make_buf(const void* base, uint32_t bytes) {
  return Buf{__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000)};
}
typedef unsigned int u32v2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32v4 __attribute__((ext_vector_type(4)));
template <typename T> __device__ __forceinline__ V2<T> buf_ld(const Buf& b, uint32_t voff, uint32_t soff);
template <> __device__ __forceinline__ float2 buf_ld<float>(const Buf& b, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(b.r, (int)voff, (int)soff, 0));
}
template <> __device__ __forceinline__ double2 buf_ld<double>(const Buf& b, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(b.r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ void buf_st(const Buf& b, uint32_t voff, uint32_t soff, float2 v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32v2, v), b.r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ void buf_st(const Buf& b, uint32_t voff, uint32_t soff, double2 v) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32v4, v), b.r, (int)voff, (int)soff, 0);
}

// Loads of data read once: the nontemporal hint lets the caches stream them
// instead of keeping lines no one will read again.
typedef float nt_float2 __attribute__((ext_vector_type(2)));
typedef double nt_double2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ld_stream(const float2* p) {
  const nt_float2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_float2*>(p));
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ double2 ld_stream(const double2* p) {
  const nt_double2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_double2*>(p));
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ float ld_stream(const float* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ double ld_stream(const double* p) { return __builtin_nontemporal_load(p); }

// Table entry W_M^k (forward) for M dividing 4096 and 0 <= k < M.
template <typename T>
__device__ __forceinline__ cx<T> twiddle(const V2<T>* __restrict__ tab, int k, int M) {
  return from2<T>(tab[k * (kTwiddleN / M)]);
}

}  // namespace fftenkf
