// Sweep 2: per frequency, the rest of the y transform, eq. (2), the gain and
// update of eq. (3) with the perturbations, and the inverse of that transform.
//
// A block owns a unit of C frequency columns (kx, k2) x all L values of y1, for
// every field (the N members and d), and keeps all of it in registers.  Thread
// (c, t2) = (tid % C, tid / C) holds, for column c, the elements
// y1 = t2 + TF2 * i (i < P) of each field: consecutive threads touch
// consecutive kx, so loads and stores are coalesced.  After the forward
// length-L transform it holds the bins k1 = t2 + TF2 * i, i.e. ky = k2 + R * k1,
// of every member and of d: statistics, gain, perturbation and update are
// thread-local.  The inverse transform starts from exactly those bins and ends
// on the y1 positions the thread loaded, which it overwrites in place.  The
// exchanges between passes go through two LDS buffers in turn (one block
// synchronisation each); every field's loads are issued before any transform,
// and each inverse round first draws and applies its members' update.
//
// The unit geometry (main and Nyquist units, XCD grouping) is spectral_unit.hpp.
#pragma once

#include <float.h>

#include "fft_core.hpp"
#include "kernels.hpp"
#include "philox.hpp"
#include "spectral_unit.hpp"

namespace fftenkf {

template <typename T> __device__ __forceinline__ T tiny_normal();
template <> __device__ __forceinline__ float tiny_normal<float>() { return FLT_MIN; }
template <> __device__ __forceinline__ double tiny_normal<double>() { return DBL_MIN; }

template <typename T> __device__ __forceinline__ T sqrt_t(T x);
template <> __device__ __forceinline__ float sqrt_t<float>(float x) { return sqrtf(x); }
template <> __device__ __forceinline__ double sqrt_t<double>(double x) { return sqrt(x); }

template <typename T>
struct K2Geom {
  // fields per LDS round: four for float32 buckets above 8 members (two waves
  // per SIMD at most, by registers); two for smaller buckets, whose registers
  // allow three or four waves per SIMD if the exchange buffers leave room
  template <int NMAX>
  static constexpr int fb() { return sizeof(T) == 4 && NMAX > 8 ? 4 : 2; }
  // columns of a full unit; a unit of fewer columns (narrow grids) leaves some unused
  template <int L>
  static constexpr int cols() { return k2_threads_target * k2_points(L) / L; }
  // LDS layout of one field's exchanges: L rows of cols() elements, swizzled
  template <int L>
  using Layout = SwizzleLayout<cols<L>(), (int)sizeof(V2<T>)>;
  template <int L>
  static constexpr int seqp() { return Layout<L>::elems(L); }
  // two exchange buffers of fb() fields, then the block's copy of W_L^k (k < L)
  template <int L, int NMAX>
  static constexpr size_t lds_bytes() { return (2 * (size_t)fb<NMAX>() * seqp<L>() + L) * sizeof(V2<T>); }
};

// The block's LDS copy of the twiddles W_L^k, k < L, of its length-L transforms.
// Reading them from LDS rather than from the device table keeps the
// transforms' waits off the vector-memory counter, which the loads and stores
// of whole fields share: a twiddle load issued behind them would make every
// pass wait for all of those to complete.
template <typename T, int L>
__device__ __forceinline__ const V2<T>* copy_twiddles(V2<T>* tw, const V2<T>* __restrict__ tab) {
  for (int k = threadIdx.x; k < L; k += blockDim.x) tw[k] = tab[k * (kTwiddleN / L)];
  return tw;
}

// The perturbation of one bin: Philox counter word 0 (the bin's canonical
// index gy * (nx/2 + 1) + kx) and the scales of the real and imaginary parts.
// In the kx = 0 and kx = nx/2 columns the bins above ny/2 take the conjugate of
// their mirror's draw and the self-conjugate bins a real draw of full variance.
template <typename T>
struct BinNoise {
  uint32_t ctr0;
  T zs, zi;
};

template <typename T>
__device__ __forceinline__ BinNoise<T> bin_noise(int kx, int ky, int nxh, int ny) {
  const bool edge = (kx == 0) || (kx == nxh);
  const bool mirrored = edge && ky > (ny >> 1);
  const bool selfconj = edge && (ky == 0 || ky == (ny >> 1));
  const int gy = mirrored ? ny - ky : ky;
  BinNoise<T> b;
  b.ctr0 = (uint32_t)(gy * (nxh + 1) + kx);
  b.zs = selfconj ? T(1) : T(0.70710678118654752440);
  b.zi = selfconj ? T(0) : (mirrored ? -b.zs : b.zs);
  return b;
}

// e_hat of members 2p and 2p + 1 at one bin, amp = sqrt(n R) (the unnormalised
// spectrum's scale): one Philox call, counter (ctr0, p, 0, 0), two Box-Muller pairs.
template <typename T>
__device__ __forceinline__ void draw_pair(const BinNoise<T>& b, int p, uint32_t key0, uint32_t key1, T amp,
                                          cx<T>& e0, cx<T>& e1) {
  const u32x4 w = philox4x32_10(u32x4{b.ctr0, (uint32_t)p, 0u, 0u}, key0, key1);
  T za, zb;
  box_muller<T>(w.x0, w.x1, za, zb);
  e0 = cx<T>{amp * b.zs * za, amp * b.zi * zb};
  box_muller<T>(w.x2, w.x3, za, zb);
  e1 = cx<T>{amp * b.zs * za, amp * b.zi * zb};
}

// Eq. (2) at point i of a thread: the sample variance of the N members'
// unnormalised coefficients times var_scale = 1 / ((N - 1) n).  The deviations
// are formed from s_f = u_f - u_0 (member 0 has s_0 = 0), which leaves them
// unchanged in exact arithmetic and makes the variance exactly zero when every
// member is the same, so the gain guard sees a collapsed ensemble as one.
template <typename T, int NMAX, int P>
__device__ __forceinline__ T sample_variance(const cx<T> (&u)[NMAX][P], int i, int N, T invN, T var_scale) {
  const cx<T> u0 = u[0][i];
  cx<T> mean{T(0), T(0)};
#pragma unroll
  for (int f = 1; f < NMAX; ++f)
    if (f < N) mean = mean + (u[f][i] - u0);
  mean = scale(mean, invN);
  T var = mean.re * mean.re + mean.im * mean.im;  // member 0: deviation -mean
#pragma unroll
  for (int f = 1; f < NMAX; ++f)
    if (f < N) {
      const cx<T> d = (u[f][i] - u0) - mean;
      var += d.re * d.re + d.im * d.im;
    }
  return var * var_scale;
}

// SPLIT compiles the modes that stop or start at the transformed fields
// (K2_STATS, K2_CHAT, K2_INVERSE); the single-pass modes are compiled without
// them.
// The work of one block; `unit` is its index within one analysis.
template <typename T, int L, int NMAX, bool SPLIT>
__device__ __forceinline__ void k2_body(const K2Args& a, int unit) {
  constexpr int P = k2_points(L);
  constexpr int TF2 = L / P;
  constexpr int FB = K2Geom<T>::template fb<NMAX>();
  constexpr int SEQP = K2Geom<T>::template seqp<L>();
  using Lay = typename K2Geom<T>::template Layout<L>;
  static_assert(NMAX % FB == 0 && FB % 2 == 0, "member bucket must be a multiple of the LDS batch");
  extern __shared__ unsigned char k2_lds_raw[];  // two buffers of FB fields, then W_L^k

  const V2<T>* __restrict__ tab = static_cast<const V2<T>*>(a.tab);
  const int C = a.C;
  const int tid = threadIdx.x;
  const int c = tid & (C - 1);
  const int t2 = tid / C;
  const int N = a.N, R = a.R, ny = a.ny;
  const int nxh = a.nx >> 1, nh = nxh + 1;

  // unit geometry: a uniform base pointer, a uniform field stride and per-thread
  // 32-bit byte offsets of the P elements
  const SpectralUnit<T> g = spectral_unit<T>(a.ws_main, a.ws_nyq, unit, c, C, R, L, ny, nxh, a.units_main,
                                             a.units_total, a.group_xcd);
  const int k2 = g.k2, kx = g.kx, cc = g.cc;
  const bool valid = g.valid;
  V2<T>* const ubase = g.ubase;
  const uint32_t fstride = g.fstride, sy = g.sy;
  uint32_t voff[P];
#pragma unroll
  for (int i = 0; i < P; ++i) voff[i] = ((uint32_t)(t2 + TF2 * i) * sy + (uint32_t)cc) * (uint32_t)sizeof(V2<T>);
  V2<T>* lds0 = reinterpret_cast<V2<T>*>(k2_lds_raw);
  LdsPair lp{lds0, lds0 + FB * SEQP, 0, c};
  // the twiddles (visible to all threads after the first exchange's barrier)
  const V2<T>* const tw = copy_twiddles<T, L>(lds0 + 2 * FB * SEQP, tab);

  // load: members into u, data into dv (first-pass layout)
  cx<T> u[NMAX][P];
  cx<T> dv[1][P];
  static_for<0, NMAX>([&](auto F) {
    constexpr int f = decltype(F)::value;
    if (f < N) {
      const V2<T>* fb = ubase + (size_t)f * fstride;
#pragma unroll
      for (int i = 0; i < P; ++i) u[f][i] = from2<T>(ld_off(fb, voff[i]));
    } else {
#pragma unroll
      for (int i = 0; i < P; ++i) u[f][i] = cx<T>{T(0), T(0)};
    }
  });
  {
    const V2<T>* fb = ubase + (size_t)N * fstride;
#pragma unroll
    for (int i = 0; i < P; ++i) dv[0][i] = from2<T>(ld_off(fb, voff[i]));
  }

  // forward length-L transforms (the inverse-only mode starts from transformed fields)
  const bool transformed = SPLIT && a.mode == K2_INVERSE;
  if (!transformed) {
#pragma unroll
  for (int f0 = 0; f0 < NMAX; f0 += FB) {
    if (f0 < N) {
      cx<T> blk[FB][P];
#pragma unroll
      for (int b = 0; b < FB; ++b)
#pragma unroll
        for (int i = 0; i < P; ++i) blk[b][i] = u[f0 + b][i];
      fft_forward<T, L, P, FB, SEQP, false, Lay, L>(blk, t2, lp, C, tw);
#pragma unroll
      for (int b = 0; b < FB; ++b)
#pragma unroll
        for (int i = 0; i < P; ++i) u[f0 + b][i] = blk[b][i];
    }
  }
  fft_forward<T, L, P, 1, SEQP, false, Lay, L>(dv, t2, lp, C, tw);
  }
  const bool valid_w = valid;

  // ---- eq. (2) per bin, then the gain of eq. (3)
  const T n_tot = T(a.nx) * T(ny);
  const T invN = T(1) / T(N);
  const T var_scale = T(1) / (T(N - 1) * n_tot);  // unitary (eigenvalue) scale
  const T sqrt_n = sqrt_t<T>(n_tot);
  const T* __restrict__ Rspec = static_cast<const T*>(a.R_spec);
  T gain[P], amp[P];
  int ky[P];
  T csum = T(0);
#pragma unroll
  for (int i = 0; i < P; ++i) {
    ky[i] = k2 + R * (t2 + TF2 * i);
    T chat = sample_variance<T, NMAX, P>(u, i, N, invN, var_scale);
    if (a.lam_map != nullptr && valid_w) chat = static_cast<const T*>(a.lam_map)[(size_t)ky[i] * nh + kx];
    T rb = T(a.r_scalar);
    if (Rspec != nullptr && valid_w) rb = Rspec[(size_t)ky[i] * nh + kx];
    const T den = chat + rb;
    gain[i] = den < tiny_normal<T>() ? T(0) : chat / den;
    if (SPLIT && (a.mode == K2_STATS || a.mode == K2_CHAT)) {
      if (valid_w) static_cast<T*>(a.chat_map)[(size_t)ky[i] * nh + kx] = chat;
      csum += valid_w ? chat : T(0);
    }
    amp[i] = sqrt_n * sqrt_t<T>(rb);  // sqrt(n R), without overflow of n R
    if (a.mode == K2_DEBUG_SPECTRA && valid_w) {
      const size_t bin = (size_t)ky[i] * nh + kx;
      static_cast<T*>(a.dbg_chat)[bin] = chat;
      static_cast<T*>(a.dbg_gain)[bin] = gain[i];
      if (a.dbg_spec != nullptr) {
        V2<T>* sp = static_cast<V2<T>*>(a.dbg_spec);
        const T us = T(1) / sqrt_t<T>(n_tot);
        const size_t plane = (size_t)ny * nh;
#pragma unroll
        for (int f = 0; f < NMAX; ++f)
          if (f < N) sp[f * plane + bin] = to2<T>(scale(u[f][i], us));
        sp[N * plane + bin] = to2<T>(scale(dv[0][i], us));
      }
    }
  }
  if (a.mode == K2_DEBUG_SPECTRA) return;  // no synchronisation follows
  if (SPLIT && (a.mode == K2_STATS || a.mode == K2_CHAT)) {
    // transformed fields back in place (K2_STATS), and this block's sum of c_hat
    if (valid && a.mode == K2_STATS) {
#pragma unroll
      for (int f = 0; f < NMAX; ++f)
        if (f < N) {
          V2<T>* fb = ubase + (size_t)f * fstride;
#pragma unroll
          for (int i = 0; i < P; ++i) st_off(fb, voff[i], to2<T>(u[f][i]));
        }
      V2<T>* fb = ubase + (size_t)N * fstride;
#pragma unroll
      for (int i = 0; i < P; ++i) st_off(fb, voff[i], to2<T>(dv[0][i]));
    }
    T* red = reinterpret_cast<T*>(k2_lds_raw);
    __syncthreads();  // the exchange buffers are free again
    red[tid] = csum;
    __syncthreads();
    if (tid == 0) {
      T tot = T(0);
      for (int k = 0; k < (int)blockDim.x; ++k) tot += red[k];
      static_cast<float*>(a.partials)[unit] = (float)tot;
    }
    return;
  }

  // ---- perturbations and update, two members per Philox call: the pairs
  // [PB, PE) of every bin the thread holds
  auto perturb = [&](auto PB, auto PE) __attribute__((always_inline)) {
    static_for<0, P>([&](auto I) __attribute__((always_inline)) {
      constexpr int i = decltype(I)::value;
      const BinNoise<T> bn = bin_noise<T>(kx, ky[i], nxh, ny);
      static_for<decltype(PB)::value, decltype(PE)::value>([&](auto PP) __attribute__((always_inline)) {
        constexpr int p = decltype(PP)::value;
        if (2 * p < N) {
          cx<T> e0, e1;
          draw_pair<T>(bn, p, a.key0, a.key1, amp[i], e0, e1);
          if (a.mode == K2_DEBUG_PERTURB) {  // test export of e_hat (unitary scale)
            if (valid_w) {
              V2<T>* ep = static_cast<V2<T>*>(a.dbg_e);
              const T us = T(1) / sqrt_t<T>(n_tot);
              const size_t bin = (size_t)ky[i] * nh + kx, plane = (size_t)ny * nh;
              ep[(2 * p) * plane + bin] = to2<T>(scale(e0, us));
              if (2 * p + 1 < N) ep[(2 * p + 1) * plane + bin] = to2<T>(scale(e1, us));
            }
          } else {
            const cx<T> ua = u[2 * p][i], ub = u[2 * p + 1][i];
            u[2 * p][i] = ua + scale(dv[0][i] + e0 - ua, gain[i]);
            if (2 * p + 1 < N) u[2 * p + 1][i] = ub + scale(dv[0][i] + e1 - ub, gain[i]);
          }
        }
      });
    });
  };
  if (a.mode == K2_DEBUG_PERTURB) {
    perturb(std::integral_constant<int, 0>{}, std::integral_constant<int, NMAX / 2>{});
    return;  // no synchronisation follows
  }

  // ---- per LDS round: update its members (their perturbations are drawn here,
  // so the stores of one round overlap the arithmetic of the next), then the
  // inverse length-L transforms, written back in place
  static_for<0, NMAX, FB>([&](auto F0) __attribute__((always_inline)) {
    constexpr int f0 = decltype(F0)::value;
    if (f0 < N) {
      if (!(SPLIT && a.mode == K2_INVERSE))
        perturb(std::integral_constant<int, f0 / 2>{}, std::integral_constant<int, (f0 + FB) / 2>{});
      cx<T> blk[FB][P];
#pragma unroll
      for (int b = 0; b < FB; ++b)
#pragma unroll
        for (int i = 0; i < P; ++i) blk[b][i] = u[f0 + b][i];
      fft_inverse<T, L, P, FB, SEQP, false, Lay, L>(blk, t2, lp, C, tw);
      if (valid) {
#pragma unroll
        for (int b = 0; b < FB; ++b)
          if (f0 + b < N) {
            V2<T>* fb = ubase + (size_t)(f0 + b) * fstride;
#pragma unroll
            for (int i = 0; i < P; ++i) st_off(fb, voff[i], to2<T>(blk[b][i]));
          }
      }
    }
  });
}

template <typename T, int L, int NMAX, bool SPLIT>
__global__ __launch_bounds__(k2_threads_target, 2) void k2_spectral(const K2Args a) {
  k2_body<T, L, NMAX, SPLIT>(a, blockIdx.x);
}

// A batch of analyses on one grid: blockIdx.y selects the analysis; b.k2 holds
// everything the analyses share.
template <typename T, int L, int NMAX>
__global__ __launch_bounds__(k2_threads_target, 2) void k2_spectral_batch(const BatchArgs b) {
  const BatchFilter& f = b.f[blockIdx.y];
  K2Args a = b.k2;
  a.ws_main = f.ws_main;
  a.ws_nyq = f.ws_nyq;
  a.R_spec = f.R_spec;
  a.r_scalar = f.r_scalar;
  a.key0 = f.key0;
  a.key1 = f.key1;
  k2_body<T, L, NMAX, false>(a, blockIdx.x);
}

template <typename T, int L, int NMAX>
hipError_t launch_k2_batch_shape(const BatchArgs& b, hipStream_t st) {
  constexpr int P = k2_points(L);
  const dim3 grid(b.k2.units_total, b.count), block(b.k2.C * (L / P));
  constexpr size_t lds_bytes = K2Geom<T>::template lds_bytes<L, NMAX>();
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&k2_spectral_batch<T, L, NMAX>),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL((k2_spectral_batch<T, L, NMAX>), grid, block, lds_bytes, st, b);
  return hipGetLastError();
}

template <typename T, int L, int NMAX, bool SPLIT>
hipError_t launch_k2_variant(const K2Args& a, hipStream_t st) {
  constexpr int P = k2_points(L);
  const dim3 grid(a.units_total), block(a.C * (L / P));
  constexpr size_t lds_bytes = K2Geom<T>::template lds_bytes<L, NMAX>();
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&k2_spectral<T, L, NMAX, SPLIT>),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL((k2_spectral<T, L, NMAX, SPLIT>), grid, block, lds_bytes, st, a);
  return hipGetLastError();
}

template <typename T, int L, int NMAX>
hipError_t launch_k2_shape(const K2Args& a, hipStream_t st) {
  const bool split = a.mode == K2_STATS || a.mode == K2_CHAT || a.mode == K2_INVERSE;
  if (split) return launch_k2_variant<T, L, NMAX, true>(a, st);
  return launch_k2_variant<T, L, NMAX, false>(a, st);
}

}  // namespace fftenkf
