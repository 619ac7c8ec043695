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

// SPLIT compiles every mode but K2_ANALYZE (the statistics-only, inverse-only
// and test-export modes); the single-pass variant is compiled without them.
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
  const int mode = SPLIT ? a.mode : K2_ANALYZE;

  // unit geometry; every field is read and written through one buffer
  // resource over the unit's region, with per-thread byte offsets of the P
  // elements (shared by all fields) and a uniform byte offset per field
  const SpectralUnit<T> g = spectral_unit<T>(a.ws_main, a.ws_nyq, unit, c, C, a.Cn, R, L, ny, nxh, a.units_main,
                                             a.units_total, a.group_xcd);
  const int k2 = g.k2, kx = g.kx;
  const bool valid = g.valid;
  const Buf buf = make_buf(g.nyq ? a.ws_nyq : a.ws_main, g.nyq ? a.nyq_bytes : a.main_bytes);
  const uint32_t fbytes = g.fstride * (uint32_t)sizeof(V2<T>);
  uint32_t voff[P];
#pragma unroll
  for (int i = 0; i < P; ++i) voff[i] = g.cbytes + (uint32_t)(t2 + TF2 * i) * g.sy * (uint32_t)sizeof(V2<T>);
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
#pragma unroll
      for (int i = 0; i < P; ++i) u[f][i] = from2<T>(buf_ld<T>(buf, voff[i], (uint32_t)f * fbytes));
    } else {
#pragma unroll
      for (int i = 0; i < P; ++i) u[f][i] = cx<T>{T(0), T(0)};
    }
  });
#pragma unroll
  for (int i = 0; i < P; ++i) dv[0][i] = from2<T>(buf_ld<T>(buf, voff[i], (uint32_t)N * fbytes));

  // forward length-L transforms (the inverse-only mode starts from transformed fields)
  if (mode != K2_INVERSE) {
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

  // ---- eq. (2) per bin, then the gain g of eq. (3).  The update of a member
  // at a bin, u + g (d + e - u) with e = sqrt(n R) (zs rho cos, zi rho sin), is
  // evaluated as u (1 - g) + g d + rho (g sqrt(n R) zs cos, g sqrt(n R) zi sin):
  // the bin's factors omg = 1 - g, gd = g d and ga_re, ga_im are formed once.
  const T n_tot = T(a.nx) * T(ny);
  const T invN = T(1) / T(N);
  const T var_scale = T(1) / (T(N - 1) * n_tot);  // unitary (eigenvalue) scale
  const T sqrt_n = sqrt_t<T>(n_tot);
  const T* __restrict__ Rspec = static_cast<const T*>(a.R_spec);
  T gain[P], amp_re[P], amp_im[P], omg[P], ga_re[P], ga_im[P];
  cx<T> gd[P];
  uint32_t ctr0[P];
  int ky[P];
  T csum = T(0);
#pragma unroll
  for (int i = 0; i < P; ++i) {
    ky[i] = k2 + R * (t2 + TF2 * i);
    T chat = sample_variance<T, NMAX, P>(u, i, N, invN, var_scale);
    if (a.lam_map != nullptr && valid) chat = static_cast<const T*>(a.lam_map)[(size_t)ky[i] * nh + kx];
    T rb = T(a.r_scalar);
    if (Rspec != nullptr && valid) rb = Rspec[(size_t)ky[i] * nh + kx];
    const T den = chat + rb;
    gain[i] = den < tiny_normal<T>() ? T(0) : chat / den;
    const BinNoise<T> bn = bin_noise<T>(kx, ky[i], nxh, ny);
    const T amp = sqrt_n * sqrt_t<T>(rb);  // sqrt(n R), without overflow of n R
    amp_re[i] = amp * bn.zs;
    amp_im[i] = amp * bn.zi;
    ctr0[i] = bn.ctr0;
    omg[i] = T(1) - gain[i];
    gd[i] = scale(dv[0][i], gain[i]);
    ga_re[i] = gain[i] * amp_re[i];
    ga_im[i] = gain[i] * amp_im[i];
    if constexpr (SPLIT) {
      if (mode == K2_STATS || mode == K2_CHAT) {
        if (valid) static_cast<T*>(a.chat_map)[(size_t)ky[i] * nh + kx] = chat;
        csum += valid ? chat : T(0);
      }
      if (mode == K2_DEBUG_SPECTRA && valid) {
        const size_t bin = (size_t)ky[i] * nh + kx;
        static_cast<T*>(a.dbg_chat)[bin] = chat;
        static_cast<T*>(a.dbg_gain)[bin] = gain[i];
        if (a.dbg_spec != nullptr) {
          V2<T>* sp = static_cast<V2<T>*>(a.dbg_spec);
          const T us = T(1) / sqrt_n;
          const size_t plane = (size_t)ny * nh;
#pragma unroll
          for (int f = 0; f < NMAX; ++f)
            if (f < N) sp[f * plane + bin] = to2<T>(scale(u[f][i], us));
          sp[N * plane + bin] = to2<T>(scale(dv[0][i], us));
        }
      }
    }
  }
  if constexpr (SPLIT) {
    if (mode == K2_DEBUG_SPECTRA) return;  // no synchronisation follows
    if (mode == K2_STATS || mode == K2_CHAT) {
      // transformed fields back in place (K2_STATS), and this block's sum of c_hat
      if (valid && mode == K2_STATS) {
#pragma unroll
        for (int f = 0; f < NMAX; ++f)
          if (f < N) {
#pragma unroll
            for (int i = 0; i < P; ++i) buf_st(buf, voff[i], (uint32_t)f * fbytes, to2<T>(u[f][i]));
          }
#pragma unroll
        for (int i = 0; i < P; ++i) buf_st(buf, voff[i], (uint32_t)N * fbytes, to2<T>(dv[0][i]));
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
  }

  // ---- perturbations and update, two members per Philox call (counter
  // (bin, p, 0, 0) gives members 2p and 2p + 1): the pairs [PB, PE) of every
  // bin the thread holds
  auto perturb = [&](auto PB, auto PE) __attribute__((always_inline)) {
    static_for<0, P>([&](auto I) __attribute__((always_inline)) {
      constexpr int i = decltype(I)::value;
      static_for<decltype(PB)::value, decltype(PE)::value>([&](auto PP) __attribute__((always_inline)) {
        constexpr int p = decltype(PP)::value;
        if (2 * p < N) {
          const u32x4 w = philox4x32_10(u32x4{ctr0[i], (uint32_t)p, 0u, 0u}, a.key0, a.key1);
          T rho0, c0, s0, rho1, c1, s1;
          box_muller_parts<T>(w.x0, w.x1, rho0, c0, s0);
          box_muller_parts<T>(w.x2, w.x3, rho1, c1, s1);
          if (SPLIT && mode == K2_DEBUG_PERTURB) {  // test export of e_hat (unitary scale)
            if (valid) {
              const cx<T> e0{amp_re[i] * (rho0 * c0), amp_im[i] * (rho0 * s0)};
              const cx<T> e1{amp_re[i] * (rho1 * c1), amp_im[i] * (rho1 * s1)};
              V2<T>* ep = static_cast<V2<T>*>(a.dbg_e);
              const T us = T(1) / sqrt_n;
              const size_t bin = (size_t)ky[i] * nh + kx, plane = (size_t)ny * nh;
              ep[(2 * p) * plane + bin] = to2<T>(scale(e0, us));
              if (2 * p + 1 < N) ep[(2 * p + 1) * plane + bin] = to2<T>(scale(e1, us));
            }
          } else {
            const cx<T> ua = u[2 * p][i], ub = u[2 * p + 1][i];
            u[2 * p][i] = cx<T>{fma_t(rho0 * ga_re[i], c0, fma_t(ua.re, omg[i], gd[i].re)),
                                fma_t(rho0 * ga_im[i], s0, fma_t(ua.im, omg[i], gd[i].im))};
            if (2 * p + 1 < N)
              u[2 * p + 1][i] = cx<T>{fma_t(rho1 * ga_re[i], c1, fma_t(ub.re, omg[i], gd[i].re)),
                                      fma_t(rho1 * ga_im[i], s1, fma_t(ub.im, omg[i], gd[i].im))};
          }
        }
      });
    });
  };
  if constexpr (SPLIT) {
    if (mode == K2_DEBUG_PERTURB) {
      perturb(std::integral_constant<int, 0>{}, std::integral_constant<int, NMAX / 2>{});
      return;  // no synchronisation follows
    }
  }

  // ---- per LDS round: update its members (their perturbations are drawn here,
  // so the stores of one round overlap the arithmetic of the next), then the
  // inverse length-L transforms, written back in place
  static_for<0, NMAX, FB>([&](auto F0) __attribute__((always_inline)) {
    constexpr int f0 = decltype(F0)::value;
    if (f0 < N) {
      if (mode != K2_INVERSE)
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
#pragma unroll
            for (int i = 0; i < P; ++i) buf_st(buf, voff[i], (uint32_t)(f0 + b) * fbytes, to2<T>(blk[b][i]));
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
  if (a.mode != K2_ANALYZE) return launch_k2_variant<T, L, NMAX, true>(a, st);
  return launch_k2_variant<T, L, NMAX, false>(a, st);
}

}  // namespace fftenkf
