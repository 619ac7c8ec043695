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
// and each inverse round first draws and applies its members' update.  Float32
// analysis units of length-64 or length-128 columns (16 or 8 of them)
// transform with wave_fft.hpp instead (one exchange per transform), which
// leaves point i of a thread at bin k1 = wave_fft_bin<L>(t2, i).
//
// The unit geometry (XCD grouping) and the folded kx = 0 column, whose packed
// rows a fold unit splits after its forward transforms and joins before its
// inverse ones, are spectral_unit.hpp.
#pragma once

#include <float.h>

#include "fft_core.hpp"
#include "kernels.hpp"
#include "philox.hpp"
#include "spectral_unit.hpp"
#include "wave_fft.hpp"

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
  // two exchange buffers of fb() fields, the block's copy of W_L^k (k < L), then
  // the two fold exchange buffers of fb() fields
  template <int L, int NMAX>
  static constexpr size_t lds_bytes() {
    return (2 * (size_t)fb<NMAX>() * seqp<L>() + L + 2 * (size_t)fb<NMAX>() * L) * sizeof(V2<T>);
  }
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
// unnormalised coefficients times var_scale = 1 / ((N - 1) n), as the sums over
// the real and the imaginary parts (their total for a bin; the two variances of
// a pair slot's real bins).  The deviations are formed from s_f = u_f - u_0
// (member 0 has s_0 = 0), which leaves them unchanged in exact arithmetic and
// makes the variance exactly zero when every member is the same, so the gain
// guard sees a collapsed ensemble as one.
template <typename T, int NMAX, int P>
__device__ __forceinline__ cx<T> sample_variance(const cx<T> (&u)[NMAX][P], int i, int N, T invN, T var_scale) {
  const cx<T> u0 = u[0][i];
  cx<T> mean{T(0), T(0)};
#pragma unroll
  for (int f = 1; f < NMAX; ++f)
    if (f < N) mean = mean + (u[f][i] - u0);
  mean = scale(mean, invN);
  T vr = mean.re * mean.re, vi = mean.im * mean.im;  // member 0: deviation -mean
#pragma unroll
  for (int f = 1; f < NMAX; ++f)
    if (f < N) {
      const cx<T> d = (u[f][i] - u0) - mean;
      vr += d.re * d.re;
      vi += d.im * d.im;
    }
  return cx<T>{vr * var_scale, vi * var_scale};
}

// Kernel variants: K2V_PLAIN runs K2_ANALYZE without a given spectrum,
// K2V_LAM K2_ANALYZE with one (lam_map), K2V_CHAT K2_CHAT (the statistics pass
// of the learned analysis: members only, d neither read nor transformed),
// K2V_SPLIT every other mode (statistics with write-back, inverse-only and the
// test exports); the analysis kernel carries none of the others' code.
enum { K2V_PLAIN = 0, K2V_LAM = 1, K2V_SPLIT = 2, K2V_CHAT = 3 };

// The work of one block; `unit` is its index within one analysis.  FOLD:
// carry the split and join of packed rows and the pair slots (needed only by
// the units with g.fold); the analysis kernels run the body without them in
// every other unit, which keeps its registers to the common case.  WF: the
// transforms of wave_fft.hpp (float32 units of 1024 / L columns without a
// packed column, L = 64 or 128), whose bins sit at wave_fft_bin rather than
// in natural order; loads and stores are the same.
template <typename T, int L, int NMAX, int VAR, bool FOLD = true, bool WF = false>
__device__ __forceinline__ void k2_body(const K2Args& a, int unit) {
  static_assert(!WF || (wave_fft_length<L>() && !FOLD && VAR != K2V_SPLIT && std::is_same<T, float>::value),
                "the wave-level transform serves float32 units of length 64 or 128 whose fields are not stored back "
                "transformed");
  constexpr bool SPLIT = VAR == K2V_SPLIT || VAR == K2V_CHAT;  // the statistics and export code
  constexpr bool NEED_D = VAR != K2V_CHAT;
  const void* const lam_map = (VAR == K2V_LAM || VAR == K2V_SPLIT) ? a.lam_map : nullptr;
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
  const int mode = VAR == K2V_CHAT ? K2_CHAT : SPLIT ? a.mode : K2_ANALYZE;

  // unit geometry; every field is read and written through one buffer
  // resource over the unit's region, with per-thread byte offsets of the P
  // elements (shared by all fields) and a uniform byte offset per field
  const SpectralUnit<T> g = spectral_unit<T>(unit, c, C, R, L, ny, nxh, a.group_xcd);
  const int k2 = g.k2, kx = g.kx;
  const bool xlane = g.fold && g.col0;  // a thread of a packed column
  const Buf buf = make_buf(a.ws_main, a.main_bytes);
  const uint32_t fbytes = g.fstride * (uint32_t)sizeof(V2<T>);
  uint32_t voff[P];
#pragma unroll
  for (int i = 0; i < P; ++i) voff[i] = g.cbytes + (uint32_t)(t2 + TF2 * i) * g.sy * (uint32_t)sizeof(V2<T>);
  V2<T>* lds0 = reinterpret_cast<V2<T>*>(k2_lds_raw);
  LdsPair lp{lds0, lds0 + FB * SEQP, 0, c};
  // the twiddles (visible to all threads after the first exchange's barrier)
  const V2<T>* const tw = copy_twiddles<T, L>(lds0 + 2 * FB * SEQP, tab);
  V2<T>* const xch = lds0 + 2 * FB * SEQP + L;  // two buffers of FB x L, used in turn
  int xpar = 0;
  if constexpr (WF) lds_barrier();  // the twiddle copy, read before the first exchange
  const V2<float>* const twf = reinterpret_cast<const V2<float>*>(tw);
  // the length-L transforms of FB2 fields through the current exchange buffer
  auto fwd = [&](auto& blk) __attribute__((always_inline)) {
    constexpr int FB2 = sizeof(blk) / sizeof(blk[0]);
    if constexpr (WF) {
      wave_fft_forward<L, FB2>(blk, twf, reinterpret_cast<V2<float>*>(lp.parity ? lp.buf1 : lp.buf0), t2, c);
      lp.parity ^= 1;
    } else {
      fft_forward<T, L, P, FB2, SEQP, false, Lay, L>(blk, t2, lp, C, tw);
    }
  };
  auto inv = [&](auto& blk) __attribute__((always_inline)) {
    constexpr int FB2 = sizeof(blk) / sizeof(blk[0]);
    if constexpr (WF) {
      wave_fft_inverse<L, FB2>(blk, twf, reinterpret_cast<V2<float>*>(lp.parity ? lp.buf1 : lp.buf0), t2, c);
      lp.parity ^= 1;
    } else {
      fft_inverse<T, L, P, FB2, SEQP, false, Lay, L>(blk, t2, lp, C, tw);
    }
  };

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
  for (int i = 0; i < P; ++i)
    dv[0][i] = NEED_D ? from2<T>(buf_ld<T>(buf, voff[i], (uint32_t)N * fbytes)) : cx<T>{T(0), T(0)};

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
        fwd(blk);
        if (FOLD && g.fold) fold_exchange<T, FB, FB, P, TF2, L>(blk, xch, xpar, t2, xlane, k2, true);
#pragma unroll
        for (int b = 0; b < FB; ++b)
#pragma unroll
          for (int i = 0; i < P; ++i) u[f0 + b][i] = blk[b][i];
      }
    }
    if constexpr (NEED_D) {
      fwd(dv);
      if (FOLD && g.fold) fold_exchange<T, 1, FB, P, TF2, L>(dv, xch, xpar, t2, xlane, k2, true);
    }
  }

  // ---- eq. (2) per bin, then the gain g of eq. (3).  The update of a member
  // at a bin, u + g (d + e - u) with e = sqrt(n R) (zs rho cos, zi rho sin), is
  // evaluated as u (1 - g) + g d + rho (g sqrt(n R) zs cos, g sqrt(n R) zi sin):
  // the bin's factors omg = 1 - g, gd = g d and ga_re, ga_im are formed once.
  // A pair slot (only ever at points 0 and P/2 of a thread) holds two real
  // bins: its real and imaginary parts take their own variance, R, gain and
  // scale (the noise then draws a for the kx = 0 bin and b for kx = nx/2,
  // the shared draw of the two self-conjugate bins of a row).
  const T n_tot = T(a.nx) * T(ny);
  const T invN = T(1) / T(N);
  const T var_scale = T(1) / (T(N - 1) * n_tot);  // unitary (eigenvalue) scale
  const T sqrt_n = sqrt_t<T>(n_tot);
  const T* __restrict__ Rspec = static_cast<const T*>(a.R_spec);
  T omg[P], omgi[P], ga_re[P], ga_im[P];
  cx<T> gd[P];
  uint32_t ctr0[P];
  const ColumnBins cb = column_bins(k2, kx, t2, R, L);
  const int kxt = cb.thr < 0 ? nxh : kx;  // outside a packed column, every point's kx
  T csum = T(0);
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const int r = WF ? wave_fft_bin<L>(t2, i) : t2 + TF2 * i;
    const int ky = cb.kyb + R * r, kxb = FOLD ? (r > cb.thr ? nxh : kx) : kxt;
    const bool pr = FOLD && (i == 0 ? cb.pair0 : (i == P / 2 ? cb.pairh : false));
    const size_t bin = (size_t)ky * nh + kxb, bin_n = (size_t)ky * nh + nxh;
    const cx<T> vv = sample_variance<T, NMAX, P>(u, i, N, invN, var_scale);
    T chat = vv.re + vv.im, chat_i = chat;
    if (pr) {
      chat = vv.re;
      chat_i = vv.im;
    }
    if (lam_map != nullptr) {
      const T* lam = static_cast<const T*>(lam_map);
      chat = lam[bin];
      chat_i = pr ? lam[bin_n] : chat;
    }
    T rb = T(a.r_scalar), rbi = rb;
    if (Rspec != nullptr) {
      rb = Rspec[bin];
      rbi = pr ? Rspec[bin_n] : rb;
    }
    const T den = chat + rb, deni = chat_i + rbi;
    T gain = den < tiny_normal<T>() ? T(0) : chat / den;
    if (lam_map != nullptr && g.col0 && !pr) {
      // a given spectrum need not be even in ky: a kx = 0 or nx/2 slot stands
      // for its bin and the mirror (ny - ky, kx), and takes the mean of their
      // two gains, as the c2r transform of the updated half spectrum does
      const T cm = static_cast<const T*>(lam_map)[(size_t)((ny - ky) & (ny - 1)) * nh + kxb];
      const T dm = cm + rb;
      gain = T(0.5) * (gain + (dm < tiny_normal<T>() ? T(0) : cm / dm));
    }
    const T gain_i = pr ? (deni < tiny_normal<T>() ? T(0) : chat_i / deni) : gain;
    BinNoise<T> bn = bin_noise<T>(kxb, ky, nxh, ny);
    if (pr) bn.zi = T(1);
    const T amp = sqrt_n * sqrt_t<T>(rb);  // sqrt(n R), without overflow of n R
    const T amp_i = pr ? sqrt_n * sqrt_t<T>(rbi) : amp;
    const T amp_re = amp * bn.zs, amp_im = amp_i * bn.zi;
    ctr0[i] = bn.ctr0;
    omg[i] = T(1) - gain;
    omgi[i] = pr ? T(1) - gain_i : omg[i];
    gd[i] = cx<T>{gain * dv[0][i].re, gain_i * dv[0][i].im};
    ga_re[i] = gain * amp_re;
    ga_im[i] = gain_i * amp_im;
    if constexpr (SPLIT) {
      // exports cover the whole half spectrum: a kx = 0 column slot also writes
      // the mirror bin (ny - ky, kx) (the conjugate), a pair slot both real bins
      const size_t mir = (size_t)((ny - ky) & (ny - 1)) * nh + kxb;
      auto put_real = [&](T* plane, T v, T vi) __attribute__((always_inline)) {
        plane[bin] = v;
        if (pr) plane[bin_n] = vi;
        else if (g.col0) plane[mir] = v;
      };
      auto put_cx = [&](V2<T>* plane, cx<T> v) __attribute__((always_inline)) {
        if (pr) {
          plane[bin] = to2<T>(cx<T>{v.re, T(0)});
          plane[bin_n] = to2<T>(cx<T>{v.im, T(0)});
        } else {
          plane[bin] = to2<T>(v);
          if (g.col0) plane[mir] = to2<T>(conj(v));
        }
      };
      if (mode == K2_STATS || mode == K2_CHAT) {
        put_real(static_cast<T*>(a.chat_map), chat, chat_i);
        csum += pr ? chat + chat_i : (g.col0 ? T(2) * chat : chat);
      }
      if (mode == K2_DEBUG_SPECTRA) {
        put_real(static_cast<T*>(a.dbg_chat), chat, chat_i);
        put_real(static_cast<T*>(a.dbg_gain), gain, gain_i);
        if (a.dbg_spec != nullptr) {
          V2<T>* sp = static_cast<V2<T>*>(a.dbg_spec);
          const T us = T(1) / sqrt_n;
          const size_t plane = (size_t)ny * nh;
#pragma unroll
          for (int f = 0; f < NMAX; ++f)
            if (f < N) put_cx(sp + f * plane, scale(u[f][i], us));
          put_cx(sp + N * plane, scale(dv[0][i], us));
        }
      }
      if (mode == K2_DEBUG_PERTURB) {  // test export of e_hat (unitary scale)
        V2<T>* ep = static_cast<V2<T>*>(a.dbg_e);
        const T us = T(1) / sqrt_n;
        const size_t plane = (size_t)ny * nh;
        for (int p = 0; 2 * p < N; ++p) {
          const u32x4 w = philox4x32_10(u32x4{ctr0[i], (uint32_t)p, 0u, 0u}, a.key0, a.key1);
          T rho0, c0, s0, rho1, c1, s1;
          box_muller_parts<T>(w.x0, w.x1, rho0, c0, s0);
          box_muller_parts<T>(w.x2, w.x3, rho1, c1, s1);
          put_cx(ep + (2 * p) * plane, scale(cx<T>{amp_re * (rho0 * c0), amp_im * (rho0 * s0)}, us));
          if (2 * p + 1 < N)
            put_cx(ep + (2 * p + 1) * plane, scale(cx<T>{amp_re * (rho1 * c1), amp_im * (rho1 * s1)}, us));
        }
      }
    }
  }
  if constexpr (SPLIT) {
    if (mode == K2_DEBUG_SPECTRA || mode == K2_DEBUG_PERTURB) return;  // no synchronisation follows
    if (mode == K2_STATS || mode == K2_CHAT) {
      // transformed fields back in place (K2_STATS), and this block's sum of c_hat
      if (mode == K2_STATS) {
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
          const cx<T> ua = u[2 * p][i], ub = u[2 * p + 1][i];
          u[2 * p][i] = cx<T>{fma_t(rho0 * ga_re[i], c0, fma_t(ua.re, omg[i], gd[i].re)),
                              fma_t(rho0 * ga_im[i], s0, fma_t(ua.im, omgi[i], gd[i].im))};
          if (2 * p + 1 < N)
            u[2 * p + 1][i] = cx<T>{fma_t(rho1 * ga_re[i], c1, fma_t(ub.re, omg[i], gd[i].re)),
                                    fma_t(rho1 * ga_im[i], s1, fma_t(ub.im, omgi[i], gd[i].im))};
        }
      });
    });
  };

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
      if (FOLD && g.fold) fold_exchange<T, FB, FB, P, TF2, L>(blk, xch, xpar, t2, xlane, k2, false);
      inv(blk);
      // kx < nx/2 always holds: the branch keeps the compiler from moving a
      // round's stores into the next round's arithmetic, which costs registers
      if (kx < nxh) {
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

// Whether unit `unit` holds a packed column (spectral_unit's g.fold).
__device__ __forceinline__ bool unit_folds(int unit, int C, int R, int nxh, int group_xcd) {
  int um = unit;
  if (group_xcd > 1) {
    const int x = um & 7, q = um >> 3;
    um = group_xcd * (((q / group_xcd) << 3) + x) + (q & (group_xcd - 1));
  }
  const int nchunk = nxh / C;
  const int k2 = um / nchunk;
  return um - k2 * nchunk == 0 && (k2 == 0 || k2 == (R >> 1));
}

// Whether the analysis body runs the wave-level transforms on this shape.
template <typename T, int L, int VAR>
constexpr bool k2_wave_fft() { return std::is_same<T, float>::value && wave_fft_length<L>() && VAR != K2V_SPLIT; }

template <typename T, int L, int NMAX, int VAR>
__global__ __launch_bounds__(k2_threads_target, 2) void k2_spectral(const K2Args a) {
  if (VAR == K2V_SPLIT || unit_folds(blockIdx.x, a.C, a.R, a.nx >> 1, a.group_xcd))
    k2_body<T, L, NMAX, VAR, true>(a, blockIdx.x);
  else if constexpr (k2_wave_fft<T, L, VAR>()) {
    if (a.C == 1024 / L)
      k2_body<T, L, NMAX, VAR, false, true>(a, blockIdx.x);
    else
      k2_body<T, L, NMAX, VAR, false>(a, blockIdx.x);
  } else
    k2_body<T, L, NMAX, VAR, false>(a, blockIdx.x);
}

// A batch of analyses on one grid: blockIdx.y selects the analysis; b.k2 holds
// everything the analyses share.
template <typename T, int L, int NMAX>
__global__ __launch_bounds__(k2_threads_target, 2) void k2_spectral_batch(const BatchArgs b) {
  const BatchFilter& f = b.f[blockIdx.y];
  K2Args a = b.k2;
  a.ws_main = f.ws_main;
  a.R_spec = f.R_spec;
  a.r_scalar = f.r_scalar;
  a.key0 = f.key0;
  a.key1 = f.key1;
  if (unit_folds(blockIdx.x, a.C, a.R, a.nx >> 1, a.group_xcd))
    k2_body<T, L, NMAX, K2V_PLAIN, true>(a, blockIdx.x);
  else if constexpr (k2_wave_fft<T, L, K2V_PLAIN>()) {
    if (a.C == 1024 / L)
      k2_body<T, L, NMAX, K2V_PLAIN, false, true>(a, blockIdx.x);
    else
      k2_body<T, L, NMAX, K2V_PLAIN, false>(a, blockIdx.x);
  } else
    k2_body<T, L, NMAX, K2V_PLAIN, false>(a, blockIdx.x);
}

template <typename T, int L, int NMAX>
hipError_t launch_k2_batch_shape(const BatchArgs& b, hipStream_t st) {
  constexpr int P = k2_points(L);
  const dim3 grid(b.k2.units, b.count), block(b.k2.C * (L / P));
  constexpr size_t lds_bytes = K2Geom<T>::template lds_bytes<L, NMAX>();
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&k2_spectral_batch<T, L, NMAX>),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL((k2_spectral_batch<T, L, NMAX>), grid, block, lds_bytes, st, b);
  return hipGetLastError();
}

template <typename T, int L, int NMAX, int VAR>
hipError_t launch_k2_variant(const K2Args& a, hipStream_t st) {
  constexpr int P = k2_points(L);
  const dim3 grid(a.units), block(a.C * (L / P));
  constexpr size_t lds_bytes = K2Geom<T>::template lds_bytes<L, NMAX>();
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&k2_spectral<T, L, NMAX, VAR>),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL((k2_spectral<T, L, NMAX, VAR>), grid, block, lds_bytes, st, a);
  return hipGetLastError();
}

template <typename T, int L, int NMAX>
hipError_t launch_k2_shape(const K2Args& a, hipStream_t st) {
  if (a.mode == K2_CHAT) return launch_k2_variant<T, L, NMAX, K2V_CHAT>(a, st);
  if (a.mode != K2_ANALYZE) return launch_k2_variant<T, L, NMAX, K2V_SPLIT>(a, st);
  if (a.lam_map != nullptr) return launch_k2_variant<T, L, NMAX, K2V_LAM>(a, st);
  return launch_k2_variant<T, L, NMAX, K2V_PLAIN>(a, st);
}

}  // namespace fftenkf
