// Spectral sweep of a state of M blocks (fields) of which the first K are
// observed (Section 2.2): the multi-block analysis (K = 1, eq. (6) with eq. (7))
// and the extended state of the morphing EnKF (eq. (9): T_x, T_y and r(1)
// observed, K = 3), with the cross-covariances among the observed fields
// neglected, so that their covariance is K diagonal matrices.
//
// Units, thread layout, transforms and the perturbation convention are those
// of the single-block sweep (k2_spectral.hpp).  Per bin, with delta^(o)_k the
// deviations of observed block o and D_o = c_hat^(oo) + R_o:
//   observed block o:    u^(o)a_k = u^(o)_k + c_hat^(oo) / D_o (d_o + e_ko - u^(o)_k)
//   unobserved block j:  u^(j)a_k = u^(j)_k + sum_o c_hat^(jo) / D_o (d_o + e_ko - u^(o)_k),
//   c_hat^(jo) = 1/(N-1) sum_k (u^(j)_k - mean^(j)) conj(delta^(o)_k)   (eq. (7),
//   the conjugate on the observed factor),
// and no update from field o where D_o is below the smallest normal number.
// e_ko is drawn with Philox counter (bin, k div 2, 0, o): field 0 draws the
// single-block stream.
//
// A unit keeps delta^(o) and d_o - mean^(o) of every observed field in
// registers.  Each observed block is updated, inverse transformed and stored
// right after its statistics; every unobserved block is then streamed through
// one more register set: loaded, transformed, centred, its K cross-covariances
// formed, updated with the regenerated perturbations, inverse transformed and
// stored.  The workspace holds member k of block j as field k M + j and d_o as
// field N M + o; each field is addressed through its own buffer resource, so
// any number of fields fits 32-bit offsets.  The packed kx = 0 column of a fold
// unit is split after each forward transform and joined before each inverse
// one (spectral_unit.hpp); a pair slot's real and imaginary parts are two real
// bins with their own statistics, gains and noise scales.
#pragma once

#include "k2_spectral.hpp"

namespace fftenkf {

// Waves per SIMD: two while the K + 1 register sets of a thread stay within
// the budget of two waves, else one (registers spread over the unified file).
template <typename T, int NMAX, int KMAX>
constexpr int k10_waves() { return (KMAX + 1) * NMAX * (int)sizeof(T) <= 80 ? 2 : 1; }

// Two exchange buffers of two fields, W_L^k (k < L), the two fold exchange
// buffers of two fields.
template <typename T, int L>
constexpr size_t k10_lds_bytes() {
  return (2 * 2 * (size_t)K2Geom<T>::template seqp<L>() + L + 2 * 2 * (size_t)L) * sizeof(V2<T>);
}

// The work of one block (unit `unit`); FOLD as for the single-block sweep.
template <typename T, int L, int NMAX, int KMAX, bool FOLD = true>
__device__ __forceinline__ void k10_body(const K10Args& a, int unit) {
  constexpr int P = k2_points(L);
  constexpr int TF2 = L / P;
  constexpr int FB = 2;  // fields per LDS round
  constexpr int SEQP = K2Geom<T>::template seqp<L>();
  using Lay = typename K2Geom<T>::template Layout<L>;
  static_assert(NMAX % FB == 0, "member bucket must be a multiple of the LDS batch");
  extern __shared__ unsigned char k10_lds_raw[];  // two buffers of FB fields, then W_L^k

  const V2<T>* __restrict__ tab = static_cast<const V2<T>*>(a.tab);
  const int C = a.C;
  const int tid = threadIdx.x;
  const int c = tid & (C - 1);
  const int t2 = tid / C;
  const int N = a.N, M = a.M, K = a.K, R = a.R, ny = a.ny;
  const int nxh = a.nx >> 1, nh = nxh + 1;
  const SpectralUnit<T> g = spectral_unit<T>(unit, c, C, R, L, ny, nxh, a.group_xcd);
  const int k2 = g.k2, kx = g.kx;
  const bool xlane = g.fold && g.col0;
  V2<T>* const region = static_cast<V2<T>*>(a.ws_main);
  const uint32_t fbytes = g.fstride * (uint32_t)sizeof(V2<T>);
  uint32_t voff[P];
#pragma unroll
  for (int i = 0; i < P; ++i) voff[i] = g.cbytes + (uint32_t)(t2 + TF2 * i) * g.sy * (uint32_t)sizeof(V2<T>);
  V2<T>* lds0 = reinterpret_cast<V2<T>*>(k10_lds_raw);
  LdsPair lp{lds0, lds0 + FB * SEQP, 0, c};
  const V2<T>* const tw = copy_twiddles<T, L>(lds0 + 2 * FB * SEQP, tab);
  V2<T>* const xch = lds0 + 2 * FB * SEQP + L;  // two buffers of FB x L, used in turn
  int xpar = 0;

  // field f through a buffer resource of its own (uniform base, 32-bit offsets)
  auto field_buf = [&](int f) __attribute__((always_inline)) -> Buf { return make_buf(region + (size_t)f * g.fstride, fbytes); };
  auto load_block = [&](int j, cx<T> (&v)[NMAX][P]) __attribute__((always_inline)) {
    static_for<0, NMAX>([&](auto F) __attribute__((always_inline)) {
      constexpr int k = decltype(F)::value;
      if (k < N) {
        const Buf b = field_buf(k * M + j);
#pragma unroll
        for (int i = 0; i < P; ++i) v[k][i] = from2<T>(buf_ld<T>(b, voff[i], 0u));
      } else {
#pragma unroll
        for (int i = 0; i < P; ++i) v[k][i] = cx<T>{T(0), T(0)};
      }
    });
  };
  auto forward = [&](cx<T> (&v)[NMAX][P]) __attribute__((always_inline)) {
#pragma unroll
    for (int f0 = 0; f0 < NMAX; f0 += FB) {
      if (f0 < N) {
        cx<T> blk[FB][P];
#pragma unroll
        for (int b = 0; b < FB; ++b)
#pragma unroll
          for (int i = 0; i < P; ++i) blk[b][i] = v[f0 + b][i];
        fft_forward<T, L, P, FB, SEQP, false, Lay, L>(blk, t2, lp, C, tw);
        if (FOLD && g.fold) fold_exchange<T, FB, FB, P, TF2, L>(blk, xch, xpar, t2, xlane, k2, true);
#pragma unroll
        for (int b = 0; b < FB; ++b)
#pragma unroll
          for (int i = 0; i < P; ++i) v[f0 + b][i] = blk[b][i];
      }
    }
  };
  // inverse transforms of one LDS round and the stores of block j
  auto inverse_store = [&](int j, int f0, cx<T> (&blk)[FB][P]) __attribute__((always_inline)) {
    if (FOLD && g.fold) fold_exchange<T, FB, FB, P, TF2, L>(blk, xch, xpar, t2, xlane, k2, false);
    fft_inverse<T, L, P, FB, SEQP, false, Lay, L>(blk, t2, lp, C, tw);
#pragma unroll
    for (int b = 0; b < FB; ++b)
      if (f0 + b < N) {
        const Buf bf = field_buf((f0 + b) * M + j);
#pragma unroll
        for (int i = 0; i < P; ++i) buf_st(bf, voff[i], 0u, to2<T>(blk[b][i]));
      }
  };

  const T n_tot = T(a.nx) * T(ny);
  const T invN = T(1) / T(N);
  const T var_scale = T(1) / (T(N - 1) * n_tot);  // unitary (eigenvalue) scale
  const T sqrt_n = sqrt_t<T>(n_tot);
  const T* __restrict__ Rspec = static_cast<const T*>(a.R_spec);
  const size_t plane = (size_t)ny * nh;

  // the bins of the thread's points: point i holds bin (bky(i), bkx(i)); a pair
  // slot only ever at points 0 and P/2
  const ColumnBins cb = column_bins(k2, kx, t2, R, L);
  const int kxt = cb.thr < 0 ? nxh : kx;  // outside a packed column, every point's kx
  auto bky = [&](int i) __attribute__((always_inline)) { return cb.kyb + R * (t2 + TF2 * i); };
  auto bkx = [&](int i) __attribute__((always_inline)) { return FOLD ? (t2 + TF2 * i > cb.thr ? nxh : kx) : kxt; };
  auto pr = [&](int i) __attribute__((always_inline)) {
    return FOLD && (i == 0 ? cb.pair0 : (i == P / 2 ? cb.pairh : false));
  };

  // e of members 2p and 2p + 1 for observed field o at point i (the bin's
  // counter word and scales are recomputed here rather than held in registers)
  auto draw = [&](int o, int p, int i, T amp_o, T amp_oi, cx<T>& e0, cx<T>& e1) __attribute__((always_inline)) {
    BinNoise<T> bn = bin_noise<T>(bkx(i), bky(i), nxh, ny);
    if (pr(i)) bn.zi = T(1);
    const u32x4 w = philox4x32_10(u32x4{bn.ctr0, (uint32_t)p, 0u, (uint32_t)o}, a.key0, a.key1);
    T rho, cs, sn;
    box_muller_parts<T>(w.x0, w.x1, rho, cs, sn);
    e0 = cx<T>{amp_o * bn.zs * (rho * cs), amp_oi * bn.zi * (rho * sn)};
    box_muller_parts<T>(w.x2, w.x3, rho, cs, sn);
    e1 = cx<T>{amp_o * bn.zs * (rho * cs), amp_oi * bn.zi * (rho * sn)};
  };

  // ---- observed blocks: deviations, eq. (2), their own update of eq. (3)
  cx<T> del[KMAX][NMAX][P];
  cx<T> dm[KMAX][P];
  T den[KMAX][P], amp[KMAX][P], deni[KMAX][P], ampi[KMAX][P];  // the ..i: a pair slot's imaginary part
  static_for<0, KMAX>([&](auto O) __attribute__((always_inline)) {
    constexpr int o = decltype(O)::value;
    if (o < K) {
      load_block(o, del[o]);
      {
        const Buf b = field_buf(N * M + o);
        cx<T> d1[1][P];
#pragma unroll
        for (int i = 0; i < P; ++i) d1[0][i] = from2<T>(buf_ld<T>(b, voff[i], 0u));
        forward(del[o]);
        fft_forward<T, L, P, 1, SEQP, false, Lay, L>(d1, t2, lp, C, tw);
        if (FOLD && g.fold) fold_exchange<T, 1, FB, P, TF2, L>(d1, xch, xpar, t2, xlane, k2, true);
#pragma unroll
        for (int i = 0; i < P; ++i) dm[o][i] = d1[0][i];
      }
      cx<T> mean[P];
      T gain[P], gaini[P];
#pragma unroll
      for (int i = 0; i < P; ++i) {
        // deviations formed from u_k - u_0 (exactly zero for a collapsed block)
        const cx<T> u0 = del[o][0][i];
        cx<T> ms{T(0), T(0)};
#pragma unroll
        for (int k = 1; k < NMAX; ++k)
          if (k < N) {
            del[o][k][i] = del[o][k][i] - u0;
            ms = ms + del[o][k][i];
          }
        del[o][0][i] = cx<T>{T(0), T(0)};
        ms = scale(ms, invN);
        T vr = T(0), vi = T(0);
#pragma unroll
        for (int k = 0; k < NMAX; ++k)
          if (k < N) {
            del[o][k][i] = del[o][k][i] - ms;
            vr += del[o][k][i].re * del[o][k][i].re;
            vi += del[o][k][i].im * del[o][k][i].im;
          }
        mean[i] = u0 + ms;
        dm[o][i] = dm[o][i] - mean[i];
        T coo = (vr + vi) * var_scale, cooi = coo;
        if (pr(i)) {
          coo = vr * var_scale;
          cooi = vi * var_scale;
        }
        T rb = T(a.r_obs[o]), rbi = rb;
        if (Rspec != nullptr) {
          const T* Ro = Rspec + (size_t)o * plane + (size_t)bky(i) * nh;
          rb = Ro[bkx(i)];
          rbi = pr(i) ? Ro[nxh] : rb;
        }
        den[o][i] = coo + rb;
        deni[o][i] = pr(i) ? cooi + rbi : den[o][i];
        gain[i] = den[o][i] < tiny_normal<T>() ? T(0) : coo / den[o][i];
        gaini[i] = pr(i) ? (deni[o][i] < tiny_normal<T>() ? T(0) : cooi / deni[o][i]) : gain[i];
        amp[o][i] = sqrt_n * sqrt_t<T>(rb);  // sqrt(n R_o)
        ampi[o][i] = pr(i) ? sqrt_n * sqrt_t<T>(rbi) : amp[o][i];
      }
      // the observed block's update: u + g (d - mean + e - delta), per LDS round
#pragma unroll
      for (int f0 = 0; f0 < NMAX; f0 += FB) {
        if (f0 < N) {
          cx<T> blk[FB][P];
#pragma unroll
          for (int i = 0; i < P; ++i) {
            cx<T> e0, e1;
            draw(o, f0 / 2, i, amp[o][i], ampi[o][i], e0, e1);
            const cx<T> x0 = dm[o][i] + e0 - del[o][f0][i], x1 = dm[o][i] + e1 - del[o][f0 + 1][i];
            blk[0][i] = mean[i] + del[o][f0][i] + cx<T>{x0.re * gain[i], x0.im * gaini[i]};
            blk[1][i] = mean[i] + del[o][f0 + 1][i] + cx<T>{x1.re * gain[i], x1.im * gaini[i]};
          }
          inverse_store(o, f0, blk);
        }
      }
    }
  });

  // ---- unobserved blocks through eq. (7): the K cross-covariances, the sum of
  // the K gain terms, the inverse
#pragma unroll 1
  for (int j = K; j < M; ++j) {
    cx<T> v[NMAX][P];
    load_block(j, v);
    forward(v);
    cx<T> G[KMAX][P];  // for a pair slot: the gains of its real and imaginary parts
#pragma unroll
    for (int i = 0; i < P; ++i) {
      // block j centred: its members relative to member 0, minus their mean
      const cx<T> v0 = v[0][i];
      cx<T> vm{T(0), T(0)};
#pragma unroll
      for (int k = 1; k < NMAX; ++k)
        if (k < N) vm = vm + (v[k][i] - v0);
      vm = scale(vm, invN);
      static_for<0, KMAX>([&](auto O) __attribute__((always_inline)) {
        constexpr int o = decltype(O)::value;
        // sum_k x_k conj(y_k) by its four real products: (rr + ii, ir - ri) for
        // a bin, (rr, ii) for a pair slot's two real bins
        T rr = T(0), ii = T(0), ir = T(0), ri = T(0);
        if (o < K) {
#pragma unroll
          for (int k = 0; k < NMAX; ++k)
            if (k < N) {
              const cx<T> x = (v[k][i] - v0) - vm, y = del[o][k][i];
              rr += x.re * y.re;
              ii += x.im * y.im;
              ir += x.im * y.re;
              ri += x.re * y.im;
            }
        }
        const cx<T> cj = pr(i) ? cx<T>{rr * var_scale, ii * var_scale}
                               : cx<T>{(rr + ii) * var_scale, (ir - ri) * var_scale};
        const bool none = !(o < K) || den[o][i] < tiny_normal<T>();
        const bool nonei = !(o < K) || deni[o][i] < tiny_normal<T>();
        const T gre = none ? T(0) : cj.re / den[o][i];
        G[o][i] = pr(i) ? cx<T>{gre, nonei ? T(0) : cj.im / deni[o][i]}
                        : cx<T>{gre, none ? T(0) : cj.im / den[o][i]};
      });
    }
#pragma unroll
    for (int f0 = 0; f0 < NMAX; f0 += FB) {
      if (f0 < N) {
        cx<T> blk[FB][P];
#pragma unroll
        for (int i = 0; i < P; ++i) {
          blk[0][i] = v[f0][i];
          blk[1][i] = v[f0 + 1][i];
          static_for<0, KMAX>([&](auto O) __attribute__((always_inline)) {
            constexpr int o = decltype(O)::value;
            if (o < K) {
              cx<T> e0, e1;
              draw(o, f0 / 2, i, amp[o][i], ampi[o][i], e0, e1);
              const cx<T> x0 = dm[o][i] + e0 - del[o][f0][i], x1 = dm[o][i] + e1 - del[o][f0 + 1][i];
              if (pr(i)) {  // two real bins: each part by its own gain
                blk[0][i] = blk[0][i] + cx<T>{G[o][i].re * x0.re, G[o][i].im * x0.im};
                blk[1][i] = blk[1][i] + cx<T>{G[o][i].re * x1.re, G[o][i].im * x1.im};
              } else {
                blk[0][i] = blk[0][i] + G[o][i] * x0;
                blk[1][i] = blk[1][i] + G[o][i] * x1;
              }
            }
          });
        }
        inverse_store(j, f0, blk);
      }
    }
  }
}

template <typename T, int L, int NMAX, int KMAX>
__global__ __launch_bounds__(k2_threads_target, (k10_waves<T, NMAX, KMAX>())) void k10_observed(const K10Args a) {
  if (unit_folds(blockIdx.x, a.C, a.R, a.nx >> 1, a.group_xcd))
    k10_body<T, L, NMAX, KMAX, true>(a, blockIdx.x);
  else
    k10_body<T, L, NMAX, KMAX, false>(a, blockIdx.x);
}

template <typename T, int L, int NMAX, int KMAX>
hipError_t launch_k10_shape(const K10Args& a, hipStream_t st) {
  constexpr int P = k2_points(L);
  const dim3 grid(a.units), block(a.C * (L / P));
  constexpr size_t lds_bytes = k10_lds_bytes<T, L>();
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&k10_observed<T, L, NMAX, KMAX>),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL((k10_observed<T, L, NMAX, KMAX>), grid, block, lds_bytes, st, a);
  return hipGetLastError();
}

}  // namespace fftenkf
