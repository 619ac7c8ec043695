// Multi-block spectral sweep (Section 2.2): the second sweep of an analysis
// whose members hold M blocks on one grid, block 0 observed.
//
// Units, thread layout, transforms and perturbations are those of the
// single-block sweep (k2_spectral.hpp).  Per bin, with delta_k = u_hat^(0)_k -
// mean^(0) the observed block's member deviations:
//   c_hat^(00) = 1/(N-1) sum_k |delta_k|^2                        (eq. (2))
//   c_hat^(j0) = 1/(N-1) sum_k (u_hat^(j)_k - mean^(j)) conj(delta_k)   (eq. (7),
//                the conjugate on the observed factor)
//   u_hat^(j)a_k = u_hat^(j)_k + c_hat^(j0) / (c_hat^(00) + R) (d_hat + e_hat_k - u_hat^(0)_k)   (eq. (6))
// with the innovation written d_hat - mean^(0) + e_hat_k - delta_k.  A unit
// keeps delta (N values per bin) and d_hat - mean^(0) in registers, and streams
// the blocks through a second register set: block 0 rebuilt from delta, then
// each block j loaded, transformed, updated, inverse transformed and stored.
// The perturbations are drawn again for every block from the same Philox
// counters, so no innovation is ever stored.
//
// Fields in the workspace: member k of block j is field k * M + j, d is field
// N * M (the member-major state vectors of the caller).
#pragma once

#include "k2_spectral.hpp"

namespace fftenkf {

// Two member sets per thread.  Buckets of up to 10 float members run two waves
// per SIMD (at 10 members that spills about 50 registers, and is still faster
// than one wave: 172 vs 185 us at 4 x 1024^2); larger buckets run one wave per
// SIMD with their registers spread over the unified file instead of spilling.
template <typename T, int NMAX>
constexpr int k6_waves() { return NMAX * (int)sizeof(T) <= 40 ? 2 : 1; }

template <typename T, int L, int NMAX>
__global__ __launch_bounds__(k2_threads_target, (k6_waves<T, NMAX>())) void k6_multiblock(const K6Args a) {
  constexpr int P = k2_points(L);
  constexpr int TF2 = L / P;
  constexpr int FB = 2;  // fields per LDS round
  constexpr int SEQP = K2Geom<T>::template seqp<L>();
  using Lay = typename K2Geom<T>::template Layout<L>;
  static_assert(NMAX % FB == 0, "member bucket must be a multiple of the LDS batch");
  extern __shared__ unsigned char k6_lds_raw[];  // two buffers of FB fields, then W_L^k

  const V2<T>* __restrict__ tab = static_cast<const V2<T>*>(a.tab);
  const int C = a.C;
  const int tid = threadIdx.x;
  const int c = tid & (C - 1);
  const int t2 = tid / C;
  const int N = a.N, M = a.M, R = a.R, ny = a.ny;
  const int nxh = a.nx >> 1, nh = nxh + 1;
  const SpectralUnit<T> g = spectral_unit<T>(a.ws_main, a.ws_nyq, blockIdx.x, c, C, C, R, L, ny, nxh, a.units_main,
                                             a.units_total, a.group_xcd);
  const int k2 = g.k2, kx = g.kx;
  uint32_t voff[P];
#pragma unroll
  for (int i = 0; i < P; ++i)
    voff[i] = ((uint32_t)(t2 + TF2 * i) * g.sy + (uint32_t)g.cc) * (uint32_t)sizeof(V2<T>);
  V2<T>* lds0 = reinterpret_cast<V2<T>*>(k6_lds_raw);
  LdsPair lp{lds0, lds0 + FB * SEQP, 0, c};
  // the twiddles (visible to all threads after the first exchange's barrier)
  const V2<T>* const tw = copy_twiddles<T, L>(lds0 + 2 * FB * SEQP, tab);

  auto field = [&](int f) -> V2<T>* { return g.ubase + (size_t)f * g.fstride; };
  // load the N members of block j (and zero the padding members)
  auto load_block = [&](int j, cx<T> (&v)[NMAX][P]) {
    static_for<0, NMAX>([&](auto F) {
      constexpr int k = decltype(F)::value;
      if (k < N) {
        const V2<T>* fb = field(k * M + j);
#pragma unroll
        for (int i = 0; i < P; ++i) v[k][i] = from2<T>(ld_off(fb, voff[i]));
      } else {
#pragma unroll
        for (int i = 0; i < P; ++i) v[k][i] = cx<T>{T(0), T(0)};
      }
    });
  };
  auto forward = [&](cx<T> (&v)[NMAX][P]) {
#pragma unroll
    for (int f0 = 0; f0 < NMAX; f0 += FB) {
      if (f0 < N) {
        cx<T> blk[FB][P];
#pragma unroll
        for (int b = 0; b < FB; ++b)
#pragma unroll
          for (int i = 0; i < P; ++i) blk[b][i] = v[f0 + b][i];
        fft_forward<T, L, P, FB, SEQP, false, Lay, L>(blk, t2, lp, C, tw);
#pragma unroll
        for (int b = 0; b < FB; ++b)
#pragma unroll
          for (int i = 0; i < P; ++i) v[f0 + b][i] = blk[b][i];
      }
    }
  };

  // ---- observed block and d: deviations, eq. (2), d_hat - mean
  cx<T> del[NMAX][P];
  cx<T> dm[1][P];
  load_block(0, del);
  {
    const V2<T>* fb = field(N * M);
#pragma unroll
    for (int i = 0; i < P; ++i) dm[0][i] = from2<T>(ld_off(fb, voff[i]));
  }
  forward(del);
  fft_forward<T, L, P, 1, SEQP, false, Lay, L>(dm, t2, lp, C, tw);

  const T n_tot = T(a.nx) * T(ny);
  const T invN = T(1) / T(N);
  const T var_scale = T(1) / (T(N - 1) * n_tot);  // unitary (eigenvalue) scale
  const T sqrt_n = sqrt_t<T>(n_tot);
  const T* __restrict__ Rspec = static_cast<const T*>(a.R_spec);
  cx<T> mean0[P];
  T c00[P], den[P], amp[P];
  bool none[P];  // c_hat^(00) + R below the smallest normal number: no update
  int ky[P];
#pragma unroll
  for (int i = 0; i < P; ++i) {
    ky[i] = k2 + R * (t2 + TF2 * i);
    // deviations formed from s_k = u_k - u_0 (exactly zero for a collapsed block)
    const cx<T> u0 = del[0][i];
    cx<T> mean{T(0), T(0)};
#pragma unroll
    for (int k = 1; k < NMAX; ++k)
      if (k < N) {
        del[k][i] = del[k][i] - u0;
        mean = mean + del[k][i];
      }
    del[0][i] = cx<T>{T(0), T(0)};
    mean = scale(mean, invN);
    T var = T(0);
#pragma unroll
    for (int k = 0; k < NMAX; ++k)
      if (k < N) {
        del[k][i] = del[k][i] - mean;
        var += del[k][i].re * del[k][i].re + del[k][i].im * del[k][i].im;
      }
    mean0[i] = u0 + mean;
    dm[0][i] = dm[0][i] - mean0[i];
    c00[i] = var * var_scale;
    T rb = T(a.r_scalar);
    if (Rspec != nullptr && g.valid) rb = Rspec[(size_t)ky[i] * nh + kx];
    den[i] = c00[i] + rb;
    none[i] = den[i] < tiny_normal<T>();
    amp[i] = sqrt_n * sqrt_t<T>(rb);  // sqrt(n R), without overflow of n R
  }

  // ---- every block: gain, update with the regenerated perturbations, inverse
  const bool edge = (kx == 0) || (kx == nxh);
  auto update_and_store = [&](int j, cx<T> (&v)[NMAX][P], const cx<T> (&G)[P]) __attribute__((always_inline)) {
    static_for<0, P>([&](auto I) __attribute__((always_inline)) {
      constexpr int i = decltype(I)::value;
      const bool mirrored = edge && ky[i] > (ny >> 1);
      const bool selfconj = edge && (ky[i] == 0 || ky[i] == (ny >> 1));
      const int gy = mirrored ? ny - ky[i] : ky[i];
      const uint32_t ctr0 = (uint32_t)(gy * nh + kx);
      const T zs = selfconj ? T(1) : T(0.70710678118654752440);
      const T zi = selfconj ? T(0) : (mirrored ? -zs : zs);
      static_for<0, (NMAX + 1) / 2>([&](auto PP) __attribute__((always_inline)) {
        constexpr int p = decltype(PP)::value;
        if (2 * p < N) {
          const u32x4 w = philox4x32_10(u32x4{ctr0, (uint32_t)p, 0u, 0u}, a.key0, a.key1);
          T za, zb;
          box_muller<T>(w.x0, w.x1, za, zb);
          const cx<T> e0{amp[i] * zs * za, amp[i] * zi * zb};
          v[2 * p][i] = v[2 * p][i] + G[i] * (dm[0][i] + e0 - del[2 * p][i]);
          if constexpr (2 * p + 1 < NMAX) {
            if (2 * p + 1 < N) {
              box_muller<T>(w.x2, w.x3, za, zb);
              const cx<T> e1{amp[i] * zs * za, amp[i] * zi * zb};
              v[2 * p + 1][i] = v[2 * p + 1][i] + G[i] * (dm[0][i] + e1 - del[2 * p + 1][i]);
            }
          }
        }
      });
    });
#pragma unroll
    for (int f0 = 0; f0 < NMAX; f0 += FB) {
      if (f0 < N) {
        cx<T> blk[FB][P];
#pragma unroll
        for (int b = 0; b < FB; ++b)
#pragma unroll
          for (int i = 0; i < P; ++i) blk[b][i] = v[f0 + b][i];
        fft_inverse<T, L, P, FB, SEQP, false, Lay, L>(blk, t2, lp, C, tw);
        if (g.valid) {
#pragma unroll
          for (int b = 0; b < FB; ++b)
            if (f0 + b < N) {
              V2<T>* fb = field((f0 + b) * M + j);
#pragma unroll
              for (int i = 0; i < P; ++i) st_off(fb, voff[i], to2<T>(blk[b][i]));
            }
        }
      }
    }
  };

  {  // the observed block: eq. (3) exactly as in the single-block sweep
    cx<T> v[NMAX][P], G[P];
#pragma unroll
    for (int k = 0; k < NMAX; ++k)
#pragma unroll
      for (int i = 0; i < P; ++i) v[k][i] = del[k][i] + mean0[i];
#pragma unroll
    for (int i = 0; i < P; ++i) G[i] = cx<T>{none[i] ? T(0) : c00[i] / den[i], T(0)};
    update_and_store(0, v, G);
  }
#pragma unroll 1
  for (int j = 1; j < M; ++j) {  // the other blocks, through eq. (7)
    cx<T> v[NMAX][P], G[P];
    load_block(j, v);
    forward(v);
#pragma unroll
    for (int i = 0; i < P; ++i) {
      // eq. (7) with both factors centred: block j's members relative to its
      // member 0, minus their mean (the deviations of block 0 sum to zero only
      // up to rounding, so block j is not left uncentred)
      const cx<T> v0 = v[0][i];
      cx<T> vm{T(0), T(0)};
#pragma unroll
      for (int k = 1; k < NMAX; ++k)
        if (k < N) vm = vm + (v[k][i] - v0);
      vm = scale(vm, invN);
      cx<T> s{T(0), T(0)};
#pragma unroll
      for (int k = 0; k < NMAX; ++k)
        if (k < N) s = s + ((v[k][i] - v0) - vm) * conj(del[k][i]);
      const cx<T> cj = scale(s, var_scale);
      G[i] = none[i] ? cx<T>{T(0), T(0)} : cx<T>{cj.re / den[i], cj.im / den[i]};
    }
    update_and_store(j, v, G);
  }
}

template <typename T, int L, int NMAX>
hipError_t launch_k6_shape(const K6Args& a, hipStream_t st) {
  constexpr int P = k2_points(L);
  const dim3 grid(a.units_total), block(a.C * (L / P));
  constexpr size_t lds_bytes = (2 * 2 * (size_t)K2Geom<T>::template seqp<L>() + L) * sizeof(V2<T>);
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&k6_multiblock<T, L, NMAX>),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL((k6_multiblock<T, L, NMAX>), grid, block, lds_bytes, st, a);
  return hipGetLastError();
}

}  // namespace fftenkf
