// Sweep 3: inverse radix-R stage of the y transform plus the inverse real x
// transform, the mirror image of sweep 1.
//
// For a tile (member f, y1) let U(k2, kx) = W_ny^(-y1 k2) B(k2, kx) / (nx ny),
// B the output of sweep 2.  The analysis member is the real part of the inverse
// 2D DFT of the Hermitian extension of the half spectrum (a c2r transform: the
// imaginary parts of the kx = 0 and kx = nx/2 entries are dropped).  Row
// y1 + L*y2 of it is
//   Re w_0(x) + (-1)^y2 Im w_0(x) + 2 Re sum_{0<j<R/2} W_R^(-y2 j) w_j(x),
// the unnormalised inverse real R-point DFT over j of (Re w_0, w_1, ..,
// w_{R/2-1}, Im w_0), where w_j is the inverse length-nx FFT of
//   Z_j(m) = U(j, m)                           0 < m < nx/2
//          = conj U(R-j, nx-m)                 nx/2 < m < nx
//          = (U(j, m) + conj U(R-j, m)) / 2    m in {0, nx/2}
// and w_0 that of H_0 + i H_{R/2}, H_j the Hermitian part of U(j, .).  The
// kx = 0 and kx = nx/2 entries are read from the folded column 0
// (spectral_unit.hpp): for a real result U(R-j, m) = conj U(j, m) there, so the
// m = 0 entry of row j is U(j, 0) and the m = nx/2 entry is the value folded
// into row R - j; rows 0 and R/2 hold both as real and imaginary parts.
#pragma once

#include "fft_core.hpp"
#include "k1_forward.hpp"
#include "kernels.hpp"

namespace fftenkf {

// The work of one block; `block` is its index within one analysis.
// SINE: row j1, x position j2 of the result goes to out(i1, i2) times
// (-1)^(i1 + i2), i = dst_rho(j) (the converse of sweep 1's reordering).
template <typename T, int NX, int R, int SB, bool SINE>
__device__ __forceinline__ void k3_body(const V2<T>* __restrict__ ws_main, int N, int ny, int L, T out_scale,
                                        T* __restrict__ out,
                                        const V2<T>* __restrict__ tab, int block) {
  using Geo = K1Geom<T, NX>;
  constexpr int P = Geo::P, TF = Geo::TF, G = Geo::G;
  constexpr int H = R / 2;
  constexpr int NXH = NX / 2;
  constexpr int SEQP = lds_padded_size(NX);
  __shared__ V2<T> lds[G * SB * SEQP];

  const int tid = threadIdx.x;
  const int g = tid / TF;
  const int t = tid - g * TF;
  const int tile = block * G + g;
  const bool active = tile < N * L;
  const int f = active ? tile / L : 0;
  const int y1 = active ? tile - f * L : 0;
  V2<T>* my = lds + g * SB * SEQP;
  LdsPair lp{my, nullptr, 0, 0};
  const size_t frow = (size_t)f * R;

  // twiddle (inverse) and normalisation for row k2
  auto tw = [&](int k2) -> cx<T> { return scale(conj(twiddle<T>(tab, y1 * k2, ny)), out_scale); };
  auto row = [&](int k2) -> const V2<T>* { return ws_main + ((frow + k2) * L + y1) * NXH; };

  // Every thread issues the same unconditional loads: element m of row j for
  // m < nx/2, element nx - m of row R - j above (at m = nx/2 that is an
  // in-bounds neighbour, replaced below).  The kx = 0 and kx = nx/2 entries
  // needed by the two special positions are tile-uniform loads; the special
  // cases are then plain selects.
  cx<T> s[H][P];
#pragma unroll
  for (int j = 1; j < H; ++j) {
    const cx<T> wj = tw(j), wc = tw(R - j);
    const V2<T>* __restrict__ rj = row(j);
    const V2<T>* __restrict__ rc = row(R - j);
    const cx<T> zero_m = wj * from2<T>(rj[0]);
    const cx<T> nyq_m = wj * from2<T>(rc[0]);
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int m = t + TF * i;
      cx<T> z;
      if (i < P / 2) {
        z = wj * from2<T>(rj[m]);
        if (i == 0) z = (t == 0) ? zero_m : z;
      } else {
        z = conj(wc * from2<T>(rc[NX - m]));
        if (i == P / 2) z = (t == 0) ? nyq_m : z;
      }
      s[j][i] = z;
    }
  }
  {
    const cx<T> w0 = tw(0), wh = tw(H);
    const V2<T>* __restrict__ r0 = row(0);
    const V2<T>* __restrict__ rh = row(H);
    const cx<T> p0 = w0 * from2<T>(r0[0]), ph = wh * from2<T>(rh[0]);  // packed
    const cx<T> zero_m{p0.re, ph.re};  // H_0 + i H_{R/2} at m = 0
    const cx<T> nyq_m{p0.im, ph.im};   // and at m = nx/2
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int m = t + TF * i;
      cx<T> z;
      if (i < P / 2) {
        z = w0 * from2<T>(r0[m]) + mul_pi(wh * from2<T>(rh[m]));
        if (i == 0) z = (t == 0) ? zero_m : z;
      } else {
        z = conj(w0 * from2<T>(r0[NX - m])) + mul_pi(conj(wh * from2<T>(rh[NX - m])));
        if (i == P / 2) z = (t == 0) ? nyq_m : z;
      }
      s[0][i] = z;
    }
  }

  // inverse length-NX FFTs
#pragma unroll
  for (int s0 = 0; s0 < H; s0 += SB) {
    cx<T> blk[SB][P];
#pragma unroll
    for (int b = 0; b < SB; ++b)
#pragma unroll
      for (int i = 0; i < P; ++i) blk[b][i] = s[s0 + b][i];
    fft_inverse<T, NX, P, SB, SEQP>(blk, t, lp, 1, tab);
#pragma unroll
    for (int b = 0; b < SB; ++b)
#pragma unroll
      for (int i = 0; i < P; ++i) s[s0 + b][i] = blk[b][i];
  }

  // inverse real R-point DFT over j, then the R output rows
  if (active) {
    T* __restrict__ dst = out + (size_t)f * ny * NX + t;
#pragma unroll
    for (int ii = 0; ii < P; ++ii) {
      // with SINE, points i and P - 1 - i in turn: the even output columns of
      // thread t and the odd ones of thread TF - 1 - t then share 128-byte lines
      // written one step apart, so the L2 merges the halves before write-back
      const int i = SINE ? ((ii & 1) ? P - 1 - (ii >> 1) : (ii >> 1)) : ii;
      cx<T> V[H + 1];
      V[0] = cx<T>{s[0][i].re, T(0)};
      V[H] = cx<T>{s[0][i].im, T(0)};
#pragma unroll
      for (int j = 1; j < H; ++j) V[j] = s[j][i];
      T col[R];
      irdft<T, R>(V, col);
      if constexpr (SINE) {
        // row j1 = y1 + L y2 goes to 2 j1 for y2 < R/2 and to 2 (ny - 1 - j1) + 1
        // above (R is even); column j2 = t + TF i likewise with i < P/2
        const int j2 = t + TF * i;
        const uint32_t i2 = (uint32_t)(i < P / 2 ? 2 * j2 : 2 * (NX - 1 - j2) + 1);
        const uint32_t step = 2u * (uint32_t)L * NX * (uint32_t)sizeof(T);
        const uint32_t even = (2u * (uint32_t)y1 * NX + i2) * (uint32_t)sizeof(T);
        const uint32_t odd = ((2u * (uint32_t)(ny - y1) - 1u) * NX + i2) * (uint32_t)sizeof(T);
        T* __restrict__ fo = out + (size_t)f * ny * NX;
#pragma unroll
        for (int y2 = 0; y2 < R; ++y2) {
          const T v = ((y2 >= R / 2) != (i >= P / 2)) ? -col[y2] : col[y2];
          st_off(fo, y2 < R / 2 ? even + (uint32_t)y2 * step : odd - (uint32_t)y2 * step, v);
        }
      } else {
#pragma unroll
        for (int y2 = 0; y2 < R; ++y2) dst[(size_t)(y1 + L * y2) * NX + TF * i] = col[y2];
      }
    }
  }
}

template <typename T, int NX, int R, int SB, bool SINE>
__global__ __launch_bounds__((K1Geom<T, NX>::threads), (SINE ? 2 : 1)) void k3_inverse(
    const V2<T>* __restrict__ ws_main, int N, int ny, int L, T out_scale, T* __restrict__ out,
    const V2<T>* __restrict__ tab) {
  k3_body<T, NX, R, SB, SINE>(ws_main, N, ny, L, out_scale, out, tab, blockIdx.x);
}

// A batch of analyses on one grid: blockIdx.y selects the analysis.
template <typename T, int NX, int R, int SB>
__global__ __launch_bounds__((K1Geom<T, NX>::threads)) void k3_inverse_batch(const BatchArgs b) {
  const BatchFilter& f = b.f[blockIdx.y];
  k3_body<T, NX, R, SB, false>(static_cast<const V2<T>*>(f.ws_main), b.N, b.ny, b.L, T(1) / (T(b.nx) * T(b.ny)),
                               static_cast<T*>(f.out), static_cast<const V2<T>*>(b.tab), blockIdx.x);
}

template <typename T, int NX, int R>
hipError_t launch_k3_batch_shape(const BatchArgs& b, hipStream_t st) {
  using Geo = K1Geom<T, NX>;
  const int tiles = b.N * b.L;
  const dim3 grid((tiles + Geo::G - 1) / Geo::G, b.count), block(Geo::threads);
  hipLaunchKernelGGL((k3_inverse_batch<T, NX, R, k1_sb<T, NX, R>()>), grid, block, 0, st, b);
  return hipGetLastError();
}

template <typename T, int NX, int R>
hipError_t launch_k3_shape(const K3Args& a, hipStream_t st) {
  using Geo = K1Geom<T, NX>;
  constexpr int SB = k1_sb<T, NX, R>();
  const int tiles = a.N * a.L;
  const dim3 grid((tiles + Geo::G - 1) / Geo::G), block(Geo::threads);
  const T out_scale = T(1) / (T(a.nx) * T(a.ny));
  if (a.sine)
    hipLaunchKernelGGL((k3_inverse<T, NX, R, SB, true>), grid, block, 0, st, static_cast<const V2<T>*>(a.ws_main),
                       a.N, a.ny, a.L, out_scale, static_cast<T*>(a.out), static_cast<const V2<T>*>(a.tab));
  else
    hipLaunchKernelGGL((k3_inverse<T, NX, R, SB, false>), grid, block, 0, st, static_cast<const V2<T>*>(a.ws_main),
                       a.N, a.ny, a.L, out_scale, static_cast<T*>(a.out), static_cast<const V2<T>*>(a.tab));
  return hipGetLastError();
}

}  // namespace fftenkf
