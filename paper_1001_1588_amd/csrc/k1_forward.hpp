// Sweep 1: forward x transform plus the radix-R stage of the y transform.
//
// One tile = one field f (member or data) and one y1 < L: the R rows
// y1 + L*y2.  Each thread owns the x positions {t + TF*i}: it loads the R rows
// there (coalesced across threads), does the real R-point DFT over y2 in
// registers, and obtains R/2 complex sequences along x:
//   S_0 = V_0 + i V_{R/2}   (both real sequences),   S_j = V_j  (0 < j < R/2).
// Their length-nx FFTs give every output: for 0 < j < R/2,
//   A[j](kx)   = W_ny^(y1 j)     * S_j^(kx)            (0 <= kx <= nx/2)
//   A[R-j](kx) = W_ny^(y1 (R-j)) * conj(S_j^(nx - kx))  (V_{R-j} = conj(V_j))
// and S_0^ is split into V_0^ and V_{R/2}^ by Hermitian symmetry.  The kx = 0
// and kx = nx/2 outputs are written folded (spectral_unit.hpp): row j < R/2
// keeps A[j](0) in column 0, row R - j takes A[j](nx/2) there, and rows 0 and
// R/2 take A[j](0) + i A[j](nx/2).
#pragma once

#include "fft_core.hpp"
#include "kernels.hpp"

namespace fftenkf {

template <typename T, int NX>
struct K1Geom {
  static constexpr int P = NX < 8 ? NX : 8;
  static constexpr int TF = NX / P;
  static constexpr int G = TF >= 64 ? 1 : 64 / TF;  // tiles per block
  static constexpr int threads = TF * G;
};

// The work of one block; `block` is its index within one analysis.
// SINE: the fields enter through the sine-basis reordering v(j1, j2) =
// (-1)^(i1 + i2) x(i1, i2), i = dst_rho(j): row j1 reads row i1, and the
// thread's x position j2 reads x(2 j2) for j2 < NX/2, -x(2 (NX - 1 - j2) + 1) above.
template <typename T, int NX, int R, int SB, bool SINE>
__device__ __forceinline__ void k1_body(const T* __restrict__ members, const T* __restrict__ data, int N, int ny,
                                        int L, V2<T>* __restrict__ ws_main, const V2<T>* __restrict__ tab,
                                        unsigned block, int n_data = 1) {
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
  const bool active = tile < (N + n_data) * L;
  const int f = active ? tile / L : 0;
  const int y1 = active ? tile - f * L : 0;
  const T* __restrict__ src = (f < N) ? members + (size_t)f * ny * NX : data + (size_t)(f - N) * ny * NX;
  V2<T>* my = lds + g * SB * SEQP;
  LdsPair lp{my, nullptr, 0, 0};

  // 1. the R rows at this thread's x positions (read once: streaming loads)
  T a[R][P];
#pragma unroll
  for (int y2 = 0; y2 < R; ++y2) {
    if constexpr (SINE) {
      // j1 = y1 + L y2 < ny/2 exactly when y2 < R/2 (R is even): row 2 j1, else
      // 2 (ny - 1 - j1) + 1; likewise j2 = t + TF i < NX/2 exactly when i < P/2.
      // The signs are therefore constants.
      const uint32_t step = 2u * (uint32_t)L * NX * (uint32_t)sizeof(T);
      const uint32_t rowoff = y2 < R / 2 ? (2u * (uint32_t)y1 * NX) * (uint32_t)sizeof(T) + (uint32_t)y2 * step
                                         : ((2u * (uint32_t)(ny - y1) - 1u) * NX) * (uint32_t)sizeof(T) - (uint32_t)y2 * step;
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const int j2 = t + TF * i;
        const uint32_t i2 = (uint32_t)(i < P / 2 ? 2 * j2 : 2 * (NX - 1 - j2) + 1);
        const T x = active ? ld_stream(reinterpret_cast<const T*>(reinterpret_cast<const char*>(src) + rowoff +
                                                                   i2 * (uint32_t)sizeof(T)))
                           : T(0);
        a[y2][i] = ((y2 >= R / 2) != (i >= P / 2)) ? -x : x;
      }
    } else {
      const T* __restrict__ row = src + (size_t)(y1 + L * y2) * NX + t;
#pragma unroll
      for (int i = 0; i < P; ++i) a[y2][i] = active ? ld_stream(row + TF * i) : T(0);
    }
  }

  // 2. real R-point DFT over y2, packed into R/2 complex sequences
  cx<T> s[H][P];
#pragma unroll
  for (int i = 0; i < P; ++i) {
    T col[R];
#pragma unroll
    for (int y2 = 0; y2 < R; ++y2) col[y2] = a[y2][i];
    cx<T> V[H + 1];
    rdft<T, R>(col, V);
    s[0][i] = cx<T>{V[0].re, V[H].re};
#pragma unroll
    for (int j = 1; j < H; ++j) s[j][i] = V[j];
  }

  // 3. length-NX FFT of each sequence, SB sequences per LDS round
#pragma unroll
  for (int s0 = 0; s0 < H; s0 += SB) {
    cx<T> blk[SB][P];
#pragma unroll
    for (int b = 0; b < SB; ++b)
#pragma unroll
      for (int i = 0; i < P; ++i) blk[b][i] = s[s0 + b][i];
    fft_forward<T, NX, P, SB, SEQP>(blk, t, lp, 1, tab);
#pragma unroll
    for (int b = 0; b < SB; ++b)
#pragma unroll
      for (int i = 0; i < P; ++i) s[s0 + b][i] = blk[b][i];
  }

  const size_t frow = (size_t)f * R;

  // 4. sequences 0 < j < R/2 give rows j and R - j directly; column 0 of row
  // R - j takes A[j](nx/2) (m = nx/2 is this thread's point P/2 when t = 0)
#pragma unroll
  for (int j = 1; j < H; ++j) {
    const cx<T> wj = twiddle<T>(tab, y1 * j, ny);
    const cx<T> wc = twiddle<T>(tab, y1 * (R - j), ny);
    V2<T>* __restrict__ rowj = ws_main + ((frow + j) * L + y1) * NXH;
    V2<T>* __restrict__ rowc = ws_main + ((frow + (R - j)) * L + y1) * NXH;
    if (active) {
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const int m = t + TF * i;
        const cx<T> val = s[j][i];
        if (i < P / 2) {
          rowj[m] = to2<T>(wj * val);
          if (m == 0) rowc[0] = to2<T>(wj * s[j][P / 2]);
        } else if (m != NXH) {
          rowc[NX - m] = to2<T>(wc * conj(val));
        }
      }
    }
  }

  // 5. sequence 0: V_0^(m) = (S(m) + conj S(-m)) / 2, V_{R/2}^(m) = (S(m) - conj S(-m)) / 2i
#pragma unroll
  for (int i = 0; i < P; ++i) my[lds_pad(t + TF * i)] = to2<T>(s[0][i]);
  lds_barrier();
  if (active) {
    const cx<T> wh = twiddle<T>(tab, y1 * H, ny);
    V2<T>* __restrict__ row0 = ws_main + ((frow + 0) * L + y1) * NXH;
    V2<T>* __restrict__ rowh = ws_main + ((frow + H) * L + y1) * NXH;
#pragma unroll
    for (int i = 0; i < P / 2; ++i) {
      const int m = t + TF * i;
      const cx<T> z = from2<T>(my[lds_pad(m)]);
      const cx<T> zc = conj(from2<T>(my[lds_pad((NX - m) & (NX - 1))]));
      cx<T> v0 = scale(z + zc, T(0.5));
      cx<T> vh = scale(mul_mi(z - zc), T(0.5));
      if (m == 0) {
        // real V_0^ and V_{R/2}^ at m = 0 and m = nx/2, packed
        const cx<T> zn = from2<T>(my[lds_pad(NXH)]);
        v0 = cx<T>{z.re, zn.re};
        vh = cx<T>{z.im, zn.im};
      }
      row0[m] = to2<T>(v0);
      rowh[m] = to2<T>(wh * vh);
    }
  }
}

template <typename T, int NX, int R, int SB, bool SINE>
__global__ __launch_bounds__((K1Geom<T, NX>::threads)) void k1_forward(
    const T* __restrict__ members, const T* __restrict__ data, int N, int ny, int L,
    V2<T>* __restrict__ ws_main, const V2<T>* __restrict__ tab, int n_data) {
  k1_body<T, NX, R, SB, SINE>(members, data, N, ny, L, ws_main, tab, blockIdx.x, n_data);
}

// A batch of analyses on one grid: blockIdx.y selects the analysis.
template <typename T, int NX, int R, int SB>
__global__ __launch_bounds__((K1Geom<T, NX>::threads)) void k1_forward_batch(const BatchArgs b) {
  const BatchFilter& f = b.f[blockIdx.y];
  k1_body<T, NX, R, SB, false>(static_cast<const T*>(f.members), static_cast<const T*>(f.data), b.N, b.ny, b.L,
                        static_cast<V2<T>*>(f.ws_main), static_cast<const V2<T>*>(b.tab), blockIdx.x);
}

template <typename T, int NX, int R>
constexpr int k1_sb() {
  // sequences per LDS round: keep the (padded) buffer within 80 KB so two
  // blocks share a CU
  constexpr int budget = 81920 / (K1Geom<T, NX>::G * lds_padded_size(NX) * (int)sizeof(V2<T>));
  return budget >= R / 2 ? R / 2 : budget >= 4 ? 4 : budget >= 2 ? 2 : 1;
}

template <typename T, int NX, int R>
hipError_t launch_k1_batch_shape(const BatchArgs& b, hipStream_t st) {
  using Geo = K1Geom<T, NX>;
  const int tiles = (b.N + 1) * b.L;
  const dim3 grid((tiles + Geo::G - 1) / Geo::G, b.count), block(Geo::threads);
  hipLaunchKernelGGL((k1_forward_batch<T, NX, R, k1_sb<T, NX, R>()>), grid, block, 0, st, b);
  return hipGetLastError();
}

template <typename T, int NX, int R>
hipError_t launch_k1_shape(const K1Args& a, hipStream_t st) {
  using Geo = K1Geom<T, NX>;
  constexpr int SB = k1_sb<T, NX, R>();
  const int tiles = (a.N + a.n_data) * a.L;
  const dim3 grid((tiles + Geo::G - 1) / Geo::G), block(Geo::threads);
  if (a.sine)
    hipLaunchKernelGGL((k1_forward<T, NX, R, SB, true>), grid, block, 0, st, static_cast<const T*>(a.members),
                       static_cast<const T*>(a.data), a.N, a.ny, a.L, static_cast<V2<T>*>(a.ws_main),
                       static_cast<const V2<T>*>(a.tab), a.n_data);
  else
    hipLaunchKernelGGL((k1_forward<T, NX, R, SB, false>), grid, block, 0, st, static_cast<const T*>(a.members),
                       static_cast<const T*>(a.data), a.N, a.ny, a.L, static_cast<V2<T>*>(a.ws_main),
                       static_cast<const V2<T>*>(a.tab), a.n_data);
  return hipGetLastError();
}

}  // namespace fftenkf
