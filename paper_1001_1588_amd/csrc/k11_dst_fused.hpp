// The analysis in the real sine basis (Section 4) as one spectral sweep: the
// length-L transforms, eq. (2)-(3) on the sine coefficients and the inverse
// transforms in one pass, between sweeps 1 and 3 (which read and write the
// fields through the reordering of k9_dst.hip).
//
// A sine coefficient X at (k1, k2) is formed from the DFT V of the reordered
// field at (k1, k2) and at (k1, -k2) = conj V(-k1, k2), so the mirror rows ky
// and -ky of one column must meet.  With ky = k2 + R k1 (k2 the row of the
// radix-R stage, k1 the bin of the length-L transform) the mirror of row k2 is
// row R - k2 at bin L - 1 - k1.  A block therefore takes CH columns of row
// rA = k2 (lanes c < CH) and the same columns of rB = R - k2 (lanes c >= CH),
// for k2 = 0 .. R/2; the rB lanes load element (L - y1) mod L times W_L^y1
// (without the twiddle for k2 = 0), so that after the common length-L
// transform the lane CH to the right of a bin holds its mirror -ky at the same
// point index.  Thread (c, t2) holds points y1, k1 = t2 + TF2 i as in the
// single-block sweep; every exchange between mirror bins is a shuffle of lanes
// c and c ^ CH inside one wave.  Rows 0 and R/2 are their own mirrors: their
// rB lanes hold a reversed copy, take part, and store nothing.
//
// Per bin (ky, kx) with 0 < kx < nx/2 a lane turns V and the mirror's V into
// the two coefficients X(ky, kx) and X(ky, -kx); the kx = 0 column (folded:
// kx = 0 bins in rows below R/2, kx = nx/2 bins in rows above, both packed in
// rows 0 and R/2, spectral_unit.hpp) gives per slot X(ky, kc) and X(-ky, kc),
// kc in {0, nx/2}, from the slot alone, after the packed rows are split through
// the same shuffle.  Eq. (2) and the update of eq. (3) then run per
// coefficient, as in k9_dst.hip (alpha^2 var(X), X + g (X_d - X) +
// (g sqrt(R_dst) / alpha) z), and the inverse conversion
//   V(k1, k2) = conj(W1(k1) W2(k2)) [X(k1, k2) - X(-k1, -k2) - i (X(-k1, k2) + X(k1, -k2))]
// (X = 0 at index n) takes the mirror's two updated coefficients by one more
// shuffle.  Shapes: L >= 16 (the mirror lane is in the same wave) and nx/2 a
// multiple of CH = 512 / L; others run the launches of k9_dst.hip.
#pragma once

#include "k2_spectral.hpp"

namespace fftenkf {

// W(k) = exp(-i pi k / (2n)) for 0 <= k < n, given inv2n = 1 / (2n) (exact:
// n is a power of two)
template <typename T>
__device__ __forceinline__ cx<T> dst_w(int k, T inv2n);
template <>
__device__ __forceinline__ cx<float> dst_w<float>(int k, float inv2n) {
  float s, c;
  sincospif((float)k * inv2n, &s, &c);
  return cx<float>{c, -s};
}
template <>
__device__ __forceinline__ cx<double> dst_w<double>(int k, double inv2n) {
  double s, c;
  sincospi((double)k * inv2n, &s, &c);
  return cx<double>{c, -s};
}

template <typename T>
__device__ __forceinline__ T lane_xor(T v, int m) {
  return __shfl_xor(v, m);
}
template <typename T>
__device__ __forceinline__ cx<T> lane_xor(cx<T> v, int m) {
  return cx<T>{__shfl_xor(v.re, m), __shfl_xor(v.im, m)};
}

constexpr int k11_min_L = 16;
#ifndef K11_THREADS
#define K11_THREADS 256
#endif
constexpr int k11_threads = K11_THREADS;

// Columns per half of a block for a transform length L (four points per thread).
__host__ __device__ constexpr int k11_half_cols(int L) { return k11_threads * 4 / L / 2; }

// LDS: two exchange buffers of fb() fields over the block's C = 2 CH columns
// (swizzled rows), then W_L^k
template <typename T, int L, int NMAX>
constexpr size_t k11_lds_bytes() {
  return (2 * (size_t)K2Geom<T>::template fb<NMAX>() * (size_t)(2 * k11_half_cols(L)) * L + L) * sizeof(V2<T>);
}

// COL0: the block holds column kx = 0 (the first chunk of a row pair); the
// other blocks run a body without the kx = 0 slots' code.
template <typename T, int L, int NMAX, bool COL0>
__device__ __forceinline__ void k11_body(const K9Args& a, int k2, int q) {
  constexpr int P = 4;
  constexpr int TF2 = L / P;
  constexpr int C = k11_threads / TF2;
  constexpr int CH = C / 2;
  constexpr int FB = K2Geom<T>::template fb<NMAX>();
  using Lay = SwizzleLayout<C, (int)sizeof(V2<T>)>;
  constexpr int SEQP = Lay::elems(L);
  static_assert(L >= k11_min_L && CH >= 1 && CH <= 32, "mirror lanes must share a wave");
  static_assert(NMAX % 4 == 0 && NMAX % FB == 0, "member bucket");
  // float32 length-64 and length-128 transforms in the wave (wave_fft.hpp:
  // 1024 / L columns, the bins of a thread at wave_fft_bin); the mirror lanes
  // hold the same permutation, so a bin's mirror stays in the lane CH away
  constexpr bool WF = std::is_same<T, float>::value && wave_fft_length<L>() && C == 1024 / L;
  extern __shared__ unsigned char k11_lds_raw[];

  const V2<T>* __restrict__ tab = static_cast<const V2<T>*>(a.tab);
  const int tid = threadIdx.x;
  const int c = tid % C, t2 = tid / C;
  const int R = a.R, H = R >> 1, ny = a.ny, nx = a.nx, nxh = nx >> 1, N = a.N;
  const bool hb = c >= CH;                   // a lane of the mirror row
  const int kx = q * CH + (c & (CH - 1));
  const int row = hb ? (R - k2) % R : k2;
  const bool self = k2 == 0 || k2 == H;      // the block's two rows are one
  const bool stores = !(hb && self);
  const bool col0 = COL0 && kx == 0;
  const bool twist = hb && k2 != 0;          // mirror rows transform x(-y1) W_L^y1

  // loads: element y1 (a) or (L - y1) mod L (b) of row `row`, column kx
  const uint32_t fbytes = (uint32_t)ny * (uint32_t)nxh * (uint32_t)sizeof(V2<T>);
  const Buf buf = make_buf(a.ws_main, a.main_bytes);
  V2<T>* lds0 = reinterpret_cast<V2<T>*>(k11_lds_raw);
  LdsPair lp{lds0, lds0 + FB * SEQP, 0, c};
  const V2<T>* const tw = copy_twiddles<T, L>(lds0 + 2 * FB * SEQP, tab);
  uint32_t voff[P];
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const int y1 = t2 + TF2 * i;
    const int yl = hb ? (L - y1) & (L - 1) : y1;
    voff[i] = (uint32_t)(((size_t)row * L + yl) * nxh + kx) * (uint32_t)sizeof(V2<T>);
  }
  // W_L^y1 of the mirror rows, from the block's LDS copy of W_L^k: applied to
  // each LDS round's fields just before their forward transforms and after
  // their inverse ones (read per round rather than kept in registers; a read
  // from the device table would wait behind every load and store in flight)
  auto tw_y = [&](int i) __attribute__((always_inline)) -> cx<T> {
    return twist ? from2<T>(tw[t2 + TF2 * i]) : cx<T>{T(1), T(0)};
  };

  cx<T> u[NMAX + 1][P];  // members, then d (field N is read into slot NMAX)
  static_for<0, NMAX + 1>([&](auto F) __attribute__((always_inline)) {
    constexpr int f = decltype(F)::value;
    const int fld = f == NMAX ? N : f;
    if (f == NMAX || f < N) {
#pragma unroll
      for (int i = 0; i < P; ++i) u[f][i] = from2<T>(buf_ld<T>(buf, voff[i], (uint32_t)fld * fbytes));
    } else {
#pragma unroll
      for (int i = 0; i < P; ++i) u[f][i] = cx<T>{T(0), T(0)};
    }
  });

  // the bins of the thread's points: X.re at (kr, kc), X.im at (kr, -kc)
  // (0 < kx < nx/2) or at (-kr, kc) (the kx = 0 slot)
  // (formed where used rather than kept in registers)
  const int n1 = ny, n2 = nx;
  auto kr_at = [&](int i) __attribute__((always_inline)) -> int {
    const int k1 = WF ? wave_fft_bin<L>(t2, i) : t2 + TF2 * i;
    const int kyA = k2 + R * k1;
    if (!col0) return hb ? (n1 - kyA) & (n1 - 1) : kyA;
    if (self) return kyA;                           // the split gives a the kx = 0 bin, b the kx = nx/2 bin
    return hb ? (k2 + R * (L - 1 - k1)) : kyA;      // b: the folded kx = nx/2 sequence of row k2
  };
  const int kc0 = col0 ? (hb ? nxh : 0) : kx;  // the column of X.re

  // The twiddles of a phase, per point: wp = W1(kr) W2(kc) and wm = W1(kr)
  // conj W2(kc), W2(kc) of a kx = 0 slot being 1 or exp(-i pi/4).  Formed once
  // per phase rather than kept in registers.
  const T inv2n1 = T(1) / T(2 * n1), inv2n2 = T(1) / T(2 * n2);
  auto phase_w = [&](cx<T> (&wp)[P], cx<T> (&wm)[P]) __attribute__((always_inline)) {
    const T h = T(0.70710678118654752440);
    const cx<T> w2 = col0 ? (hb ? cx<T>{h, -h} : cx<T>{T(1), T(0)}) : dst_w<T>(kx, inv2n2);
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const cx<T> w1 = dst_w<T>(kr_at(i), inv2n1);
      wp[i] = w1 * w2;
      wm[i] = w1 * conj(w2);
    }
  };

  // V -> X for one field at point i (own value v, the mirror lane's value w).
  // With A = W1 W2 v and B = W1 conj(W2) conj(w) (V(kr, -kx) = conj w,
  // W2(-kx) = -i conj W2(kx)): X(kr, kx) = Re(A + B) / 2, X(kr, -kx) = Im(B - A) / 2.
  // A kx = 0 slot s (V(-kr, kc) = conj s, W1(-kr) = -i conj W1(kr), X at index
  // n1 is 0): X(kr, kc) = Re W2 Re(W1 s) and X(-kr, kc) = -Re W2 Im(W1 s); with
  // q = W1 W2 s that is q at kc = 0 (W2 = 1), and (q.re - q.im, q.re + q.im) / 2
  // at kc = nx/2 (W2 = (1 - i) / sqrt 2).
  auto to_x = [&](int i, cx<T> v, cx<T> w, const cx<T>(&wp)[P], const cx<T>(&wm)[P]) __attribute__((always_inline)) -> cx<T> {
    if (!col0) {
      const cx<T> A = wp[i] * v, B = wm[i] * conj(w);
      return cx<T>{T(0.5) * (A.re + B.re), T(0.5) * (B.im - A.im)};
    }
    cx<T> s = v;
    if (self)  // split the packed slot: a F_0 = (Z + conj Z(m)) / 2, b F_n = (Z - conj Z(m)) / 2i
      s = hb ? scale(mul_mi(w - conj(v)), T(0.5)) : scale(v + conj(w), T(0.5));
    const cx<T> qv = wp[i] * s;
    const cx<T> g = hb ? cx<T>{T(0.5) * (qv.re - qv.im), T(0.5) * (qv.re + qv.im)} : qv;  // Re W2 (W1 s)
    return cx<T>{g.re, kr_at(i) == 0 ? T(0) : -g.im};
  };

  // forward transforms (the mirror rows twisted first), then the coefficients
  // of every field.  tw is read only after the first round's barrier.
  cx<T> wpf[P], wmf[P];
  phase_w(wpf, wmf);
  lds_barrier();  // the LDS twiddles are visible
  auto fwd = [&](auto& blk) __attribute__((always_inline)) {
    constexpr int FB2 = sizeof(blk) / sizeof(blk[0]);
    if constexpr (WF) {
      wave_fft_forward<L, FB2>(blk, reinterpret_cast<const V2<float>*>(tw),
                               reinterpret_cast<V2<float>*>(lp.parity ? lp.buf1 : lp.buf0), t2, c);
      lp.parity ^= 1;
    } else {
      fft_forward<T, L, P, FB2, SEQP, false, Lay, L>(blk, t2, lp, C, tw);
    }
  };
  static_for<0, NMAX, FB>([&](auto F0) __attribute__((always_inline)) {
    constexpr int f0 = decltype(F0)::value;
    if (f0 < N) {
      cx<T> blk[FB][P];
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const cx<T> t = tw_y(i);
#pragma unroll
        for (int b = 0; b < FB; ++b) blk[b][i] = u[f0 + b][i] * t;
      }
      fwd(blk);
#pragma unroll
      for (int b = 0; b < FB; ++b)
#pragma unroll
        for (int i = 0; i < P; ++i) u[f0 + b][i] = to_x(i, blk[b][i], lane_xor(blk[b][i], CH), wpf, wmf);
    }
  });
  {
    cx<T> dv[1][P];
#pragma unroll
    for (int i = 0; i < P; ++i) dv[0][i] = u[NMAX][i] * tw_y(i);
    fwd(dv);
#pragma unroll
    for (int i = 0; i < P; ++i) u[NMAX][i] = to_x(i, dv[0][i], lane_xor(dv[0][i], CH), wpf, wmf);
  }

  // ---- eq. (2)-(3) per coefficient, all members of a point at once
  const T* __restrict__ Rd = static_cast<const T*>(a.R_dst);
  const T invN = T(1) / T(N), invN1 = T(1) / T(N - 1);
  const T sa1 = sqrt_t<T>(T(1) / T(n1)), sb1 = sqrt_t<T>(T(2) / T(n1));
  const T sa2 = sqrt_t<T>(T(1) / T(n2)), sb2 = sqrt_t<T>(T(2) / T(n2));
  static_for<0, P>([&](auto I) __attribute__((always_inline)) {
    constexpr int i = decltype(I)::value;
    static_for<0, 2>([&](auto W) __attribute__((always_inline)) {
      constexpr int which = decltype(W)::value;  // 0: X.re, 1: X.im
      const int kri = kr_at(i);
      int p1, p2;  // the coefficient's indices
      if (!col0) {
        p1 = kri;
        p2 = which == 0 ? kx : n2 - kx;
      } else {
        p1 = which == 0 ? kri : n1 - kri;
        p2 = kc0;
      }
      const bool live = !(col0 && which == 1 && kri == 0);  // X at index n1 is not a coefficient
      const T alpha = (p1 == 0 ? sa1 : sb1) * (p2 == 0 ? sa2 : sb2);
      const int s1 = n1 - 1 - p1, s2 = n2 - 1 - p2;
      auto xr = [&](int f) __attribute__((always_inline)) -> T& { return which == 0 ? u[f][i].re : u[f][i].im; };
      // deviations formed from X_f - X_0 (exactly zero for a collapsed ensemble)
      const T x0 = xr(0);
      T mean = T(0);
#pragma unroll
      for (int f = 1; f < NMAX; ++f)
        if (f < N) mean += xr(f) - x0;
      mean *= invN;
      T var = mean * mean;
#pragma unroll
      for (int f = 1; f < NMAX; ++f)
        if (f < N) var += ((xr(f) - x0) - mean) * ((xr(f) - x0) - mean);
      const T cv = alpha * alpha * var * invN1;
      const T r = Rd != nullptr ? Rd[(size_t)s1 * n2 + s2] : T(a.r_scalar);
      const T den = cv + r;
      const T g = (den < tiny_normal<T>() || !live) ? T(0) : cv / den;
      const T ge = live ? g * sqrt_t<T>(r) / alpha : T(0);
      const T xd = xr(NMAX);
      const uint32_t ctr0 = (uint32_t)(s1 * n2 + s2);
      static_for<0, NMAX / 4>([&](auto QI) __attribute__((always_inline)) {
        constexpr int qq = decltype(QI)::value;
        if (4 * qq < N) {
          const u32x4 wd = philox4x32_10(u32x4{ctr0, (uint32_t)qq, 1u, 0u}, a.key0, a.key1);
          T z[4];
          box_muller<T>(wd.x0, wd.x1, z[0], z[1]);
          box_muller<T>(wd.x2, wd.x3, z[2], z[3]);
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (4 * qq + j < N) xr(4 * qq + j) += g * (xd - xr(4 * qq + j)) + ge * z[j];
        }
      });
    });
  });

  // X -> V at point i from the thread's coefficients x and the mirror lane's m
  auto from_x = [&](int i, cx<T> x, cx<T> m, const cx<T>(&wp)[P]) __attribute__((always_inline)) -> cx<T> {
    const cx<T> cw = conj(wp[i]);  // conj(W1(kr) W2(kc))
    if (!col0) {
      // X(kr,kx) = x.re, X(kr,-kx) = x.im, X(-kr,kx) = m.re, X(-kr,-kx) = m.im (0 at index n1)
      const bool edge = kr_at(i) == 0;
      const T mr = edge ? T(0) : m.re, mi = edge ? T(0) : m.im;
      return cw * cx<T>{x.re - mi, -(mr + x.im)};
    }
    // X(kr, kc) = x.re, X(-kr, kc) = x.im (0 at index n1); X(., -kc) is X(., kc) at
    // kc = nx/2 and 0 (index n2) at kc = 0
    const T xm = kc0 == 0 ? T(0) : x.im, xc = kc0 == 0 ? T(0) : x.re;
    return cw * cx<T>{x.re - xm, -(x.im + xc)};
  };

  // ---- per LDS round: back to V (the kx = 0 slots of rows 0 and R/2 join
  // F_0 + i F_n from the two lanes), inverse transforms, stores (the mirror row
  // back through its reversal and twiddle)
  cx<T> wpb[P], wmb[P];
  phase_w(wpb, wmb);
  static_for<0, NMAX, FB>([&](auto F0) __attribute__((always_inline)) {
    constexpr int f0 = decltype(F0)::value;
    if (f0 < N) {
      cx<T> blk[FB][P];
#pragma unroll
      for (int b = 0; b < FB; ++b)
#pragma unroll
        for (int i = 0; i < P; ++i) {
          const cx<T> x = u[f0 + b][i];
          // what the mirror lane needs: the coefficients, or a kx = 0 slot's V
          const cx<T> send = col0 ? from_x(i, x, x, wpb) : x;
          const cx<T> got = lane_xor(send, CH);
          cx<T> v;
          if (!col0)
            v = from_x(i, x, got, wpb);
          else if (self)
            v = hb ? send : send + mul_pi(got);  // a: F_0 + i F_n
          else
            v = send;
          blk[b][i] = v;
        }
      if constexpr (WF) {
        wave_fft_inverse<L, FB>(blk, reinterpret_cast<const V2<float>*>(tw),
                                reinterpret_cast<V2<float>*>(lp.parity ? lp.buf1 : lp.buf0), t2, c);
        lp.parity ^= 1;
      } else {
        fft_inverse<T, L, P, FB, SEQP, false, Lay, L>(blk, t2, lp, C, tw);
      }
      if (stores) {
#pragma unroll
        for (int b = 0; b < FB; ++b)
          if (f0 + b < N) {
#pragma unroll
            for (int i = 0; i < P; ++i)
              buf_st(buf, voff[i], (uint32_t)(f0 + b) * fbytes, to2<T>(blk[b][i] * conj(tw_y(i))));
          }
      }
    }
  });
}

template <typename T, int L, int NMAX>
__global__ __launch_bounds__(k11_threads, 512 / k11_threads) void k11_dst_fused(const K9Args a) {
  constexpr int CH = k11_half_cols(L);
  const int nchunk = (a.nx >> 1) / CH;
  int um = blockIdx.x;
  if (a.group_xcd > 1) {
    // the G blocks sharing each 128-byte line of a row go to blocks b, b + 8,
    // .., b + 8 (G - 1), which the hardware sends to one XCD in turn: the later
    // reads of a line are L2 hits
    const int G = a.group_xcd, x = um & 7, qq = um >> 3;
    um = G * (((qq / G) << 3) + x) + (qq & (G - 1));
  }
  const int k2 = um / nchunk, q = um - k2 * nchunk;
  if (q == 0)
    k11_body<T, L, NMAX, true>(a, k2, q);
  else
    k11_body<T, L, NMAX, false>(a, k2, q);
}

template <typename T, int L, int NMAX>
hipError_t launch_k11_shape(const K9Args& a, hipStream_t st) {
  const int blocks = (a.R / 2 + 1) * ((a.nx / 2) / k11_half_cols(L));
  constexpr size_t lds_bytes = k11_lds_bytes<T, L, NMAX>();
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&k11_dst_fused<T, L, NMAX>),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL((k11_dst_fused<T, L, NMAX>), dim3(blocks), dim3(k11_threads), lds_bytes, st, a);
  return hipGetLastError();
}

}  // namespace fftenkf
