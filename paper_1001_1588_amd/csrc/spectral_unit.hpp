// Geometry of one unit of the spectral sweep, shared by the single-block and
// multi-block forms, and the folded layout of the kx = 0 column.
//
// A unit covers C adjacent kx < nx/2 of one k2 ([NF][R][L][nx/2]).  A unit's
// row segments are C complex values; when that is less than a 128-byte line,
// the G units sharing each line are given to blocks b, b + 8, .., b + 8 (G - 1),
// which the hardware sends to the same XCD one after the other, so the later
// reads of every line are L2 hits rather than further HBM fetches.
//
// Folded Nyquist column.  For a real field the x transforms at kx = 0 and at
// kx = nx/2 are real sequences along y, so after the radix-R stage of sweep 1
// the rows k2 and R - k2 of each are copies of one another,
// A(R - k2, y1) = W_L^y1 conj A(k2, y1), and kx = nx/2 needs no storage of its
// own.  Column kx = 0 of the workspace holds, per row k2 (H = R/2):
//   0 < k2 < H:    A_0(k2, y1)                   (the kx = 0 sequence)
//   H < k2 < R:    A_n(R - k2, y1)               (the kx = nx/2 sequence of row R - k2)
//   k2 in {0, H}:  A_0(k2, y1) + i A_n(k2, y1)   (packed: the two rows are
//                                                 self-mirrored)
// After the length-L transform of sweep 2, slot k1 of a row k2 < H holds bin
// (k2 + R k1, 0), of a row k2 > H bin (R - k2 + R k1, nx/2).  A packed row's
// transform Z = F_0 + i F_n is split with the symmetry of a real sequence's
// transform, F(m(k1)) = conj F(k1), m(k1) = (L - k1) mod L for k2 = 0 and
// L - 1 - k1 for k2 = H:
//   k1 < m(k1):  F_0(k1) = (Z(k1) + conj Z(m)) / 2         bin (k2 + R k1, 0)
//   k1 > m(k1):  F_n(k1) = (Z(k1) - conj Z(m)) / (2i)      bin (k2 + R k1, nx/2)
//   k1 = m(k1):  Z(k1) itself: the real bins (k2 + R k1, 0) and (k2 + R k1, nx/2)
//                as its real and imaginary parts (a "pair" slot)
// and joined again before the inverse transform.  Every bin of the half
// spectrum not held by a slot is the conjugate of one that is (the kx = 0 and
// nx/2 bins above ny/2).  With no Nyquist units the sweep's grid is exactly
// R (nx/2) / C units.
#pragma once

#include "fft_core.hpp"

namespace fftenkf {

template <typename T>
struct SpectralUnit {
  int k2, kx;        // this thread's column: frequency k2 of the radix-R stage and kx
  bool fold;         // the unit holds column kx = 0 of a packed row (k2 in {0, R/2}): block-uniform
  bool col0;         // this thread holds column kx = 0
  uint32_t cbytes;   // byte offset of this thread's column of field 0
  uint32_t fstride;  // elements between fields
  uint32_t sy;       // elements between consecutive y1 (or k1)
};

// Thread column c < C of block `unit`.
template <typename T>
__device__ __forceinline__ SpectralUnit<T> spectral_unit(int unit, int c, int C, int R, int L, int ny, int nxh,
                                                         int group_xcd) {
  SpectralUnit<T> g;
  int um = unit;
  if (group_xcd > 1) {
    const int G = group_xcd;  // a power of two
    const int x = um & 7, q = um >> 3;
    um = G * (((q / G) << 3) + x) + (q & (G - 1));
  }
  const int nchunk = nxh / C;
  g.k2 = um / nchunk;
  const int kxc = um - g.k2 * nchunk;
  g.kx = kxc * C + c;
  g.fold = kxc == 0 && (g.k2 == 0 || g.k2 == (R >> 1));
  g.col0 = g.kx == 0;
  const size_t off = (size_t)g.k2 * L * nxh + (size_t)kxc * C;
  g.fstride = (uint32_t)ny * (uint32_t)nxh;
  g.sy = (uint32_t)nxh;
  g.cbytes = (uint32_t)((off + (size_t)c) * sizeof(V2<T>));
  return g;
}

// Mirror slot of k1 in a packed row k2 in {0, R/2}.
__host__ __device__ __forceinline__ int fold_mirror(int k2, int k1, int L) {
  return k2 == 0 ? (L - k1) & (L - 1) : L - 1 - k1;
}

// The bin held by slot k1 of column kx of row k2 (after the split): (ky, kx);
// pair: the slot holds the real bins (ky, 0) and (ky, nx/2) as its real and
// imaginary parts (then kx = 0).
struct SlotBin {
  int ky, kx;
  bool pair;
};
__host__ __device__ __forceinline__ SlotBin slot_bin(int k2, int k1, int kx, int R, int L, int nxh) {
  const int H = R >> 1;
  if (kx != 0) return SlotBin{k2 + R * k1, kx, false};
  if (k2 > H) return SlotBin{R - k2 + R * k1, nxh, false};
  if (k2 != 0 && k2 != H) return SlotBin{k2 + R * k1, 0, false};
  const int m = fold_mirror(k2, k1, L);
  return SlotBin{k2 + R * k1, k1 <= m ? 0 : nxh, k1 == m};
}

// slot_bin for the P points of one thread (rows t2 + TF2 i of column kx of row
// k2) in a form that costs the sweep two registers: point i holds bin
// (kyb + R r, r > thr ? nx/2 : kx), r = t2 + TF2 i, and a pair slot only at
// point 0 (pair0) or at point P/2 (pairh, row L/2).
struct ColumnBins {
  int kyb, thr;
  bool pair0, pairh;
};
__host__ __device__ __forceinline__ ColumnBins column_bins(int k2, int kx, int t2, int R, int L) {
  const int H = R >> 1;
  ColumnBins b{k2, L, false, false};
  if (kx != 0) return b;
  if (k2 > H) {
    b.kyb = R - k2;
    b.thr = -1;
  } else if (k2 == 0) {
    b.thr = L >> 1;
    b.pair0 = t2 == 0;
    b.pairh = t2 == 0 && L >= 2;
  } else if (k2 == H) {
    b.thr = (L - 1) >> 1;
    b.pair0 = t2 == 0 && L == 1;
  }
  return b;
}

// Where bin (ky, kx) of the half spectrum lives: slot (k2, k1) of column col,
// read as op 0 the value, 1 its conjugate, 2 the real part, 3 the imaginary
// part.  Ops 0, 2 and 3 mark the bin that owns the slot.
struct BinSlot {
  int k2, k1, col, op;
};
__host__ __device__ __forceinline__ BinSlot bin_slot(int ky, int kx, int R, int L, int nxh) {
  const int k2 = ky % R, k1 = ky / R, H = R >> 1;
  if (kx != 0 && kx != nxh) return BinSlot{k2, k1, kx, 0};
  const bool nyq = kx == nxh;
  if (k2 != 0 && k2 != H) {
    const bool low = k2 < H;
    // a high row's bins are the conjugates of the low row R - k2 at L - 1 - k1
    if (!nyq) return low ? BinSlot{k2, k1, 0, 0} : BinSlot{R - k2, L - 1 - k1, 0, 1};
    return low ? BinSlot{R - k2, k1, 0, 0} : BinSlot{k2, L - 1 - k1, 0, 1};
  }
  const int m = fold_mirror(k2, k1, L);
  if (k1 == m) return BinSlot{k2, k1, 0, nyq ? 3 : 2};
  const bool own = nyq ? (k1 > m) : (k1 < m);
  return own ? BinSlot{k2, k1, 0, 0} : BinSlot{k2, m, 0, 1};
}

// Split (forward) or join (inverse) the packed column of a fold unit, for F
// fields of P points per thread (rows t2 + TF2 i): threads of column kx = 0
// exchange with the mirror rows through one of two buffers of F x L elements
// at xch, taken in turn (par): the barrier of one exchange also orders the
// reads of the exchange before it against the writes of the one after, so one
// barrier suffices.  Each buffer holds FCAP >= F fields.  Block-uniform: every
// thread of the block calls it.
template <typename T, int F, int FCAP, int P, int TF2, int L>
__device__ __forceinline__ void fold_exchange(cx<T> (&v)[F][P], V2<T>* xch0, int& par, int t2, bool lane, int k2,
                                              bool split) {
  static_assert(F <= FCAP, "fold exchange buffer too small");
  V2<T>* const xch = xch0 + par * FCAP * L;
  par ^= 1;
  if (lane) {
#pragma unroll
    for (int b = 0; b < F; ++b)
#pragma unroll
      for (int i = 0; i < P; ++i) xch[b * L + t2 + TF2 * i] = to2<T>(v[b][i]);
  }
  __syncthreads();
  if (lane) {
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int r = t2 + TF2 * i;
      const int m = fold_mirror(k2, r, L);
#pragma unroll
      for (int b = 0; b < F; ++b) {
        const cx<T> own = v[b][i];
        const cx<T> pc = conj(from2<T>(xch[b * L + m]));
        cx<T> w;
        if (split)  // F_0 = (Z + conj Z(m)) / 2, F_n = (Z - conj Z(m)) / (2i)
          w = r < m ? scale(own + pc, T(0.5)) : scale(mul_mi(own - pc), T(0.5));
        else        // Z = F_0 + i F_n: own F_0 with conj of the mirror's F_n, or the converse
          w = r < m ? own + mul_pi(pc) : pc + mul_pi(own);
        v[b][i] = r == m ? own : w;
      }
    }
  }
}

}  // namespace fftenkf
