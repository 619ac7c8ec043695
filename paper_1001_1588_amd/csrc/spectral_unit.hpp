// Geometry of one unit of the spectral sweep, shared by the single-block and
// multi-block forms.
//
// Main units cover kx < nx/2 ([NF][R][L][nx/2]: C adjacent kx of one k2); the
// Nyquist column kx = nx/2 ([NF][L][R]) is covered by extra units over C
// adjacent k2, placed first in the grid so they do not trail.  A unit's row
// segments are C complex values; when that is less than a 128-byte line, the G
// units sharing each line are given to blocks b, b + 8, .., b + 8 (G - 1),
// which the hardware sends to the same XCD one after the other, so the later
// reads of every line are L2 hits rather than further HBM fetches.
#pragma once

#include "fft_core.hpp"

namespace fftenkf {

template <typename T>
struct SpectralUnit {
  int k2, kx;         // this thread's column: frequency k2 of the radix-R stage and kx
  bool valid;         // false for padding threads of a Nyquist unit
  bool nyq;           // a Nyquist unit (its fields live in ws_nyq)
  V2<T>* ubase;       // uniform base of field 0 of this unit
  uint32_t fstride;   // elements between fields
  uint32_t sy;        // elements between consecutive y1 (or k1)
  int cc;             // this thread's column offset from ubase (0 if not valid)
  uint32_t cbytes;    // byte offset of this thread's column of field 0 from the start of its region
};

// Thread column c < C of block `unit`.  Nyquist units cover Cn <= C adjacent k2
// (threads with c >= Cn, and those beyond R, are padding: they read column 0
// and never write).
template <typename T>
__device__ __forceinline__ SpectralUnit<T> spectral_unit(void* ws_main, void* ws_nyq, int unit, int c, int C, int Cn,
                                                         int R, int L, int ny, int nxh, int units_main,
                                                         int units_total, int group_xcd) {
  SpectralUnit<T> g;
  const int units_nyq = units_total - units_main;
  if (unit >= units_nyq) {
    int um = unit - units_nyq;
    if (group_xcd > 1) {
      const int G = group_xcd;  // a power of two
      const int x = um & 7, q = um >> 3;
      um = G * (((q / G) << 3) + x) + (q & (G - 1));
    }
    const int nchunk = nxh / C;
    g.k2 = um / nchunk;
    const int kxc = um - g.k2 * nchunk;
    g.kx = kxc * C + c;
    g.valid = true;
    g.nyq = false;
    const size_t off = (size_t)g.k2 * L * nxh + (size_t)kxc * C;
    g.ubase = static_cast<V2<T>*>(ws_main) + off;
    g.fstride = (uint32_t)ny * (uint32_t)nxh;
    g.sy = (uint32_t)nxh;
    g.cc = c;
    g.cbytes = (uint32_t)((off + (size_t)c) * sizeof(V2<T>));
  } else {
    const int v = unit;
    g.k2 = v * Cn + c;
    g.kx = nxh;
    g.valid = c < Cn && g.k2 < R;
    g.nyq = true;
    g.ubase = static_cast<V2<T>*>(ws_nyq) + (size_t)v * Cn;
    g.fstride = (uint32_t)ny;
    g.sy = (uint32_t)R;
    g.cc = g.valid ? c : 0;
    g.cbytes = (uint32_t)(((size_t)v * Cn + (size_t)g.cc) * sizeof(V2<T>));
  }
  return g;
}

}  // namespace fftenkf
