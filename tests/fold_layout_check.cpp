// Host check of the folded kx = 0 column (spectral_unit.hpp): slot_bin,
// column_bins and bin_slot describe one layout, and every bin of the kx = 0
// and kx = nx/2 columns is held by exactly one slot, directly or as the
// conjugate of its mirror (ny - ky).  Prints "ok" and exits 0 on success.
#include <cstdio>

#include "spectral_unit.hpp"

using namespace fftenkf;

static int fails = 0;
#define CHECK(c, ...)             \
  do {                            \
    if (!(c)) {                   \
      if (++fails < 20) {         \
        std::printf(__VA_ARGS__); \
        std::printf("\n");        \
      }                           \
    }                             \
  } while (0)

int main() {
  const int nxh = 8;
  for (int R : {4, 8, 16}) {
    for (int L : {1, 2, 4, 8, 16, 64, 128}) {
      const int ny = R * L;
      const int P = L < 4 ? L : 4, TF2 = L / P;
      // slots of column 0 -> bins -> back to the same slot
      int pairs = 0;
      for (int k2 = 0; k2 < R; ++k2)
        for (int k1 = 0; k1 < L; ++k1) {
          const SlotBin sb = slot_bin(k2, k1, 0, R, L, nxh);
          CHECK(sb.ky >= 0 && sb.ky < ny && (sb.kx == 0 || sb.kx == nxh), "R=%d L=%d slot (%d,%d): bin out of range", R,
                L, k2, k1);
          const BinSlot bs = bin_slot(sb.ky, sb.kx, R, L, nxh);
          CHECK(bs.k2 == k2 && bs.k1 == k1 && bs.col == 0 && (bs.op == 0 || (sb.pair && bs.op == 2)),
                "R=%d L=%d slot (%d,%d) -> bin (%d,%d) -> slot (%d,%d) op %d", R, L, k2, k1, sb.ky, sb.kx, bs.k2, bs.k1,
                bs.op);
          if (sb.pair) {
            ++pairs;
            CHECK((sb.ky == 0 || sb.ky == ny / 2) && sb.kx == 0, "R=%d L=%d pair slot (%d,%d) not self-conjugate", R, L,
                  k2, k1);
            const BinSlot bn = bin_slot(sb.ky, nxh, R, L, nxh);
            CHECK(bn.k2 == k2 && bn.k1 == k1 && bn.op == 3, "R=%d L=%d pair slot (%d,%d): nx/2 bin elsewhere", R, L, k2,
                  k1);
          }
          // the per-thread form: thread t2 holds rows t2 + TF2 i
          const int t2 = k1 % TF2, i = k1 / TF2;
          const ColumnBins cb = column_bins(k2, 0, t2, R, L);
          const int ky = cb.kyb + R * k1, kx = k1 > cb.thr ? nxh : 0;
          const bool pr = i == 0 ? cb.pair0 : (i == P / 2 ? cb.pairh : false);
          CHECK(ky == sb.ky && kx == sb.kx && pr == sb.pair,
                "R=%d L=%d slot (%d,%d): column_bins (%d,%d,%d) vs slot_bin (%d,%d,%d)", R, L, k2, k1, ky, kx, (int)pr,
                sb.ky, sb.kx, (int)sb.pair);
        }
      CHECK(pairs == 2, "R=%d L=%d: %d pair slots, 2 expected", R, L, pairs);
      // bins -> slots: a bin that does not own its slot is the conjugate of its mirror, which does
      int owners = 0;
      for (int kx : {0, nxh})
        for (int ky = 0; ky < ny; ++ky) {
          const BinSlot bs = bin_slot(ky, kx, R, L, nxh);
          CHECK(bs.k2 >= 0 && bs.k2 < R && bs.k1 >= 0 && bs.k1 < L && bs.col == 0, "R=%d L=%d bin (%d,%d): bad slot",
                R, L, ky, kx);
          if (bs.op == 1) {
            const BinSlot bm = bin_slot((ny - ky) % ny, kx, R, L, nxh);
            CHECK(bm.op == 0 && bm.k2 == bs.k2 && bm.k1 == bs.k1, "R=%d L=%d bin (%d,%d): mirror does not own the slot",
                  R, L, ky, kx);
          } else {
            ++owners;
            const SlotBin sb = slot_bin(bs.k2, bs.k1, 0, R, L, nxh);
            CHECK(sb.ky == ky && (sb.kx == kx || (sb.pair && bs.op == 3)), "R=%d L=%d bin (%d,%d) owns slot of (%d,%d)",
                  R, L, ky, kx, sb.ky, sb.kx);
          }
        }
      CHECK(owners == R * L + pairs, "R=%d L=%d: %d owning bins for %d slots", R, L, owners, R * L);
      // interior columns are not folded
      const BinSlot b3 = bin_slot(1, 3, R, L, nxh);
      CHECK(b3.k2 == 1 && b3.k1 == 0 && b3.col == 3 && b3.op == 0, "R=%d L=%d: interior bin moved", R, L);
      const ColumnBins c3 = column_bins(1, 3, 0, R, L);
      CHECK(c3.kyb == 1 && c3.thr >= L - 1 && !c3.pair0 && !c3.pairh, "R=%d L=%d: interior column folded", R, L);
    }
  }
  if (fails) {
    std::printf("%d failures\n", fails);
    return 1;
  }
  std::printf("ok\n");
  return 0;
}
