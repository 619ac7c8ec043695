// Dispatch of the fused sine-basis sweep over member buckets and dtypes.
#include "k11_dst_fused.hpp"
namespace fftenkf {
hipError_t launch_k11_f32_n8(const K9Args& a, hipStream_t s);
hipError_t launch_k11_f32_n12(const K9Args& a, hipStream_t s);
hipError_t launch_k11_f32_n16(const K9Args& a, hipStream_t s);
hipError_t launch_k11_f32_n20(const K9Args& a, hipStream_t s);
hipError_t launch_k11_f32_n24(const K9Args& a, hipStream_t s);

namespace {
hipError_t launch_f64(const K9Args& a, hipStream_t s) {
  if (a.N > 8) return hipErrorNotSupported;
  switch (a.L) {
    case 16: return launch_k11_shape<double, 16, 8>(a, s);
    case 32: return launch_k11_shape<double, 32, 8>(a, s);
    case 64: return launch_k11_shape<double, 64, 8>(a, s);
    case 128: return launch_k11_shape<double, 128, 8>(a, s);
    case 256: return launch_k11_shape<double, 256, 8>(a, s);
    case 512: return launch_k11_shape<double, 512, 8>(a, s);
    default: return hipErrorNotSupported;
  }
}
}  // namespace

bool k11_supports(int L, int nx) {
  if (L < k11_min_L || L > 512) return false;
  const int ch = k11_half_cols(L);
  return ch >= 1 && (nx / 2) % ch == 0 && nx / 2 >= ch;
}

hipError_t launch_k11(const K9Args& a_in, int dtype, hipStream_t s) {
  if (!k11_supports(a_in.L, a_in.nx)) return hipErrorNotSupported;
  K9Args a = a_in;
  const int ch = k11_half_cols(a.L), nchunk = (a.nx / 2) / ch, blocks = (a.R / 2 + 1) * nchunk;
  const int seg = ch * (dtype == 0 ? 8 : 16);
  const int g = seg < 128 ? 128 / seg : 1;
  a.group_xcd = (g > 1 && nchunk % g == 0 && blocks % (8 * g) == 0) ? g : 1;
  if (dtype != 0) return launch_f64(a, s);
  if (a.N <= 8) return launch_k11_f32_n8(a, s);
  if (a.N <= 12) return launch_k11_f32_n12(a, s);
  if (a.N <= 16) return launch_k11_f32_n16(a, s);
  if (a.N <= 20) return launch_k11_f32_n20(a, s);
  if (a.N <= 24) return launch_k11_f32_n24(a, s);
  return hipErrorNotSupported;
}
}  // namespace fftenkf
