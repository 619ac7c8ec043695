#include "k1_forward.hpp"
namespace fftenkf {
template <int NX>
static hipError_t k1_f32_R(const K1Args& a, hipStream_t s) {
  if constexpr (NX <= 2048) {
    if (a.R == 16) return launch_k1_shape<float, NX, 16>(a, s);
  }
  if (a.R == 8) return launch_k1_shape<float, NX, 8>(a, s);
  return hipErrorInvalidValue;
}
hipError_t launch_k1_f32(const K1Args& a, hipStream_t s) {
  switch (a.nx) {
    case 8: return k1_f32_R<8>(a, s);
    case 16: return k1_f32_R<16>(a, s);
    case 32: return k1_f32_R<32>(a, s);
    case 64: return k1_f32_R<64>(a, s);
    case 128: return k1_f32_R<128>(a, s);
    case 256: return k1_f32_R<256>(a, s);
    case 512: return k1_f32_R<512>(a, s);
    case 1024: return k1_f32_R<1024>(a, s);
    case 2048: return k1_f32_R<2048>(a, s);
    case 4096: return k1_f32_R<4096>(a, s);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace fftenkf
