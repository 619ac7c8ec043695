#include "k3_inverse.hpp"
namespace fftenkf {
template <int NX>
static hipError_t k3_f32_R(const K3Args& a, int R, hipStream_t s) {
  if constexpr (NX <= 2048) {
    if (R == 16) return launch_k3_shape<float, NX, 16>(a, s);
    if (R == 4) return launch_k3_shape<float, NX, 4>(a, s);
  }
  if (R == 8) return launch_k3_shape<float, NX, 8>(a, s);
  return hipErrorInvalidValue;
}
hipError_t launch_k3_f32(const K3Args& a, hipStream_t s) {
  const int R = a.R;
  switch (a.nx) {
    case 8: return k3_f32_R<8>(a, R, s);
    case 16: return k3_f32_R<16>(a, R, s);
    case 32: return k3_f32_R<32>(a, R, s);
    case 64: return k3_f32_R<64>(a, R, s);
    case 128: return k3_f32_R<128>(a, R, s);
    case 256: return k3_f32_R<256>(a, R, s);
    case 512: return k3_f32_R<512>(a, R, s);
    case 1024: return k3_f32_R<1024>(a, R, s);
    case 2048: return k3_f32_R<2048>(a, R, s);
    case 4096: return k3_f32_R<4096>(a, R, s);
    default: return hipErrorInvalidValue;
  }
}
template <int NX>
static hipError_t k3_f32_R_batch(const BatchArgs& a, int R, hipStream_t s) {
  if constexpr (NX <= 2048) {
    if (R == 16) return launch_k3_batch_shape<float, NX, 16>(a, s);
    if (R == 4) return launch_k3_batch_shape<float, NX, 4>(a, s);
  }
  if (R == 8) return launch_k3_batch_shape<float, NX, 8>(a, s);
  return hipErrorInvalidValue;
}
hipError_t launch_k3_batch_f32(const BatchArgs& a, int R, hipStream_t s) {
  switch (a.nx) {
    case 8: return k3_f32_R_batch<8>(a, R, s);
    case 16: return k3_f32_R_batch<16>(a, R, s);
    case 32: return k3_f32_R_batch<32>(a, R, s);
    case 64: return k3_f32_R_batch<64>(a, R, s);
    case 128: return k3_f32_R_batch<128>(a, R, s);
    case 256: return k3_f32_R_batch<256>(a, R, s);
    case 512: return k3_f32_R_batch<512>(a, R, s);
    case 1024: return k3_f32_R_batch<1024>(a, R, s);
    case 2048: return k3_f32_R_batch<2048>(a, R, s);
    case 4096: return k3_f32_R_batch<4096>(a, R, s);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace fftenkf
