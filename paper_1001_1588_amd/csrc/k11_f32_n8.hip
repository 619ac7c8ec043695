#include "k11_dst_fused.hpp"
namespace fftenkf {
hipError_t launch_k11_f32_n8(const K9Args& a, hipStream_t s) {
  switch (a.L) {
    case 16: return launch_k11_shape<float, 16, 8>(a, s);
    case 32: return launch_k11_shape<float, 32, 8>(a, s);
    case 64: return launch_k11_shape<float, 64, 8>(a, s);
    case 128: return launch_k11_shape<float, 128, 8>(a, s);
    case 256: return launch_k11_shape<float, 256, 8>(a, s);
    case 512: return launch_k11_shape<float, 512, 8>(a, s);
    default: return hipErrorNotSupported;
  }
}
}  // namespace fftenkf
