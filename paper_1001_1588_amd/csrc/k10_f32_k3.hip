#include "k10_observed.hpp"
namespace fftenkf {
static hipError_t k10_f32_k3_n4(const K10Args& a, hipStream_t s) {
  switch (a.L) {
    case 1: return launch_k10_shape<float, 1, 4, 3>(a, s);
    case 2: return launch_k10_shape<float, 2, 4, 3>(a, s);
    case 4: return launch_k10_shape<float, 4, 4, 3>(a, s);
    case 8: return launch_k10_shape<float, 8, 4, 3>(a, s);
    case 16: return launch_k10_shape<float, 16, 4, 3>(a, s);
    case 32: return launch_k10_shape<float, 32, 4, 3>(a, s);
    case 64: return launch_k10_shape<float, 64, 4, 3>(a, s);
    case 128: return launch_k10_shape<float, 128, 4, 3>(a, s);
    case 256: return launch_k10_shape<float, 256, 4, 3>(a, s);
    case 512: return launch_k10_shape<float, 512, 4, 3>(a, s);
    default: return hipErrorInvalidValue;
  }
}
static hipError_t k10_f32_k3_n8(const K10Args& a, hipStream_t s) {
  switch (a.L) {
    case 1: return launch_k10_shape<float, 1, 8, 3>(a, s);
    case 2: return launch_k10_shape<float, 2, 8, 3>(a, s);
    case 4: return launch_k10_shape<float, 4, 8, 3>(a, s);
    case 8: return launch_k10_shape<float, 8, 8, 3>(a, s);
    case 16: return launch_k10_shape<float, 16, 8, 3>(a, s);
    case 32: return launch_k10_shape<float, 32, 8, 3>(a, s);
    case 64: return launch_k10_shape<float, 64, 8, 3>(a, s);
    case 128: return launch_k10_shape<float, 128, 8, 3>(a, s);
    case 256: return launch_k10_shape<float, 256, 8, 3>(a, s);
    case 512: return launch_k10_shape<float, 512, 8, 3>(a, s);
    default: return hipErrorInvalidValue;
  }
}
hipError_t launch_k10_f32_k3(const K10Args& a, hipStream_t s) {
  if (a.N <= 4) return k10_f32_k3_n4(a, s);
  if (a.N <= 8) return k10_f32_k3_n8(a, s);
  return hipErrorInvalidValue;
}
}  // namespace fftenkf
