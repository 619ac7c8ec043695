#include "k2_spectral.hpp"
namespace fftenkf {
hipError_t launch_k2_f32_n24(const K2Args& a, hipStream_t s) {
  switch (a.L) {
    case 1: return launch_k2_shape<float, 1, 24>(a, s);
    case 2: return launch_k2_shape<float, 2, 24>(a, s);
    case 4: return launch_k2_shape<float, 4, 24>(a, s);
    case 8: return launch_k2_shape<float, 8, 24>(a, s);
    case 16: return launch_k2_shape<float, 16, 24>(a, s);
    case 32: return launch_k2_shape<float, 32, 24>(a, s);
    case 64: return launch_k2_shape<float, 64, 24>(a, s);
    case 128: return launch_k2_shape<float, 128, 24>(a, s);
    case 256: return launch_k2_shape<float, 256, 24>(a, s);
    case 512: return launch_k2_shape<float, 512, 24>(a, s);

    default: return hipErrorInvalidValue;
  }
}
hipError_t launch_k2_batch_f32_n24(const BatchArgs& b, hipStream_t s) {
  switch (b.L) {
    case 1: return launch_k2_batch_shape<float, 1, 24>(b, s);
    case 2: return launch_k2_batch_shape<float, 2, 24>(b, s);
    case 4: return launch_k2_batch_shape<float, 4, 24>(b, s);
    case 8: return launch_k2_batch_shape<float, 8, 24>(b, s);
    case 16: return launch_k2_batch_shape<float, 16, 24>(b, s);
    case 32: return launch_k2_batch_shape<float, 32, 24>(b, s);
    case 64: return launch_k2_batch_shape<float, 64, 24>(b, s);
    case 128: return launch_k2_batch_shape<float, 128, 24>(b, s);
    case 256: return launch_k2_batch_shape<float, 256, 24>(b, s);
    case 512: return launch_k2_batch_shape<float, 512, 24>(b, s);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace fftenkf
