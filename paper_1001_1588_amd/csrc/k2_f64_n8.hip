#include "k2_spectral.hpp"
namespace fftenkf {
hipError_t launch_k2_f64_n8(const K2Args& a, hipStream_t s) {
  switch (a.L) {
    case 1: return launch_k2_shape<double, 1, 8>(a, s);
    case 2: return launch_k2_shape<double, 2, 8>(a, s);
    case 4: return launch_k2_shape<double, 4, 8>(a, s);
    case 8: return launch_k2_shape<double, 8, 8>(a, s);
    case 16: return launch_k2_shape<double, 16, 8>(a, s);
    case 32: return launch_k2_shape<double, 32, 8>(a, s);
    case 64: return launch_k2_shape<double, 64, 8>(a, s);
    case 128: return launch_k2_shape<double, 128, 8>(a, s);
    case 256: return launch_k2_shape<double, 256, 8>(a, s);
    case 512: return launch_k2_shape<double, 512, 8>(a, s);
    case 1024: return launch_k2_shape<double, 1024, 8>(a, s);
    default: return hipErrorInvalidValue;
  }
}
hipError_t launch_k2_batch_f64_n8(const BatchArgs& b, hipStream_t s) {
  switch (b.L) {
    case 1: return launch_k2_batch_shape<double, 1, 8>(b, s);
    case 2: return launch_k2_batch_shape<double, 2, 8>(b, s);
    case 4: return launch_k2_batch_shape<double, 4, 8>(b, s);
    case 8: return launch_k2_batch_shape<double, 8, 8>(b, s);
    case 16: return launch_k2_batch_shape<double, 16, 8>(b, s);
    case 32: return launch_k2_batch_shape<double, 32, 8>(b, s);
    case 64: return launch_k2_batch_shape<double, 64, 8>(b, s);
    case 128: return launch_k2_batch_shape<double, 128, 8>(b, s);
    case 256: return launch_k2_batch_shape<double, 256, 8>(b, s);
    case 512: return launch_k2_batch_shape<double, 512, 8>(b, s);
    case 1024: return launch_k2_batch_shape<double, 1024, 8>(b, s);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace fftenkf
