#include "k2_spectral.hpp"
namespace fftenkf {
hipError_t launch_k2_f64_n4(const K2Args& a, hipStream_t s) {
  switch (a.L) {
    case 1: return launch_k2_shape<double, 1, 4>(a, s);
    case 2: return launch_k2_shape<double, 2, 4>(a, s);
    case 4: return launch_k2_shape<double, 4, 4>(a, s);
    case 8: return launch_k2_shape<double, 8, 4>(a, s);
    case 16: return launch_k2_shape<double, 16, 4>(a, s);
    case 32: return launch_k2_shape<double, 32, 4>(a, s);
    case 64: return launch_k2_shape<double, 64, 4>(a, s);
    case 128: return launch_k2_shape<double, 128, 4>(a, s);
    case 256: return launch_k2_shape<double, 256, 4>(a, s);
    case 512: return launch_k2_shape<double, 512, 4>(a, s);
    case 1024: return launch_k2_shape<double, 1024, 4>(a, s);
    default: return hipErrorInvalidValue;
  }
}
hipError_t launch_k2_batch_f64_n4(const BatchArgs& b, hipStream_t s) {
  switch (b.L) {
    case 1: return launch_k2_batch_shape<double, 1, 4>(b, s);
    case 2: return launch_k2_batch_shape<double, 2, 4>(b, s);
    case 4: return launch_k2_batch_shape<double, 4, 4>(b, s);
    case 8: return launch_k2_batch_shape<double, 8, 4>(b, s);
    case 16: return launch_k2_batch_shape<double, 16, 4>(b, s);
    case 32: return launch_k2_batch_shape<double, 32, 4>(b, s);
    case 64: return launch_k2_batch_shape<double, 64, 4>(b, s);
    case 128: return launch_k2_batch_shape<double, 128, 4>(b, s);
    case 256: return launch_k2_batch_shape<double, 256, 4>(b, s);
    case 512: return launch_k2_batch_shape<double, 512, 4>(b, s);
    case 1024: return launch_k2_batch_shape<double, 1024, 4>(b, s);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace fftenkf
