#include "k6_multiblock.hpp"
namespace fftenkf {
template <int NMAX>
hipError_t launch_k6_f32_bucket(const K6Args& a, hipStream_t s) {
  switch (a.L) {
    case 1: return launch_k6_shape<float, 1, NMAX>(a, s);
    case 2: return launch_k6_shape<float, 2, NMAX>(a, s);
    case 4: return launch_k6_shape<float, 4, NMAX>(a, s);
    case 8: return launch_k6_shape<float, 8, NMAX>(a, s);
    case 16: return launch_k6_shape<float, 16, NMAX>(a, s);
    case 32: return launch_k6_shape<float, 32, NMAX>(a, s);
    case 64: return launch_k6_shape<float, 64, NMAX>(a, s);
    case 128: return launch_k6_shape<float, 128, NMAX>(a, s);
    case 256: return launch_k6_shape<float, 256, NMAX>(a, s);
    case 512: return launch_k6_shape<float, 512, NMAX>(a, s);
    default: return hipErrorInvalidValue;
  }
}
hipError_t launch_k6_f32(const K6Args& a, hipStream_t s) {
  if (a.N <= 4) return launch_k6_f32_bucket<4>(a, s);
  if (a.N <= 6) return launch_k6_f32_bucket<6>(a, s);
  if (a.N <= 8) return launch_k6_f32_bucket<8>(a, s);
  if (a.N <= 10) return launch_k6_f32_bucket<10>(a, s);
  if (a.N <= 12) return launch_k6_f32_bucket<12>(a, s);
  return hipErrorInvalidValue;
}
}  // namespace fftenkf
