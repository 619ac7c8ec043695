#include "k10_observed.hpp"
namespace fftenkf {
static hipError_t k10_f32_k1_n4(const K10Args& a, hipStream_t s) {
  switch (a.L) {
    case 1: return launch_k10_shape<float, 1, 4, 1>(a, s);
    case 2: return launch_k10_shape<float, 2, 4, 1>(a, s);
    case 4: return launch_k10_shape<float, 4, 4, 1>(a, s);
    case 8: return launch_k10_shape<float, 8, 4, 1>(a, s);
    case 16: return launch_k10_shape<float, 16, 4, 1>(a, s);
    case 32: return launch_k10_shape<float, 32, 4, 1>(a, s);
    case 64: return launch_k10_shape<float, 64, 4, 1>(a, s);
    case 128: return launch_k10_shape<float, 128, 4, 1>(a, s);
    case 256: return launch_k10_shape<float, 256, 4, 1>(a, s);
    case 512: return launch_k10_shape<float, 512, 4, 1>(a, s);
    default: return hipErrorInvalidValue;
  }
}
static hipError_t k10_f32_k1_n6(const K10Args& a, hipStream_t s) {
  switch (a.L) {
    case 1: return launch_k10_shape<float, 1, 6, 1>(a, s);
    case 2: return launch_k10_shape<float, 2, 6, 1>(a, s);
    case 4: return launch_k10_shape<float, 4, 6, 1>(a, s);
    case 8: return launch_k10_shape<float, 8, 6, 1>(a, s);
    case 16: return launch_k10_shape<float, 16, 6, 1>(a, s);
    case 32: return launch_k10_shape<float, 32, 6, 1>(a, s);
    case 64: return launch_k10_shape<float, 64, 6, 1>(a, s);
    case 128: return launch_k10_shape<float, 128, 6, 1>(a, s);
    case 256: return launch_k10_shape<float, 256, 6, 1>(a, s);
    case 512: return launch_k10_shape<float, 512, 6, 1>(a, s);
    default: return hipErrorInvalidValue;
  }
}
static hipError_t k10_f32_k1_n8(const K10Args& a, hipStream_t s) {
  switch (a.L) {
    case 1: return launch_k10_shape<float, 1, 8, 1>(a, s);
    case 2: return launch_k10_shape<float, 2, 8, 1>(a, s);
    case 4: return launch_k10_shape<float, 4, 8, 1>(a, s);
    case 8: return launch_k10_shape<float, 8, 8, 1>(a, s);
    case 16: return launch_k10_shape<float, 16, 8, 1>(a, s);
    case 32: return launch_k10_shape<float, 32, 8, 1>(a, s);
    case 64: return launch_k10_shape<float, 64, 8, 1>(a, s);
    case 128: return launch_k10_shape<float, 128, 8, 1>(a, s);
    case 256: return launch_k10_shape<float, 256, 8, 1>(a, s);
    case 512: return launch_k10_shape<float, 512, 8, 1>(a, s);
    default: return hipErrorInvalidValue;
  }
}
static hipError_t k10_f32_k1_n10(const K10Args& a, hipStream_t s) {
  switch (a.L) {
    case 1: return launch_k10_shape<float, 1, 10, 1>(a, s);
    case 2: return launch_k10_shape<float, 2, 10, 1>(a, s);
    case 4: return launch_k10_shape<float, 4, 10, 1>(a, s);
    case 8: return launch_k10_shape<float, 8, 10, 1>(a, s);
    case 16: return launch_k10_shape<float, 16, 10, 1>(a, s);
    case 32: return launch_k10_shape<float, 32, 10, 1>(a, s);
    case 64: return launch_k10_shape<float, 64, 10, 1>(a, s);
    case 128: return launch_k10_shape<float, 128, 10, 1>(a, s);
    case 256: return launch_k10_shape<float, 256, 10, 1>(a, s);
    case 512: return launch_k10_shape<float, 512, 10, 1>(a, s);
    default: return hipErrorInvalidValue;
  }
}
static hipError_t k10_f32_k1_n12(const K10Args& a, hipStream_t s) {
  switch (a.L) {
    case 1: return launch_k10_shape<float, 1, 12, 1>(a, s);
    case 2: return launch_k10_shape<float, 2, 12, 1>(a, s);
    case 4: return launch_k10_shape<float, 4, 12, 1>(a, s);
    case 8: return launch_k10_shape<float, 8, 12, 1>(a, s);
    case 16: return launch_k10_shape<float, 16, 12, 1>(a, s);
    case 32: return launch_k10_shape<float, 32, 12, 1>(a, s);
    case 64: return launch_k10_shape<float, 64, 12, 1>(a, s);
    case 128: return launch_k10_shape<float, 128, 12, 1>(a, s);
    case 256: return launch_k10_shape<float, 256, 12, 1>(a, s);
    case 512: return launch_k10_shape<float, 512, 12, 1>(a, s);
    default: return hipErrorInvalidValue;
  }
}
hipError_t launch_k10_f32_k1(const K10Args& a, hipStream_t s) {
  if (a.N <= 4) return k10_f32_k1_n4(a, s);
  if (a.N <= 6) return k10_f32_k1_n6(a, s);
  if (a.N <= 8) return k10_f32_k1_n8(a, s);
  if (a.N <= 10) return k10_f32_k1_n10(a, s);
  if (a.N <= 12) return k10_f32_k1_n12(a, s);
  return hipErrorInvalidValue;
}
}  // namespace fftenkf
