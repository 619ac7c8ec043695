#include "k10_observed.hpp"
namespace fftenkf {
static hipError_t k10_f64_k1_n2(const K10Args& a, hipStream_t s) {
  switch (a.L) {
    case 1: return launch_k10_shape<double, 1, 2, 1>(a, s);
    case 2: return launch_k10_shape<double, 2, 2, 1>(a, s);
    case 4: return launch_k10_shape<double, 4, 2, 1>(a, s);
    case 8: return launch_k10_shape<double, 8, 2, 1>(a, s);
    case 16: return launch_k10_shape<double, 16, 2, 1>(a, s);
    case 32: return launch_k10_shape<double, 32, 2, 1>(a, s);
    case 64: return launch_k10_shape<double, 64, 2, 1>(a, s);
    case 128: return launch_k10_shape<double, 128, 2, 1>(a, s);
    case 256: return launch_k10_shape<double, 256, 2, 1>(a, s);
    case 512: return launch_k10_shape<double, 512, 2, 1>(a, s);
    case 1024: return launch_k10_shape<double, 1024, 2, 1>(a, s);
    default: return hipErrorInvalidValue;
  }
}
static hipError_t k10_f64_k1_n4(const K10Args& a, hipStream_t s) {
  switch (a.L) {
    case 1: return launch_k10_shape<double, 1, 4, 1>(a, s);
    case 2: return launch_k10_shape<double, 2, 4, 1>(a, s);
    case 4: return launch_k10_shape<double, 4, 4, 1>(a, s);
    case 8: return launch_k10_shape<double, 8, 4, 1>(a, s);
    case 16: return launch_k10_shape<double, 16, 4, 1>(a, s);
    case 32: return launch_k10_shape<double, 32, 4, 1>(a, s);
    case 64: return launch_k10_shape<double, 64, 4, 1>(a, s);
    case 128: return launch_k10_shape<double, 128, 4, 1>(a, s);
    case 256: return launch_k10_shape<double, 256, 4, 1>(a, s);
    case 512: return launch_k10_shape<double, 512, 4, 1>(a, s);
    case 1024: return launch_k10_shape<double, 1024, 4, 1>(a, s);
    default: return hipErrorInvalidValue;
  }
}
static hipError_t k10_f64_k3_n2(const K10Args& a, hipStream_t s) {
  switch (a.L) {
    case 1: return launch_k10_shape<double, 1, 2, 3>(a, s);
    case 2: return launch_k10_shape<double, 2, 2, 3>(a, s);
    case 4: return launch_k10_shape<double, 4, 2, 3>(a, s);
    case 8: return launch_k10_shape<double, 8, 2, 3>(a, s);
    case 16: return launch_k10_shape<double, 16, 2, 3>(a, s);
    case 32: return launch_k10_shape<double, 32, 2, 3>(a, s);
    case 64: return launch_k10_shape<double, 64, 2, 3>(a, s);
    case 128: return launch_k10_shape<double, 128, 2, 3>(a, s);
    case 256: return launch_k10_shape<double, 256, 2, 3>(a, s);
    case 512: return launch_k10_shape<double, 512, 2, 3>(a, s);
    case 1024: return launch_k10_shape<double, 1024, 2, 3>(a, s);
    default: return hipErrorInvalidValue;
  }
}
static hipError_t k10_f64_k3_n4(const K10Args& a, hipStream_t s) {
  switch (a.L) {
    case 1: return launch_k10_shape<double, 1, 4, 3>(a, s);
    case 2: return launch_k10_shape<double, 2, 4, 3>(a, s);
    case 4: return launch_k10_shape<double, 4, 4, 3>(a, s);
    case 8: return launch_k10_shape<double, 8, 4, 3>(a, s);
    case 16: return launch_k10_shape<double, 16, 4, 3>(a, s);
    case 32: return launch_k10_shape<double, 32, 4, 3>(a, s);
    case 64: return launch_k10_shape<double, 64, 4, 3>(a, s);
    case 128: return launch_k10_shape<double, 128, 4, 3>(a, s);
    case 256: return launch_k10_shape<double, 256, 4, 3>(a, s);
    case 512: return launch_k10_shape<double, 512, 4, 3>(a, s);
    case 1024: return launch_k10_shape<double, 1024, 4, 3>(a, s);
    default: return hipErrorInvalidValue;
  }
}
hipError_t launch_k10_f64(const K10Args& a, hipStream_t s) {
  if (a.N > 4) return hipErrorInvalidValue;
  if (a.K == 1) return a.N <= 2 ? k10_f64_k1_n2(a, s) : k10_f64_k1_n4(a, s);
  return a.N <= 2 ? k10_f64_k3_n2(a, s) : k10_f64_k3_n4(a, s);
}
}  // namespace fftenkf
