// Test exports only: copy half spectra between the caller's [N][ny][nx/2+1]
// layout and the transformed layout of the spectral sweep, one thread per bin.
#include <hip/hip_runtime.h>

#include "fft_core.hpp"
#include "kernels.hpp"

namespace fftenkf {

namespace {

template <typename T, bool GATHER>
__global__ void k8_layout(const K8Args a) {
  const int nxh = a.nx / 2, nh = nxh + 1;
  const size_t plane = (size_t)a.ny * nh;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)a.N * plane) return;
  const int f = (int)(idx / plane);
  const size_t b = idx - (size_t)f * plane;
  const int ky = (int)(b / nh), kx = (int)(b - (size_t)ky * nh);
  const int k2 = ky % a.R, k1 = ky / a.R;
  V2<T>* ws = kx < nxh ? static_cast<V2<T>*>(a.ws_main) + (((size_t)f * a.R + k2) * a.L + k1) * nxh + kx
                       : static_cast<V2<T>*>(a.ws_nyq) + ((size_t)f * a.L + k1) * a.R + k2;
  V2<T>* sp = static_cast<V2<T>*>(a.spectra) + idx;
  const T sc = (T)a.scale;
  if (GATHER) {
    const V2<T> v = *ws;
    *sp = V2<T>{v.x * sc, v.y * sc};
  } else {
    const V2<T> v = *sp;
    *ws = V2<T>{v.x * sc, v.y * sc};
  }
}

template <bool GATHER>
hipError_t launch(const K8Args& a, int dtype, hipStream_t s) {
  const size_t total = (size_t)a.N * a.ny * (a.nx / 2 + 1);
  const dim3 block(256), grid((unsigned)((total + 255) / 256));
  if (dtype == 0)
    hipLaunchKernelGGL((k8_layout<float, GATHER>), grid, block, 0, s, a);
  else
    hipLaunchKernelGGL((k8_layout<double, GATHER>), grid, block, 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_k8_gather(const K8Args& a, int dtype, hipStream_t s) { return launch<true>(a, dtype, s); }
hipError_t launch_k8_scatter(const K8Args& a, int dtype, hipStream_t s) { return launch<false>(a, dtype, s); }

}  // namespace fftenkf
