// Test exports only: copy half spectra between the caller's [N][ny][nx/2+1]
// layout and the transformed layout of the spectral sweep, one thread per bin.
#include <hip/hip_runtime.h>

#include "fft_core.hpp"
#include "kernels.hpp"
#include "spectral_unit.hpp"

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
  const BinSlot sl = bin_slot(ky, kx, a.R, a.L, nxh);
  V2<T>* ws = static_cast<V2<T>*>(a.ws_main) + (((size_t)f * a.R + sl.k2) * a.L + sl.k1) * nxh + sl.col;
  V2<T>* sp = static_cast<V2<T>*>(a.spectra) + idx;
  const T sc = (T)a.scale;
  if (GATHER) {
    const V2<T> v = *ws;
    const V2<T> w = sl.op == 0 ? v : sl.op == 1 ? V2<T>{v.x, -v.y} : sl.op == 2 ? V2<T>{v.x, T(0)} : V2<T>{v.y, T(0)};
    *sp = V2<T>{w.x * sc, w.y * sc};
  } else {
    V2<T> v = *sp;
    if (sl.op == 0 && (kx == 0 || kx == nxh)) {
      // the Hermitian part (v + conj v(ny - ky, kx)) / 2 of a kx = 0 or nx/2 bin,
      // as a c2r transform takes it
      const V2<T> w = static_cast<const V2<T>*>(a.spectra)[(size_t)f * plane + (size_t)((a.ny - ky) % a.ny) * nh + kx];
      v = V2<T>{T(0.5) * (v.x + w.x), T(0.5) * (v.y - w.y)};
    }
    T* c = reinterpret_cast<T*>(ws);
    if (sl.op == 0) *ws = V2<T>{v.x * sc, v.y * sc};
    else if (sl.op == 2) c[0] = v.x * sc;  // the two real bins of a pair slot: one part each
    else if (sl.op == 3) c[1] = v.x * sc;
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
