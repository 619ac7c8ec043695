// Twiddle tables W_4096^k = exp(-2 pi i k / 4096), k < 4096, one per precision, in
// static device memory.  Values are computed in float64 on the host and rounded
// once to the table's precision.  Each device gets its own copy of the arrays;
// their device addresses come from hipGetSymbolAddress on that device.
#include <math.h>

#include <mutex>

#include "fft_core.hpp"
#include "kernels.hpp"

namespace fftenkf {

__device__ float2 g_twiddle_f32[kTwiddleN];
__device__ double2 g_twiddle_f64[kTwiddleN];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
const void* g_addr[kMaxDevices][2];
}  // namespace

hipError_t twiddle_table(int dtype, const void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices || dtype < 0 || dtype > 1) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_addr[dev][dtype] == nullptr) {
    static float2 hf[kTwiddleN];
    static double2 hd[kTwiddleN];
    for (int k = 0; k < kTwiddleN; ++k) {
      const double a = 2.0 * M_PI * (double)k / (double)kTwiddleN;
      hd[k] = make_double2(cos(a), -sin(a));
      hf[k] = make_float2((float)hd[k].x, (float)hd[k].y);
    }
    void* p = nullptr;
    if (dtype == 0) {
      e = hipMemcpyToSymbol(HIP_SYMBOL(g_twiddle_f32), hf, sizeof(hf));
      if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_twiddle_f32));
    } else {
      e = hipMemcpyToSymbol(HIP_SYMBOL(g_twiddle_f64), hd, sizeof(hd));
      if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_twiddle_f64));
    }
    if (e != hipSuccess) return e;
    g_addr[dev][dtype] = p;
  }
  *out = g_addr[dev][dtype];
  return hipSuccess;
}

}  // namespace fftenkf
