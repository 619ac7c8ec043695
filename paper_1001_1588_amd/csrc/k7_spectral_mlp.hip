// Learned spectral covariance: a per-wavenumber perceptron on matrix cores.
//
// For every stored bin (ky, kx) of the half spectrum the input is the log
// sample spectrum of eq. (2) in the 5 x 5 wavenumber neighbourhood plus
// log(1 + |k|) (26 features, padded to 32); three hidden layers of 64 with ReLU
// and one output give y, and lambda_hat = mu exp(y), mu the mean of c_hat over
// the stored bins.  Features, weights and hidden activations are bfloat16,
// products accumulate in float32 (v_mfma_f32_16x16x16_bf16).
//
// Each layer is computed transposed, H^T = W^T X^T, with a 16-bin tile as the
// N dimension: the accumulator of output block m (lane l holds rows
// 16 m + 4 (l / 16) + j of column l % 16) is exactly the B operand of input
// block m of the next layer, so activations never leave registers.  The weight
// matrices W^T are the A operands and stay in registers for the whole kernel.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "kernels.hpp"

namespace fftenkf {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kIn = 26;      // features used
constexpr int kInPad = 32;   // features padded to two 16-wide blocks
constexpr int kWidth = 64;   // hidden width
constexpr int kBinsPerWave = 64;
constexpr int kThreads = 256;
constexpr float kEps = 1e-6f;

// float32 -> bfloat16, round to nearest, ties to even (finite inputs)
__device__ __forceinline__ short to_bf16(float x) {
  uint32_t b = __float_as_uint(x);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (short)(b >> 16);
}

__device__ __forceinline__ float bf16_to_f(short h) { return __uint_as_float(((uint32_t)(uint16_t)h) << 16); }

__device__ __forceinline__ f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// c_hat at a full-spectrum position (ky, kx) with 0 <= ky < ny, -2 <= kx <= nx/2 + 2
__device__ __forceinline__ float chat_full(const float* __restrict__ chat, int ky, int kx, int ny, int nx) {
  const int nh = nx / 2 + 1;
  if (kx < 0) kx += nx;
  if (kx > nx / 2) {  // mirror: c(ky, kx) = c(ny - ky, nx - kx)
    ky = (ny - ky) & (ny - 1);
    kx = nx - kx;
  }
  return chat[(size_t)ky * nh + kx];
}

}  // namespace

__global__ __launch_bounds__(kThreads) void k7_spectral_mlp(const K7Args a) {
  __shared__ float red[kThreads];
  __shared__ float s_bias[3][kWidth];
  __shared__ float s_w4[kWidth];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, grp = lane >> 4;  // MFMA column (bin in tile) and row group
  const int ny = a.ny, nx = a.nx, nh = nx / 2 + 1;
  const long total = (long)ny * nh;

  // mu: every block sums the per-block partials in the same fixed order
  float s = 0.f;
  for (int k = tid; k < a.n_partials; k += kThreads) s += a.partials[k];
  red[tid] = s;
  if (tid < kWidth) {
    s_bias[0][tid] = a.b1[tid];
    s_bias[1][tid] = a.b2[tid];
    s_bias[2][tid] = a.b3[tid];
    // the output layer multiplies bfloat16 weights
    s_w4[tid] = bf16_to_f(to_bf16(a.w4[tid]));
  }
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const float mu = red[0] / (float)total;
  if (blockIdx.x == 0 && tid == 0 && a.mu_out != nullptr) *a.mu_out = mu;
  const float inv_mu = 1.f / mu;
  const float b4 = a.b4[0];

  // A operands: W^T fragments.  Fragment (m, k) of a layer: lane holds
  // W^T[16 m + col][16 k + 4 grp + j] = W[16 k + 4 grp + j][16 m + col].
  bf16x4 A1[4][2], A2[4][4], A3[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int in = 16 * k + 4 * grp + j;
        A1[m][k][j] = in < kIn ? to_bf16(a.W1[in * kWidth + 16 * m + col]) : (short)0;
      }
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int in = 16 * k + 4 * grp + j;
        A2[m][k][j] = to_bf16(a.W2[in * kWidth + 16 * m + col]);
        A3[m][k][j] = to_bf16(a.W3[in * kWidth + 16 * m + col]);
      }
  }

  const long wave_base = ((long)blockIdx.x * (kThreads / 64) + wave) * kBinsPerWave;
#pragma unroll 1
  for (int tile = 0; tile < kBinsPerWave / 16; ++tile) {
    const long bin = wave_base + tile * 16 + col;
    const bool live = bin < total;
    const long b = live ? bin : 0;
    const int ky = (int)(b / nh), kx = (int)(b - (long)ky * nh);

    // B operand of layer 1: features 16 k + 4 grp + j of this lane's bin
    bf16x4 X[2];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int f = 16 * k + 4 * grp + j;
        float v = 0.f;
        if (f < 25) {
          const int dy = f / 5 - 2, dx = f % 5 - 2;
          const float c = chat_full(a.chat, (ky + dy + ny) & (ny - 1), kx + dx, ny, nx);
          v = logf(c * inv_mu + kEps);
        } else if (f == 25) {
          const int kyw = ky < ny - ky ? ky : ny - ky;
          v = log1pf(sqrtf((float)kyw * (float)kyw + (float)kx * (float)kx));
        }
        X[k][j] = to_bf16(v);
      }

    // hidden layers
    bf16x4 H[4];
    {
      f32x4 D[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        D[m] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < 2; ++k) D[m] = mfma(A1[m][k], X[k], D[m]);
#pragma unroll
        for (int j = 0; j < 4; ++j) H[m][j] = to_bf16(fmaxf(D[m][j] + s_bias[0][16 * m + 4 * grp + j], 0.f));
      }
    }
    {
      f32x4 D[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        D[m] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < 4; ++k) D[m] = mfma(A2[m][k], H[k], D[m]);
      }
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int j = 0; j < 4; ++j) H[m][j] = to_bf16(fmaxf(D[m][j] + s_bias[1][16 * m + 4 * grp + j], 0.f));
    }
    float y;
    {
      f32x4 D[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        D[m] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < 4; ++k) D[m] = mfma(A3[m][k], H[k], D[m]);
      }
      // output layer: this lane's 16 rows, then the four row groups of the column
      float part = 0.f;
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int r = 16 * m + 4 * grp + j;
          const float h = bf16_to_f(to_bf16(fmaxf(D[m][j] + s_bias[2][r], 0.f)));
          part += s_w4[r] * h;
        }
      part += __shfl_xor(part, 16);
      part += __shfl_xor(part, 32);
      y = part + b4;
    }
    if (live && grp == 0) a.lam[bin] = mu * expf(y);
  }
}

hipError_t launch_k7(const K7Args& a, hipStream_t s) {
  const long total = (long)a.ny * (a.nx / 2 + 1);
  const long per_block = (long)(kThreads / 64) * kBinsPerWave;
  const dim3 grid((unsigned)((total + per_block - 1) / per_block)), block(kThreads);
  hipLaunchKernelGGL(k7_spectral_mlp, grid, block, 0, s, a);
  return hipGetLastError();
}

}  // namespace fftenkf
