// Learned spectral covariance: a per-wavenumber perceptron on matrix cores.
//
// For every stored bin (ky, kx) of the half spectrum the input is the log
// sample spectrum of eq. (2) in the 5 x 5 wavenumber neighbourhood plus
// log(1 + |k|) (26 features, padded to 32); three hidden layers of 64 with ReLU
// and one output give y, and lambda_hat = mu exp(y), mu the mean of c_hat over
// the stored bins.  Features, weights and hidden activations are bfloat16
// (v_cvt_pk_bf16_f32, round to nearest even), products accumulate in float32
// (v_mfma_f32_16x16x32_bf16).
//
// Each layer is computed transposed, H^T = W^T X^T, with 16 bins as the N
// dimension.  The accumulator of output block m holds, in lane l, hidden units
// h = 16 m + 4 (l / 16) + r (r < 4) of bin l % 16.  The next layer takes its
// B operand for K block kb from the accumulators of blocks 2 kb and 2 kb + 1 of
// the same lane, which puts hidden unit h at K position
//   kpos(h) = 32 (m / 2) + 8 (l / 16) + 4 (m % 2) + r;
// the A operand (W^T, held in registers) is loaded in that same K order, so the
// activations never leave registers and need no exchange between lanes.
//
// The grid is persistent: a block loads the weights once and walks tiles of
// 8 x 32 bins (each wave: two rows, as two pairs of 16-bin tiles).  Each tile's bfloat16 log spectrum, with a 2-bin halo (columns
// beyond nx/2 taken from the mirror c_hat(-ky, -kx)), goes to one of two LDS
// buffers; the next tile's c_hat values are loaded into registers while the
// current tile is computed.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "kernels.hpp"

namespace fftenkf {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kIn = 26;     // features used
constexpr int kWidth = 64;  // hidden width
constexpr int kThreads = 256;
constexpr int kTY = 8, kTX = 32;             // bins of a block tile (4 waves x 2 rows x 32 columns)
constexpr int kHY = kTY + 4, kHX = kTX + 4;  // the tile with its halo
constexpr int kHalo = kHY * kHX;             // 432 <= 2 * kThreads
constexpr float kEps = 1e-6f;
constexpr float kLn2 = 0.69314718055994530942f;
constexpr int kMaxBlocks = 512;  // two resident blocks on each of 256 compute units
static_assert(kHalo <= 2 * kThreads, "two halo values per thread");

__device__ __forceinline__ __bf16 bf(float x) { return (__bf16)x; }

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// natural logarithm by the hardware log2 (arguments here are >= 1e-6, normal)
__device__ __forceinline__ float ln(float x) { return __builtin_amdgcn_logf(x) * kLn2; }

// hidden unit held at K position 8 g + e of K block kb by a lane of row group g
__device__ __forceinline__ int hidden_at(int kb, int g, int e) { return 16 * (2 * kb + (e >> 2)) + 4 * g + (e & 3); }

// one hidden layer on two 16-bin tiles: D_m = b + W^T X for the 4 output
// blocks of each (the accumulators start at the bias; the two tiles' products
// are issued together so one tile's epilogue overlaps the other's products),
// rounded to bfloat16, then ReLU, packed as the next layer's B operands.  ReLU
// acts on the rounded bits as a signed 16-bit maximum with 0: rounding is
// monotone and keeps the sign, so this equals rounding relu(D).
template <int KB>
__device__ __forceinline__ void layer2(const bf16x8 (&A)[4][KB], const bf16x8 (&X0)[KB], const bf16x8 (&X1)[KB],
                                       const float* bias, int grp, bf16x8 (&H0)[2], bf16x8 (&H1)[2]) {
  f32x4 D0[4], D1[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    D0[m] = *reinterpret_cast<const f32x4*>(bias + 16 * m + 4 * grp);
    D1[m] = D0[m];
  }
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      D0[m] = mfma(A[m][k], X0[k], D0[m]);
      D1[m] = mfma(A[m][k], X1[k], D1[m]);
    }
  u32x4 w0[2], w1[2];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const bf16x2 p0 = __builtin_convertvector((f32x2{D0[m][2 * q], D0[m][2 * q + 1]}), bf16x2);
      const bf16x2 p1 = __builtin_convertvector((f32x2{D1[m][2 * q], D1[m][2 * q + 1]}), bf16x2);
      w0[m >> 1][2 * (m & 1) + q] = __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s16x2, p0), s16x2(0)));
      w1[m >> 1][2 * (m & 1) + q] = __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s16x2, p1), s16x2(0)));
    }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    H0[i] = __builtin_bit_cast(bf16x8, w0[i]);
    H1[i] = __builtin_bit_cast(bf16x8, w1[i]);
  }
}

}  // namespace

__global__ __launch_bounds__(kThreads, 2) void k7_spectral_mlp(const K7Args a) {
  __shared__ float red[kThreads];
  __shared__ __attribute__((aligned(16))) float s_bias[3][kWidth];
  __shared__ __bf16 s_x[2][kHalo];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, grp = lane >> 4;  // MFMA column (bin in tile) and row group
  const int ny = a.ny, nx = a.nx, nh = nx / 2 + 1;
  const long total = (long)ny * nh;
  const float* __restrict__ chat = a.chat;

  // mu: every block sums the per-block partials in the same fixed order
  float s = 0.f;
  for (int k = tid; k < a.n_partials; k += kThreads) s += a.partials[k];
  red[tid] = s;
  if (tid < kWidth) {
    s_bias[0][tid] = a.b1[tid];
    s_bias[1][tid] = a.b2[tid];
    s_bias[2][tid] = a.b3[tid];
  }
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const float mu = red[0] / (float)total;
  if (blockIdx.x == 0 && tid == 0 && a.mu_out != nullptr) *a.mu_out = mu;
  // the features divide by mu: where it is not a positive normal number (no
  // spread anywhere, or an overflow; NaN fails both tests) the estimate falls
  // back to the plain sample spectrum
  if (!(mu >= 1.17549435e-38f && mu <= 3.40282347e+38f)) {
    for (long b = (long)blockIdx.x * kThreads + tid; b < total; b += (long)gridDim.x * kThreads) a.lam[b] = chat[b];
    return;
  }
  const float inv_mu = 1.f / mu;
  const float b4 = a.b4[0];

  // A operands.  Layer 1: lane holds W1[8 grp + e][16 m + col] (feature f =
  // 8 grp + e at K position f); layers 2, 3: W[hidden_at(kb, grp, e)][16 m + col].
  bf16x8 A1[4][1], A2[4][2], A3[4][2], A4[1][2];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int f = 8 * grp + e;
      A1[m][0][e] = bf(f < kIn ? a.W1[f * kWidth + 16 * m + col] : 0.f);
    }
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int h = hidden_at(kb, grp, e);
        A2[m][kb][e] = bf(a.W2[h * kWidth + 16 * m + col]);
        A3[m][kb][e] = bf(a.W3[h * kWidth + 16 * m + col]);
      }
  }
  // output layer as one more product: row 0 of A4 is w4 (same K order), rows
  // 1..15 are zero, so row 0 of the accumulator is y for the 16 bins
#pragma unroll
  for (int kb = 0; kb < 2; ++kb)
#pragma unroll
    for (int e = 0; e < 8; ++e) A4[0][kb][e] = bf(col == 0 ? a.w4[hidden_at(kb, grp, e)] : 0.f);

  // this lane's features f = 8 grp + e: LDS offset and bit masks selecting the
  // neighbourhood value (f < 25), |k| (f = 25) or zero
  int foff[8];
  uint32_t mnb[8], mk[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int f = 8 * grp + e;
    foff[e] = f < 25 ? (f / 5) * kHX + (f % 5) : 0;
    mnb[e] = f < 25 ? 0xFFFFu : 0u;
    mk[e] = f == 25 ? 0xFFFFu : 0u;
  }

  // the (up to) two halo positions this thread loads for every tile
  const int hy0 = tid / kHX, hx0 = tid - hy0 * kHX;
  const bool has1 = tid + kThreads < kHalo;
  const int hy1 = (tid + kThreads) / kHX, hx1 = (tid + kThreads) - hy1 * kHX;
  const int ntx = (nh + kTX - 1) / kTX;
  const int ntiles = (ny / kTY) * ntx;
  auto halo_index = [&](int tile, int hy, int hx) -> uint32_t {
    const int ty0 = (tile / ntx) * kTY, tx0 = (tile % ntx) * kTX;
    int ky = (ty0 + hy - 2) & (ny - 1);
    int kx = (tx0 + hx - 2) & (nx - 1);
    if (kx > nx / 2) {  // c_hat is even: c(ky, kx) = c(-ky, -kx)
      ky = (ny - ky) & (ny - 1);
      kx = nx - kx;
    }
    return (uint32_t)ky * (uint32_t)nh + (uint32_t)kx;
  };

  int tile = blockIdx.x;
  float c0 = 0.f, c1 = 0.f;
  if (tile < ntiles) {
    c0 = chat[halo_index(tile, hy0, hx0)];
    if (has1) c1 = chat[halo_index(tile, hy1, hx1)];
  }
  for (int buf = 0; tile < ntiles; tile += gridDim.x, buf ^= 1) {
    __bf16* sx = s_x[buf];
    sx[tid] = bf(ln(c0 * inv_mu + kEps));
    if (has1) sx[tid + kThreads] = bf(ln(c1 * inv_mu + kEps));
    __syncthreads();  // also: every thread is done with the buffer written next
    const int next = tile + gridDim.x;
    if (next < ntiles) {  // prefetch, consumed at the top of the next iteration
      c0 = chat[halo_index(next, hy0, hx0)];
      if (has1) c1 = chat[halo_index(next, hy1, hx1)];
    }
    const int ty0 = (tile / ntx) * kTY, tx0 = (tile % ntx) * kTX;

#pragma unroll 1
    for (int t = 0; t < 2; ++t) {
      const int row = 2 * wave + t;
      const int ky = ty0 + row;
      const int kyw = ky < ny - ky ? ky : ny - ky;
      bf16x8 X[2][1];
      int kxs[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int cb = 16 * u;
        const int kx = tx0 + cb + col;
        kxs[u] = kx;
        const float kmag = __builtin_amdgcn_sqrtf((float)kyw * (float)kyw + (float)kx * (float)kx);
        const uint32_t kbits = __builtin_bit_cast(uint16_t, bf(ln(1.f + kmag)));
        const uint16_t* xs = reinterpret_cast<const uint16_t*>(sx) + row * kHX + cb + col;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const uint32_t v = xs[foff[e]];
          X[u][0][e] = __builtin_bit_cast(__bf16, (uint16_t)((v & mnb[e]) | (kbits & mk[e])));
        }
      }
      bf16x8 Ha[2], Hb[2], Ga[2], Gb[2];  // the two tiles' activations
      layer2<1>(A1, X[0], X[1], s_bias[0], grp, Ha, Hb);
      layer2<2>(A2, Ha, Hb, s_bias[1], grp, Ga, Gb);
      layer2<2>(A3, Ga, Gb, s_bias[2], grp, Ha, Hb);
      // output layer: y = b4 + w4 . h3 in row 0, held by the lanes of row group 0
      f32x4 Y0 = f32x4{b4, b4, b4, b4}, Y1 = Y0;
      Y0 = mfma(A4[0][0], Ha[0], Y0);
      Y1 = mfma(A4[0][0], Hb[0], Y1);
      Y0 = mfma(A4[0][1], Ha[1], Y0);
      Y1 = mfma(A4[0][1], Hb[1], Y1);
      if (grp == 0 && kxs[0] < nh) a.lam[(size_t)ky * nh + kxs[0]] = mu * expf(Y0[0]);
      if (grp == 0 && kxs[1] < nh) a.lam[(size_t)ky * nh + kxs[1]] = mu * expf(Y1[0]);
    }
  }
}

hipError_t launch_k7(const K7Args& a, hipStream_t s) {
  const int nh = a.nx / 2 + 1;
  const int ntiles = (a.ny / kTY) * ((nh + kTX - 1) / kTX);
  const dim3 grid((unsigned)(ntiles < kMaxBlocks ? ntiles : kMaxBlocks)), block(kThreads);
  hipLaunchKernelGGL(k7_spectral_mlp, grid, block, 0, s, a);
  return hipGetLastError();
}

}  // namespace fftenkf

