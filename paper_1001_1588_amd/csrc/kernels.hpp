// Internal launch interface of the three sweeps of one analysis.
//
// Grid factorisation: ny = R * L.  A row index is y = y1 + L * y2 and a
// frequency ky = k2 + R * k1 (y1, k1 < L; y2, k2 < R).  Then
//   X[k2 + R k1] = sum_y1 W_L^(y1 k1) * [ W_ny^(y1 k2) * sum_y2 W_R^(y2 k2) x[y1 + L y2] ],
// so the first sweep (k1) does the x transform of R rows y1 + L*y2 plus the
// radix-R stage over y2 and the W_ny^(y1 k2) twiddle; the second sweep (k2) does
// the remaining length-L transform over y1 for each (k2, kx), the statistics,
// the gain, the perturbations and the update, then the inverse length-L
// transform; the third sweep (k3) undoes the first.
//
// Workspace (complex, dtype T): [NF][R][L][nx/2], element (f, k2, y1, kx), with
// NF = N + 1 fields (the N members, then the data d).  The Nyquist column
// kx = nx/2 has no storage of its own: it is folded into column kx = 0
// (spectral_unit.hpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace fftenkf {

struct K1Args {
  const void* members;  // [N][ny][nx]
  const void* data;     // [n_data][ny][nx]: fields N .. N + n_data - 1
  int N, ny, nx, R, L;
  void* ws_main;
  const void* tab;  // W_4096^k table of dtype's complex type (device)
  int sine = 0;     // 1: transform the sine-basis reordering of the fields (dst_rho)
  int n_data = 1;   // data fields after the N member fields
};

// K2_STATS: forward transforms and eq. (2) only -- writes c_hat to chat_map,
//   one partial sum of c_hat per block to partials, and the transformed fields
//   back in place.
// K2_CHAT: K2_STATS without writing the fields back (the learned analysis
//   transforms them again in its K2_ANALYZE pass).
// In any mode a non-null lam_map replaces eq. (2) in the gain: the covariance
//   eigenvalues are read from it (an estimate, or a prescribed spectrum).
// K2_INVERSE: starts from transformed fields and only applies the inverse
//   length-L transforms (the c2r test export).
// Only K2_ANALYZE runs in the single-pass kernel variant; every other mode is
// compiled into a separate variant, so the analysis kernel carries none of their code.
enum K2Mode {
  K2_ANALYZE = 0,
  K2_DEBUG_SPECTRA = 1,
  K2_DEBUG_PERTURB = 2,
  K2_STATS = 3,
  K2_CHAT = 4,
  K2_INVERSE = 5
};

struct K2Args {
  void* ws_main;
  uint32_t main_bytes;  // size of the workspace's spectral region (below 2^31)
  const void* R_spec;  // [ny][nx/2+1] or nullptr
  double r_scalar;
  int N, ny, nx, R, L, C, units;
  int group_xcd;  // G > 1: blocks b, b+8, .., b+8(G-1) take G adjacent kx chunks of one k2
  uint32_t key0, key1;
  int mode;
  void* dbg_chat;  // [ny][nx/2+1] real
  void* dbg_gain;  // [ny][nx/2+1] real
  void* dbg_spec;  // [N+1][ny][nx/2+1] complex, or nullptr
  void* dbg_e;     // [N][ny][nx/2+1] complex
  void* chat_map;  // [ny][nx/2+1] real (K2_STATS)
  void* partials;  // [units] float (K2_STATS)
  const void* lam_map;  // [ny][nx/2+1] real, or nullptr
  const void* tab;
};

// Spectral sweep of an M-block state whose first K blocks are observed
// (k10_observed.hpp): member k of block j is field k * M + j, the data of
// observed block o is field N * M + o; the other fields as in K2Args.
constexpr int kMaxObserved = 3;
struct K10Args {
  void* ws_main;
  const void* R_spec;          // [K][ny][nx/2+1] or nullptr
  double r_obs[kMaxObserved];  // R_o = r_obs[o] I when R_spec is nullptr
  int N, M, K, ny, nx, R, L, C, units, group_xcd;
  uint32_t key0, key1;
  const void* tab;
};

// A batch of analyses with one member count, dtype and grid, run by the same
// sweep kernels with blockIdx.y selecting the analysis.  Passed by value as a
// kernel argument (kMaxBatch analyses per launch), so a captured graph keeps it.
struct BatchFilter {
  const void* members;  // [N][ny][nx]
  const void* data;     // [ny][nx]
  const void* R_spec;   // [ny][nx/2+1] or nullptr
  void* out;            // [N][ny][nx]
  void* ws_main;
  double r_scalar;
  uint32_t key0, key1;
};
constexpr int kMaxBatch = 40;
struct BatchArgs {
  int count, N, ny, nx, L;
  const void* tab;
  K2Args k2;  // the shared part of sweep 2's arguments (mode K2_ANALYZE)
  BatchFilter f[kMaxBatch];
};

struct K3Args {
  const void* ws_main;
  int N, ny, nx, R, L;
  void* out;  // [N][ny][nx]
  const void* tab;
  int sine;  // 1: write the result back through the sine-basis reordering (dst_rho)
};

// The reordering of the sine-basis analysis (Makhoul): the transformed field is
// v(j1, j2) = (-1)^(i1 + i2) x(i1, i2) with i = dst_rho(j, n), i.e. the even
// indices in order, then the odd ones in reverse.
__host__ __device__ __forceinline__ int dst_rho(int j, int n) { return j < n / 2 ? 2 * j : 2 * (n - 1 - j) + 1; }

// K2 geometry chosen for a given length L (shared by host planning and kernels).
constexpr int k2_points(int L) { return L < 4 ? L : 4; }
constexpr int k2_threads_target = 256;

// Largest member count held in registers by the fused spectral sweep.
constexpr int kMaxMembersF32 = 24;
constexpr int kMaxMembersF64 = 8;
// The sweep of a state with K observed blocks holds K + 1 register sets of
// members: up to 12 (float32) or 4 (float64) members with one observed block,
// 8 or 4 with two or three.
constexpr int kMaxMembersMultiF32 = 12;
constexpr int kMaxMembersMultiF64 = 4;
constexpr int kMaxMembersObsF32 = 8;
constexpr int kMaxMembersObsF64 = 4;
constexpr int kMaxStateBlocks = 64;  // blocks of the multi-block analysis

hipError_t launch_k1_f32(const K1Args& a, hipStream_t s);
hipError_t launch_k1_f64(const K1Args& a, hipStream_t s);
hipError_t launch_k2_f32(const K2Args& a, hipStream_t s);
hipError_t launch_k2_f64(const K2Args& a, hipStream_t s);
hipError_t launch_k10(const K10Args& a, int dtype, hipStream_t s);
hipError_t launch_k3_f32(const K3Args& a, hipStream_t s);
hipError_t launch_k3_f64(const K3Args& a, hipStream_t s);

// Learned spectral covariance (float32): lambda_hat per stored bin from the
// sample spectrum c_hat by a perceptron on matrix cores.
struct K7Args {
  const float* chat;      // [ny][nx/2+1]
  const float* partials;  // [n_partials] partial sums of chat
  int n_partials;
  int ny, nx;
  const float* W1;  // [26][64]
  const float* b1;  // [64]
  const float* W2;  // [64][64]
  const float* b2;  // [64]
  const float* W3;  // [64][64]
  const float* b3;  // [64]
  const float* w4;  // [64]
  const float* b4;  // [1]
  float* lam;       // [ny][nx/2+1]
  float* mu_out;    // [1] or nullptr
};
hipError_t launch_k7(const K7Args& a, hipStream_t s);

// Test exports: move N half spectra ([N][ny][nx/2+1] complex, scaled by
// `scale`) out of / into the transformed layout the spectral sweep leaves in
// the workspace ([f][k2][k1][kx < nx/2], ky = k2 + R k1, the kx = 0 and
// kx = nx/2 columns folded as bin_slot describes).  The scatter writes only the
// slot-owning bins: the kx = 0 and nx/2 bins above ny/2 are implied.
struct K8Args {
  void* ws_main;
  int N, ny, nx, R, L;
  double scale;
  void* spectra;
};
hipError_t launch_k8_gather(const K8Args& a, int dtype, hipStream_t s);
hipError_t launch_k8_scatter(const K8Args& a, int dtype, hipStream_t s);

// The analysis in the sine basis (k9_dst.hip): the per-bin kernel reads and
// writes the transformed fields in the workspace layout of K2Args.
struct K9Args {
  void* ws_main;
  const void* R_dst;  // [ny][nx] eigenvalues of R in the sine basis, or nullptr
  double r_scalar;
  int N, ny, nx, R, L;
  uint32_t key0, key1;
  void* dbg_coeffs;  // test export: [N+1][ny][nx] orthonormal sine coefficients, or nullptr
  const void* tab = nullptr;  // W_4096^k (the fused sweep)
  uint32_t main_bytes = 0;    // size of the spectral region (the fused sweep)
  int group_xcd = 1;          // the fused sweep's XCD grouping of blocks sharing 128-byte lines
};
hipError_t launch_dst_quad(const K9Args& a, int dtype, hipStream_t s);
// The sine-basis analysis as one spectral sweep (k11_dst_fused.hpp) for the
// shapes it takes (L >= 16, nx/2 a multiple of 512 / L); hipErrorNotSupported
// otherwise.
hipError_t launch_k11(const K9Args& a, int dtype, hipStream_t s);
bool k11_supports(int L, int nx);

// Device address of the W_4096^k table (float2 for dtype 0, double2 for 1) on
// the current device, filled from float64 host values on first use.
hipError_t twiddle_table(int dtype, const void** out);

// Supported member counts of the spectral sweep are grouped in buckets of
// register arrays; returns the bucket for N, or 0 if N is too large.
int k2_member_bucket(int dtype, int N);

}  // namespace fftenkf
