// The analysis in the real sine basis (Section 4): orthonormal 2D DST-II
// coefficients through the 2D FFT of the analysis, by Makhoul's reordering.
//
// With y(j1, j2) = (-1)^(j1 + j2) x(j1, j2), the DST-II of x at (s1, s2) is the
// DCT-II of y at (n1-1-s1, n2-1-s2).  With v(j1, j2) = y(rho1(j1), rho2(j2)),
// rho(j) = 2j for j < n/2 and 2(n-1-j)+1 above, and V its unnormalised 2D DFT,
//   X(k1, k2) = 1/2 Re[ W1(k1) (W2(k2) V(k1, k2) + conj W2(k2) V(k1, -k2)) ],
//   W(k) = exp(-i pi k / (2n)),
// is the unnormalised DCT-II of y, and conversely
//   V(k1, k2) = conj(W1(k1) W2(k2)) [ X(k1, k2) - X(n1-k1, n2-k2) - i (X(n1-k1, k2) + X(k1, n2-k2)) ]
// with X = 0 at index n.  The orthonormal coefficient is alpha1(k1) alpha2(k2)
// X(k1, k2), alpha(0) = sqrt(1/n), alpha(k > 0) = sqrt(2/n).
//
// Launches: sweep 1 reading x through the reordering (x -> V, members and d)
// and the statistics mode of sweep 2 (V left in the workspace), dst_quad (per
// mirror set of bins: V -> X -> eq. (2)-(3) in the sine basis -> X^a -> V^a),
// the inverse-only mode of sweep 2 and sweep 3 writing through the reordering
// (V^a -> x^a).
#include <hip/hip_runtime.h>
#include <math.h>

#include "fft_core.hpp"
#include "kernels.hpp"
#include "philox.hpp"
#include "spectral_unit.hpp"

namespace fftenkf {

namespace {


template <typename T> __device__ __forceinline__ void sincospi_t(T x, T* s, T* c);
template <> __device__ __forceinline__ void sincospi_t<float>(float x, float* s, float* c) { sincospif(x, s, c); }
template <> __device__ __forceinline__ void sincospi_t<double>(double x, double* s, double* c) { sincospi(x, s, c); }

// W(k) = exp(-i pi k / (2n))
template <typename T>
__device__ __forceinline__ cx<T> wq(int k, int n) {
  T s, c;
  sincospi_t<T>(T(k) / T(2 * n), &s, &c);
  return cx<T>{c, -s};
}

template <typename T> __device__ __forceinline__ T tiny_t();
template <> __device__ __forceinline__ float tiny_t<float>() { return 1.17549435e-38f; }
template <> __device__ __forceinline__ double tiny_t<double>() { return 2.2250738585072014e-308; }

// V(ky, kx) of field 0 in the transformed layout of sweep 2 (field f is f *
// fstride elements further): its slot and how it is read (bin_slot).
template <typename T>
struct SpecRef {
  V2<T>* p;
  int op;
  __device__ __forceinline__ cx<T> load(size_t off) const {
    const cx<T> v = from2<T>(p[off]);
    return op == 0 ? v : op == 1 ? conj(v) : op == 2 ? cx<T>{v.re, T(0)} : cx<T>{v.im, T(0)};
  }
  // only the bin that owns the slot writes it (a pair slot: its own part)
  __device__ __forceinline__ void store(size_t off, cx<T> v) const {
    if (op == 0) p[off] = to2<T>(v);
    else if (op == 2) reinterpret_cast<T*>(p + off)[0] = v.re;
    else if (op == 3) reinterpret_cast<T*>(p + off)[1] = v.re;
  }
};
template <typename T>
__device__ __forceinline__ SpecRef<T> spectrum_at(const K9Args& a, int ky, int kx) {
  const int nxh = a.nx / 2;
  const BinSlot sl = bin_slot(ky, kx, a.R, a.L, nxh);
  return SpecRef<T>{static_cast<V2<T>*>(a.ws_main) + ((size_t)sl.k2 * a.L + sl.k1) * nxh + sl.col, sl.op};
}

// One thread per mirror set {a, n1-a} x {b, n2-b}, 0 <= a <= n1/2, 0 <= b <= n2/2.
// The thread works on the unnormalised coefficients X = s / alpha: eq. (2)
// takes alpha^2 var(X), and eq. (3) becomes
//   X^a_k = X_k + g (X_d - X_k) + (g sqrt(R_dst) / alpha) z_k.
// Perturbations: Philox counter (bin, k div 4, 1, 0) at DST bin (s1, s2), bin =
// s1 * nx + s2; Box-Muller on words (x0, x1) gives members 4q and 4q + 1, on
// (x2, x3) members 4q + 2 and 4q + 3.
template <typename T, int NMAX>
__global__ __launch_bounds__(256) void dst_quad(const K9Args a) {
  static_assert(NMAX % 4 == 0, "member bucket must be a multiple of 4");
  const int n1 = a.ny, n2 = a.nx;
  const int hb = n2 / 2 + 1;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (n1 / 2 + 1) * hb) return;
  const int qa = idx / hb, qb = idx - qa * hb;
  const int ma = (n1 - qa) % n1, mb = (n2 - qb) % n2;  // the mirror rows and columns
  const bool da = ma != qa, db = mb != qb;             // distinct mirror point
  const int N = a.N;
  // the four points: 0 (qa, qb), 1 (ma, qb), 2 (qa, mb), 3 (ma, mb).  For a
  // distinct mirror m = n - k, W(m) = -i conj W(k); a coinciding mirror point
  // is never used.
  const cx<T> w1 = wq<T>(qa, n1), w2 = wq<T>(qb, n2);
  const cx<T> W1[4] = {w1, mul_mi(conj(w1)), w1, mul_mi(conj(w1))};
  const cx<T> W2[4] = {w2, w2, mul_mi(conj(w2)), mul_mi(conj(w2))};
  const int pk1[4] = {qa, ma, qa, ma}, pk2[4] = {qb, qb, mb, mb};
  const T r1 = sqrt(T(1) / T(n1)), r1b = sqrt(T(2) / T(n1)), r2 = sqrt(T(1) / T(n2)), r2b = sqrt(T(2) / T(n2));
  T alpha[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) alpha[p] = (pk1[p] == 0 ? r1 : r1b) * (pk2[p] == 0 ? r2 : r2b);
  // the two stored points of every field
  const size_t fstride = (size_t)a.R * a.L * (n2 / 2);
  const SpecRef<T> va = spectrum_at<T>(a, qa, qb);
  const SpecRef<T> vm = spectrum_at<T>(a, ma, qb);

  // X of every field at the four points (member k in row k, d in row NMAX;
  // padding rows are never read)
  T X[NMAX + 1][4];
#pragma unroll
  for (int f = 0; f <= NMAX; ++f) {
    if (f < N || f == NMAX) {
      const size_t off = (size_t)(f == NMAX ? N : f) * fstride;
      const cx<T> Vab = va.load(off);
      const cx<T> Vmb = vm.load(off);
      // V at (qa, -qb) = conj V(ma, qb); at (ma, -qb) = conj V(qa, qb)
      const cx<T> Vp[4] = {Vab, Vmb, conj(Vmb), conj(Vab)};
      const cx<T> Vn[4] = {conj(Vmb), conj(Vab), Vab, Vmb};  // V at (k1, -k2) of each point
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const cx<T> z = W1[p] * (W2[p] * Vp[p] + conj(W2[p]) * Vn[p]);
        X[f][p] = T(0.5) * z.re;
      }
    }
  }
  // eq. (2)-(3) at each distinct point; the DST bin is (n1-1-k1, n2-1-k2)
  const bool live[4] = {true, da, db, da && db};
  const T* __restrict__ Rd = static_cast<const T*>(a.R_dst);
  const T invN = T(1) / T(N), invN1 = T(1) / T(N - 1);
  static_for<0, 4>([&](auto PI) __attribute__((always_inline)) {
    constexpr int p = decltype(PI)::value;
    if (!live[p]) return;
    const int s1 = n1 - 1 - pk1[p], s2 = n2 - 1 - pk2[p];
    if (a.dbg_coeffs != nullptr) {  // test export: the sine coefficients of every field
      T* dc = static_cast<T*>(a.dbg_coeffs);
      const size_t plane = (size_t)n1 * n2, bin = (size_t)s1 * n2 + s2;
#pragma unroll
      for (int f = 0; f < NMAX; ++f)
        if (f < N) dc[f * plane + bin] = alpha[p] * X[f][p];
      dc[N * plane + bin] = alpha[p] * X[NMAX][p];
      return;
    }
    // deviations formed from X_f - X_0 (exactly zero for a collapsed ensemble)
    const T x0 = X[0][p];
    T mean = T(0);
#pragma unroll
    for (int f = 1; f < NMAX; ++f)
      if (f < N) mean += X[f][p] - x0;
    mean *= invN;
    T var = mean * mean;
#pragma unroll
    for (int f = 1; f < NMAX; ++f)
      if (f < N) var += ((X[f][p] - x0) - mean) * ((X[f][p] - x0) - mean);
    const T c = alpha[p] * alpha[p] * var * invN1;
    const T r = Rd != nullptr ? Rd[(size_t)s1 * n2 + s2] : T(a.r_scalar);
    const T den = c + r;
    const T g = den < tiny_t<T>() ? T(0) : c / den;
    const T ge = g * sqrt(r) / alpha[p];
    const T xd = X[NMAX][p];
    const uint32_t ctr0 = (uint32_t)(s1 * n2 + s2);
    static_for<0, NMAX / 4>([&](auto QI) __attribute__((always_inline)) {
      constexpr int q = decltype(QI)::value;
      if (4 * q < N) {
        const u32x4 w = philox4x32_10(u32x4{ctr0, (uint32_t)q, 1u, 0u}, a.key0, a.key1);
        T z[4];
        box_muller<T>(w.x0, w.x1, z[0], z[1]);
        if (4 * q + 2 < N) box_muller<T>(w.x2, w.x3, z[2], z[3]);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (4 * q + j < N) X[4 * q + j][p] += g * (xd - X[4 * q + j][p]) + ge * z[j];
      }
    });
  });
  if (a.dbg_coeffs != nullptr) return;
  // back to V at the two stored points (qa, qb) and (ma, qb); a mirror point
  // that coincides with another holds that point's updated value
#pragma unroll
  for (int f = 0; f < NMAX; ++f) {
    if (f >= N) continue;
    T Y[4] = {X[f][0], X[f][1], X[f][2], X[f][3]};
    if (!da) {
      Y[1] = Y[0];
      Y[3] = Y[2];
    }
    if (!db) {
      Y[2] = Y[0];
      Y[3] = Y[1];
    }
    // X at index n (a mirror of row or column 0) is zero
    const T x_ab = Y[0];
    const T x_mr = qa == 0 ? T(0) : Y[1];              // X(n1 - qa, qb)
    const T x_mc = qb == 0 ? T(0) : Y[2];              // X(qa, n2 - qb)
    const T x_mm = (qa == 0 || qb == 0) ? T(0) : Y[3];  // X(n1 - qa, n2 - qb)
    const size_t off = (size_t)f * fstride;
    va.store(off, conj(W1[0] * W2[0]) * cx<T>{x_ab - x_mm, -(x_mr + x_mc)});
    if (da) {
      // for the point (ma, qb): X(n1 - ma, .) = X(qa, .), never at index n
      const T y_ab = Y[1], y_mr = Y[0];
      const T y_mc = qb == 0 ? T(0) : Y[3];
      const T y_mm = qb == 0 ? T(0) : Y[2];
      vm.store(off, conj(W1[1] * W2[1]) * cx<T>{y_ab - y_mm, -(y_mr + y_mc)});
    }
  }
}

template <typename T, int NMAX>
hipError_t launch_quad(const K9Args& a, hipStream_t s) {
  const int total = (a.ny / 2 + 1) * (a.nx / 2 + 1);
  hipLaunchKernelGGL((dst_quad<T, NMAX>), dim3((total + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_quad_f32(const K9Args& a, hipStream_t s) {
  if (a.N <= 8) return launch_quad<float, 8>(a, s);
  if (a.N <= 12) return launch_quad<float, 12>(a, s);
  if (a.N <= 16) return launch_quad<float, 16>(a, s);
  if (a.N <= 20) return launch_quad<float, 20>(a, s);
  if (a.N <= 24) return launch_quad<float, 24>(a, s);
  return hipErrorInvalidValue;
}

hipError_t launch_quad_f64(const K9Args& a, hipStream_t s) {
  if (a.N <= 8) return launch_quad<double, 8>(a, s);
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_dst_quad(const K9Args& a, int dtype, hipStream_t s) {
  return dtype == 0 ? launch_quad_f32(a, s) : launch_quad_f64(a, s);
}

}  // namespace fftenkf
