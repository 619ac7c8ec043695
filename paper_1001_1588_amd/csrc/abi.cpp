// C ABI of the FFT EnKF analysis: argument validation, planning and dispatch
// of the three sweeps onto the caller's stream.  See include/fftenkf.h.
#include "fftenkf.h"

#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "kernels.hpp"

namespace fftenkf {

hipError_t launch_k2_f32_n4(const K2Args&, hipStream_t);
hipError_t launch_k2_f32_n8(const K2Args&, hipStream_t);
hipError_t launch_k2_f32_n12(const K2Args&, hipStream_t);
hipError_t launch_k2_f32_n16(const K2Args&, hipStream_t);
hipError_t launch_k2_f32_n20(const K2Args&, hipStream_t);
hipError_t launch_k2_f32_n24(const K2Args&, hipStream_t);
hipError_t launch_k2_f64_n4(const K2Args&, hipStream_t);
hipError_t launch_k2_f64_n8(const K2Args&, hipStream_t);

int k2_member_bucket(int dtype, int N) {
  static const int f32[] = {4, 8, 12, 16, 20, 24};
  static const int f64[] = {4, 8};
  const int* b = dtype == FFTENKF_F32 ? f32 : f64;
  const int nb = dtype == FFTENKF_F32 ? 6 : 2;
  for (int i = 0; i < nb; ++i)
    if (N <= b[i]) return b[i];
  return 0;
}

hipError_t launch_k2_f32(const K2Args& a, hipStream_t s) {
  switch (k2_member_bucket(FFTENKF_F32, a.N)) {
    case 4: return launch_k2_f32_n4(a, s);
    case 8: return launch_k2_f32_n8(a, s);
    case 12: return launch_k2_f32_n12(a, s);
    case 16: return launch_k2_f32_n16(a, s);
    case 20: return launch_k2_f32_n20(a, s);
    case 24: return launch_k2_f32_n24(a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_k1_batch_f32(const BatchArgs&, int, hipStream_t);
hipError_t launch_k1_batch_f64(const BatchArgs&, int, hipStream_t);
hipError_t launch_k3_batch_f32(const BatchArgs&, int, hipStream_t);
hipError_t launch_k3_batch_f64(const BatchArgs&, int, hipStream_t);
hipError_t launch_k2_batch_f32_n4(const BatchArgs&, hipStream_t);
hipError_t launch_k2_batch_f32_n8(const BatchArgs&, hipStream_t);
hipError_t launch_k2_batch_f32_n12(const BatchArgs&, hipStream_t);
hipError_t launch_k2_batch_f32_n16(const BatchArgs&, hipStream_t);
hipError_t launch_k2_batch_f32_n20(const BatchArgs&, hipStream_t);
hipError_t launch_k2_batch_f32_n24(const BatchArgs&, hipStream_t);
hipError_t launch_k2_batch_f64_n4(const BatchArgs&, hipStream_t);
hipError_t launch_k2_batch_f64_n8(const BatchArgs&, hipStream_t);

hipError_t launch_k10_f32_k1(const K10Args&, hipStream_t);
hipError_t launch_k10_f32_k3(const K10Args&, hipStream_t);
hipError_t launch_k10_f64(const K10Args&, hipStream_t);

hipError_t launch_k10(const K10Args& a, int dtype, hipStream_t s) {
  if (dtype == FFTENKF_F64) return launch_k10_f64(a, s);
  return a.K == 1 ? launch_k10_f32_k1(a, s) : launch_k10_f32_k3(a, s);
}

hipError_t launch_k2_f64(const K2Args& a, hipStream_t s) {
  switch (k2_member_bucket(FFTENKF_F64, a.N)) {
    case 4: return launch_k2_f64_n4(a, s);
    case 8: return launch_k2_f64_n8(a, s);
    default: return hipErrorInvalidValue;
  }
}

namespace {

thread_local std::string t_last_error;
thread_local int t_fail_next = 0;
thread_local hipEvent_t t_events[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
thread_local int t_nevents = 0;
thread_local bool t_events_on = false;

hipError_t mark(int i, hipStream_t s) {
  if (!t_events_on) return hipSuccess;
  return hipEventRecord(t_events[i], s);
}

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  t_last_error = buf;
  return code;
}

bool pow2_in_range(int v) { return v >= 8 && v <= 4096 && (v & (v - 1)) == 0; }

size_t dsize(int dtype) { return dtype == FFTENKF_F64 ? 8 : 4; }

// Grid factorisation ny = R * L and the unit shape of the spectral sweep.
struct Plan {
  int R, L, P, C, units, group_xcd;
  size_t main_elems;                   // complex elements of the spectral region
  size_t off_chat, off_lam, off_part;  // byte offsets in the workspace
  size_t ws_bytes;
};

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// Default rows per sweep-1/3 tile (the tile schedule ny = R * L).  Timed with
// the autotuner at N = 5 to 20: R = 8 is faster for every float32 grid up to
// 1024 wide, and R = 16 for 2048-wide grids from N = 16 up (at N = 5 there R = 8
// is faster; fftenkf_set_tile_rows overrides per grid, among the compiled
// choices of tile_rows_options).
int rows_per_tile(int dtype, int nx) {
  if (dtype == FFTENKF_F32) return nx == 2048 ? 16 : 8;
  return nx <= 2048 ? 8 : 4;
}

// Row counts R of the sweep-1/3 tiles compiled for a dtype and nx (each also
// needs R <= ny and ny / R <= 512, the longest transform of the spectral sweeps).
int tile_rows_options(int dtype, int nx, int* out) {
  if (dtype == FFTENKF_F32) {
    if (nx <= 2048) {
      out[0] = 4;
      out[1] = 8;
      out[2] = 16;
      return 3;
    }
    out[0] = 8;
    return 1;
  }
  out[0] = nx <= 2048 ? 8 : 4;
  return 1;
}

bool tile_rows_fit(int rows, int ny) { return rows <= ny && ny / rows <= 512; }

// Tile rows chosen by a tuner for a grid, process-wide; the default otherwise.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, int> g_tune;

int tile_rows(int ny, int nx, int dtype) {
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune.find(std::make_tuple(ny, nx, dtype));
    if (it != g_tune.end()) return it->second;
  }
  const int rmax = rows_per_tile(dtype, nx);
  return ny < rmax ? ny : rmax;
}

Plan make_plan(int N, int ny, int nx, int dtype) {
  Plan p{};
  p.R = tile_rows(ny, nx, dtype);
  p.L = ny / p.R;
  p.P = k2_points(p.L);
  const int tf2 = p.L / p.P;
  const int nxh = nx / 2;
  int c = k2_threads_target / tf2;
  if (c > nxh) c = nxh;
  if (c < 1) c = 1;
  p.C = c;
  p.units = p.R * (nxh / c);  // the Nyquist column is folded into kx = 0: no units of its own
  // group the units that share 128-byte lines on one XCD when segments are shorter
  const int seg = c * 2 * (int)dsize(dtype);
  const int g = seg < 128 ? 128 / seg : 1;
  p.group_xcd = (g > 1 && (nxh / c) % g == 0 && p.units % (8 * g) == 0) ? g : 1;
  const size_t nf = (size_t)N + 1;
  p.main_elems = nf * (size_t)ny * (size_t)nxh;
  const size_t cplx = 2 * dsize(dtype);
  const size_t plane = (size_t)ny * (size_t)(nxh + 1) * dsize(dtype);
  p.off_chat = round256(p.main_elems * cplx);
  p.off_lam = round256(p.off_chat + plane);
  p.off_part = round256(p.off_lam + plane);
  p.ws_bytes = round256(p.off_part + (size_t)p.units * sizeof(float));
  return p;
}

// The spectral sweep's share of K2Args: the plan's geometry and the byte size
// of the spectral region (addressed with 32-bit offsets).
void set_k2_geometry(K2Args& a, const Plan& p, int N, int ny, int nx, int dtype) {
  const size_t cplx = 2 * dsize(dtype);
  a.N = N;
  a.ny = ny;
  a.nx = nx;
  a.R = p.R;
  a.L = p.L;
  a.C = p.C;
  a.units = p.units;
  a.group_xcd = p.group_xcd;
  a.main_bytes = (uint32_t)(p.main_elems * cplx);
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + nb && y < x + na;
}

bool misaligned(const void* p, size_t a) { return ((uintptr_t)p % a) != 0; }

// R = r I when no R_spec array is given: r must be >= 0 and finite in the
// working precision (an infinite r would make the perturbation amplitude
// infinite where the gain is exactly 0, and 0 * inf is NaN).
int check_r_scalar(double r, int dtype, const char* prefix) {
  const double rmax = dtype == FFTENKF_F32 ? (double)3.4028234663852886e+38 : 1.7976931348623157e+308;
  if (!(r >= 0.0) || !(r <= rmax))
    return fail(FFTENKF_EINVAL, "%sr_scalar = %g: it must be >= 0 and finite in the working precision when R_spec is NULL",
                prefix, r);
  return FFTENKF_OK;
}

// Shape, dtype, N and workspace checks common to every entry point.
int validate_shape(const fftenkf_ens* e, Plan* plan) {
  if (e == nullptr) return fail(FFTENKF_EINVAL, "ens is NULL");
  if (e->dtype != FFTENKF_F32 && e->dtype != FFTENKF_F64) return fail(FFTENKF_EINVAL, "dtype %d is not 0 (f32) or 1 (f64)", e->dtype);
  if (e->n_members < 2) return fail(FFTENKF_EINVAL, "n_members = %d, eq. (2) needs N >= 2", e->n_members);
  if (!pow2_in_range(e->ny) || !pow2_in_range(e->nx))
    return fail(FFTENKF_EUNSUPPORTED, "grid %d x %d: each side must be a power of two in [8, 4096]", e->ny, e->nx);
  if (k2_member_bucket(e->dtype, e->n_members) == 0)
    return fail(FFTENKF_EUNSUPPORTED, "n_members = %d exceeds %d for this dtype", e->n_members, fftenkf_max_members(e->dtype));
  *plan = make_plan(e->n_members, e->ny, e->nx, e->dtype);
  if (plan->main_elems * 2 * dsize(e->dtype) >= ((size_t)1 << 31))
    return fail(FFTENKF_EUNSUPPORTED, "the spectra of %d fields on a %d x %d grid exceed 2 GiB", e->n_members + 1,
                e->ny, e->nx);
  if (e->members == nullptr) return fail(FFTENKF_EINVAL, "members is NULL");
  if (e->workspace == nullptr) return fail(FFTENKF_EINVAL, "workspace is NULL");
  if (e->workspace_bytes < plan->ws_bytes)
    return fail(FFTENKF_EINVAL, "workspace of %zu bytes, %zu needed", e->workspace_bytes, plan->ws_bytes);
  if (misaligned(e->members, 16)) return fail(FFTENKF_EINVAL, "members is not 16-byte aligned");
  if (misaligned(e->workspace, 256)) return fail(FFTENKF_EINVAL, "workspace is not 256-byte aligned");
  return FFTENKF_OK;
}

// Every pointer must be device memory of the current device.
int check_device_pointer(const void* p, const char* what, int dev) {
  hipPointerAttribute_t attr;
  memset(&attr, 0, sizeof(attr));
  const hipError_t err = hipPointerGetAttributes(&attr, p);
  if (err != hipSuccess) {
    (void)hipGetLastError();
    return fail(FFTENKF_EDEVICE, "%s: not a HIP allocation (%s)", what, hipGetErrorString(err));
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
    return fail(FFTENKF_EINVAL, "%s is not device memory", what);
  if (attr.device != dev) return fail(FFTENKF_EINVAL, "%s lives on device %d, current device is %d", what, attr.device, dev);
  return FFTENKF_OK;
}

struct Ptr {
  const void* p;
  size_t bytes;
  const char* name;
};

int check_pointers(const Ptr* ptrs, int n) {
  int dev = 0;
  hipError_t err = hipGetDevice(&dev);
  if (err != hipSuccess) return fail(FFTENKF_EDEVICE, "hipGetDevice: %s", hipGetErrorString(err));
  for (int i = 0; i < n; ++i)
    if (ptrs[i].p != nullptr) {
      const int st = check_device_pointer(ptrs[i].p, ptrs[i].name, dev);
      if (st != FFTENKF_OK) return st;
    }
  return FFTENKF_OK;
}

bool log_enabled() {
  static int on = -1;
  if (on < 0) {
    const char* v = getenv("FFTENKF_LOG");
    on = (v != nullptr && v[0] == '1') ? 1 : 0;
  }
  return on == 1;
}

// Enqueue sweeps 1 and 2 (mode) and, for an analysis, sweep 3.
// With mlp, sweep 2 runs twice around the perceptron: K2_CHAT (statistics
// only), then (for an analysis) K2_ANALYZE with the perceptron's spectrum in
// place of eq. (2); mlp_chat/mlp_lam/mlp_mu request the spectra only.
int run(const fftenkf_ens* e, const Plan& plan, const void* data, const void* R_spec, uint64_t seed, void* out,
        int mode, void* dbg_chat, void* dbg_gain, void* dbg_spec, void* dbg_e, const fftenkf_mlp* mlp = nullptr,
        void* mlp_chat = nullptr, void* mlp_lam = nullptr, void* mlp_mu = nullptr, const void* lam = nullptr) {
  if (t_fail_next != 0) {
    const int st = t_fail_next;
    t_fail_next = 0;
    return fail(st, "failure forced by fftenkf_debug_fail_next");
  }
  hipStream_t stream = static_cast<hipStream_t>(e->stream);
  const void* tab = nullptr;
  hipError_t err = twiddle_table(e->dtype, &tab);
  if (err != hipSuccess) return fail(FFTENKF_EDEVICE, "twiddle table: %s", hipGetErrorString(err));
  const size_t cplx = 2 * dsize(e->dtype);
  char* ws = static_cast<char*>(e->workspace);
  void* ws_main = ws;
  (void)cplx;
  if (log_enabled())
    fprintf(stderr, "fftenkf: N=%d grid %dx%d dtype=%d R=%d L=%d C=%d units=%d group_xcd=%d mode=%d\n", e->n_members,
            e->ny, e->nx, e->dtype, plan.R, plan.L, plan.C, plan.units, plan.group_xcd, mode);

  const bool profiled = t_events_on && mode == K2_ANALYZE && t_nevents == (mlp != nullptr ? 6 : 4);
  if (!profiled) t_events_on = false;
  err = mark(0, stream);
  if (err != hipSuccess) return fail(FFTENKF_EDEVICE, "profile event: %s", hipGetErrorString(err));
  K1Args a1{e->members, data, e->n_members, e->ny, e->nx, plan.R, plan.L, ws_main, tab};
  err = e->dtype == FFTENKF_F32 ? launch_k1_f32(a1, stream) : launch_k1_f64(a1, stream);
  if (err == hipSuccess) err = mark(1, stream);
  if (err != hipSuccess) return fail(FFTENKF_EDEVICE, "sweep 1 launch: %s", hipGetErrorString(err));

  K2Args a2{};
  a2.ws_main = ws_main;
  a2.R_spec = R_spec;
  a2.r_scalar = e->r_scalar;
  set_k2_geometry(a2, plan, e->n_members, e->ny, e->nx, e->dtype);
  a2.key0 = (uint32_t)(seed & 0xFFFFFFFFu);
  a2.key1 = (uint32_t)(seed >> 32);
  a2.mode = mode;
  a2.dbg_chat = dbg_chat;
  a2.dbg_gain = dbg_gain;
  a2.dbg_spec = dbg_spec;
  a2.dbg_e = dbg_e;
  a2.lam_map = lam;
  a2.tab = tab;
  if (mlp != nullptr) {
    // the perceptron needs c_hat of every bin, and their mean, before any update
    a2.mode = K2_CHAT;
    a2.chat_map = mlp_chat != nullptr ? mlp_chat : ws + plan.off_chat;
    a2.partials = ws + plan.off_part;
    err = launch_k2_f32(a2, stream);
    if (err == hipSuccess) err = mark(2, stream);
    if (err != hipSuccess) return fail(FFTENKF_EDEVICE, "sweep 2 (statistics) launch: %s", hipGetErrorString(err));
    K7Args a7{};
    a7.chat = static_cast<const float*>(a2.chat_map);
    a7.partials = static_cast<const float*>(a2.partials);
    a7.n_partials = plan.units;
    a7.ny = e->ny;
    a7.nx = e->nx;
    a7.W1 = mlp->W1;
    a7.b1 = mlp->b1;
    a7.W2 = mlp->W2;
    a7.b2 = mlp->b2;
    a7.W3 = mlp->W3;
    a7.b3 = mlp->b3;
    a7.w4 = mlp->w4;
    a7.b4 = mlp->b4;
    a7.lam = static_cast<float*>(mlp_lam != nullptr ? mlp_lam : ws + plan.off_lam);
    a7.mu_out = static_cast<float*>(mlp_mu);
    err = launch_k7(a7, stream);
    if (err == hipSuccess) err = mark(3, stream);
    if (err != hipSuccess) return fail(FFTENKF_EDEVICE, "perceptron launch: %s", hipGetErrorString(err));
    if (mode != K2_ANALYZE) return FFTENKF_OK;
    a2.mode = K2_ANALYZE;
    a2.lam_map = a7.lam;
    err = launch_k2_f32(a2, stream);
    if (err == hipSuccess) err = mark(4, stream);
  } else {
    err = e->dtype == FFTENKF_F32 ? launch_k2_f32(a2, stream) : launch_k2_f64(a2, stream);
  }
  if (err == hipSuccess && mlp == nullptr) err = mark(2, stream);
  if (err != hipSuccess) return fail(FFTENKF_EDEVICE, "sweep 2 launch: %s", hipGetErrorString(err));
  if (mode != K2_ANALYZE) return FFTENKF_OK;

  K3Args a3{ws_main, e->n_members, e->ny, e->nx, plan.R, plan.L, out, tab};
  err = e->dtype == FFTENKF_F32 ? launch_k3_f32(a3, stream) : launch_k3_f64(a3, stream);
  if (err == hipSuccess) err = mark(mlp != nullptr ? 5 : 3, stream);
  t_events_on = false;
  if (err != hipSuccess) return fail(FFTENKF_EDEVICE, "sweep 3 launch: %s", hipGetErrorString(err));
  return FFTENKF_OK;
}

// Read on every call, so the switch can be flipped while the process runs.
bool check_enabled() {
  const char* v = getenv("FFTENKF_CHECK");
  return v != nullptr && v[0] == '1' && v[1] == '\0';
}

// With FFTENKF_CHECK=1: every entry of a device array of n reals is finite and >= 0.
int check_spectrum_values(const void* p, size_t n, int dtype, hipStream_t stream, const char* what) {
  if (p == nullptr || !check_enabled()) return FFTENKF_OK;
  hipError_t err = hipStreamSynchronize(stream);
  std::vector<double> host(n);
  if (err == hipSuccess) {
    if (dtype == FFTENKF_F64) {
      err = hipMemcpy(host.data(), p, n * sizeof(double), hipMemcpyDeviceToHost);
    } else {
      std::vector<float> f(n);
      err = hipMemcpy(f.data(), p, n * sizeof(float), hipMemcpyDeviceToHost);
      for (size_t i = 0; i < n; ++i) host[i] = f[i];
    }
  }
  if (err != hipSuccess) return fail(FFTENKF_EDEVICE, "%s check: %s", what, hipGetErrorString(err));
  for (size_t i = 0; i < n; ++i)
    if (!(host[i] >= 0.0) || !std::isfinite(host[i]))
      return fail(FFTENKF_EINVAL, "%s[%zu] = %g: entries must be finite and >= 0", what, i, host[i]);
  return FFTENKF_OK;
}

// The 2D transform alone: forward (sweep 1, the statistics mode of sweep 2,
// gather) or inverse (scatter, the inverse-only mode of sweep 2, sweep 3).
int run_fft2(const fftenkf_ens* e, const Plan& plan, int inverse, const void* spectra, void* out) {
  if (t_fail_next != 0) {
    const int st = t_fail_next;
    t_fail_next = 0;
    return fail(st, "failure forced by fftenkf_debug_fail_next");
  }
  hipStream_t stream = static_cast<hipStream_t>(e->stream);
  const void* tab = nullptr;
  hipError_t err = twiddle_table(e->dtype, &tab);
  if (err != hipSuccess) return fail(FFTENKF_EDEVICE, "twiddle table: %s", hipGetErrorString(err));
  char* ws = static_cast<char*>(e->workspace);
  void* ws_main = ws;
  const double n = (double)e->ny * (double)e->nx;
  K2Args a2{};
  a2.ws_main = ws_main;
  a2.r_scalar = 1.0;
  set_k2_geometry(a2, plan, e->n_members, e->ny, e->nx, e->dtype);
  a2.chat_map = ws + plan.off_chat;
  a2.partials = ws + plan.off_part;
  a2.tab = tab;
  K8Args a8{ws_main, e->n_members, e->ny, e->nx, plan.R, plan.L, 0.0, nullptr};
  auto k2 = [&]() { return e->dtype == FFTENKF_F32 ? launch_k2_f32(a2, stream) : launch_k2_f64(a2, stream); };
  if (!inverse) {
    // the members double as d: sweep 2 needs a data field, which is not used here
    K1Args a1{e->members, e->members, e->n_members, e->ny, e->nx, plan.R, plan.L, ws_main, tab};
    err = e->dtype == FFTENKF_F32 ? launch_k1_f32(a1, stream) : launch_k1_f64(a1, stream);
    a2.mode = K2_STATS;
    if (err == hipSuccess) err = k2();
    a8.scale = 1.0 / std::sqrt(n);
    a8.spectra = out;
    if (err == hipSuccess) err = launch_k8_gather(a8, e->dtype, stream);
  } else {
    a8.scale = std::sqrt(n);
    a8.spectra = const_cast<void*>(spectra);
    err = launch_k8_scatter(a8, e->dtype, stream);
    a2.mode = K2_INVERSE;
    if (err == hipSuccess) err = k2();
    K3Args a3{ws_main, e->n_members, e->ny, e->nx, plan.R, plan.L, out, tab};
    if (err == hipSuccess) err = e->dtype == FFTENKF_F32 ? launch_k3_f32(a3, stream) : launch_k3_f64(a3, stream);
  }
  if (err != hipSuccess) return fail(FFTENKF_EDEVICE, "transform launch: %s", hipGetErrorString(err));
  return FFTENKF_OK;
}

// Largest N of the sweep with K observed blocks.
int max_members_observed(int dtype, int K) {
  if (dtype == FFTENKF_F32) return K == 1 ? kMaxMembersMultiF32 : kMaxMembersObsF32;
  if (dtype == FFTENKF_F64) return K == 1 ? kMaxMembersMultiF64 : kMaxMembersObsF64;
  return 0;
}

// Shape and workspace checks of an M-block state with K observed blocks; the
// plan covers the N * M member fields and the K data fields.
int validate_observed(const fftenkf_ens* e, int M, int K, Plan* plan) {
  if (e == nullptr) return fail(FFTENKF_EINVAL, "ens is NULL");
  if (e->dtype != FFTENKF_F32 && e->dtype != FFTENKF_F64) return fail(FFTENKF_EINVAL, "dtype %d is not 0 (f32) or 1 (f64)", e->dtype);
  if (e->n_members < 2) return fail(FFTENKF_EINVAL, "n_members = %d, eq. (2) needs N >= 2", e->n_members);
  if (M < 1 || M > kMaxStateBlocks) return fail(FFTENKF_EINVAL, "n_blocks = %d outside [1, %d]", M, kMaxStateBlocks);
  if (K < 1 || K > kMaxObserved || K > M)
    return fail(FFTENKF_EINVAL, "n_obs = %d outside [1, min(%d, n_blocks = %d)]", K, kMaxObserved, M);
  if (!pow2_in_range(e->ny) || !pow2_in_range(e->nx))
    return fail(FFTENKF_EUNSUPPORTED, "grid %d x %d: each side must be a power of two in [8, 4096]", e->ny, e->nx);
  if (e->n_members > max_members_observed(e->dtype, K))
    return fail(FFTENKF_EUNSUPPORTED, "n_members = %d exceeds %d for %d observed block(s)", e->n_members,
                max_members_observed(e->dtype, K), K);
  *plan = make_plan(e->n_members * M + K - 1, e->ny, e->nx, e->dtype);
  if (e->members == nullptr) return fail(FFTENKF_EINVAL, "members is NULL");
  if (e->workspace == nullptr) return fail(FFTENKF_EINVAL, "workspace is NULL");
  if (e->workspace_bytes < plan->ws_bytes)
    return fail(FFTENKF_EINVAL, "workspace of %zu bytes, %zu needed", e->workspace_bytes, plan->ws_bytes);
  if (misaligned(e->members, 16)) return fail(FFTENKF_EINVAL, "members is not 16-byte aligned");
  if (misaligned(e->workspace, 256)) return fail(FFTENKF_EINVAL, "workspace is not 256-byte aligned");
  return FFTENKF_OK;
}

// Sweep 1 over the N * M member fields and the K data fields, the sweep of
// the observed-block state, sweep 3 over the member fields.
int run_observed(const fftenkf_ens* e, int M, int K, const Plan& plan, const void* data, const void* R_spec,
                 const double* r_obs, uint64_t seed, void* out) {
  if (t_fail_next != 0) {
    const int st = t_fail_next;
    t_fail_next = 0;
    return fail(st, "failure forced by fftenkf_debug_fail_next");
  }
  hipStream_t stream = static_cast<hipStream_t>(e->stream);
  const void* tab = nullptr;
  hipError_t err = twiddle_table(e->dtype, &tab);
  if (err != hipSuccess) return fail(FFTENKF_EDEVICE, "twiddle table: %s", hipGetErrorString(err));
  char* ws = static_cast<char*>(e->workspace);
  void* ws_main = ws;
  const int fields = e->n_members * M;
  if (!(t_events_on && t_nevents == 4)) t_events_on = false;
  err = mark(0, stream);
  K1Args a1{e->members, data, fields, e->ny, e->nx, plan.R, plan.L, ws_main, tab};
  a1.n_data = K;
  if (err == hipSuccess) err = e->dtype == FFTENKF_F32 ? launch_k1_f32(a1, stream) : launch_k1_f64(a1, stream);
  if (err == hipSuccess) err = mark(1, stream);
  if (err != hipSuccess) return fail(FFTENKF_EDEVICE, "sweep 1 launch: %s", hipGetErrorString(err));
  K10Args a10{};
  a10.ws_main = ws_main;
  a10.R_spec = R_spec;
  for (int o = 0; o < K; ++o) a10.r_obs[o] = r_obs != nullptr ? r_obs[o] : 0.0;
  a10.N = e->n_members;
  a10.M = M;
  a10.K = K;
  a10.ny = e->ny;
  a10.nx = e->nx;
  a10.R = plan.R;
  a10.L = plan.L;
  a10.C = plan.C;
  a10.units = plan.units;
  a10.group_xcd = plan.group_xcd;
  a10.key0 = (uint32_t)(seed & 0xFFFFFFFFu);
  a10.key1 = (uint32_t)(seed >> 32);
  a10.tab = tab;
  err = launch_k10(a10, e->dtype, stream);
  if (err == hipSuccess) err = mark(2, stream);
  if (err != hipSuccess) return fail(FFTENKF_EDEVICE, "observed-block sweep launch: %s", hipGetErrorString(err));
  K3Args a3{ws_main, fields, e->ny, e->nx, plan.R, plan.L, out, tab};
  err = e->dtype == FFTENKF_F32 ? launch_k3_f32(a3, stream) : launch_k3_f64(a3, stream);
  if (err == hipSuccess) err = mark(3, stream);
  t_events_on = false;
  if (err != hipSuccess) return fail(FFTENKF_EDEVICE, "sweep 3 launch: %s", hipGetErrorString(err));
  return FFTENKF_OK;
}

// Argument checks and dispatch of the state with K observed blocks.  R per
// observed block: R_spec ([K][ny][nx/2+1]) or, when it is NULL, r_obs[o].
int analyze_observed(const fftenkf_ens* e, int M, int K, const void* data, const void* R_spec, const double* r_obs,
                     uint64_t seed, void* out) {
  Plan plan;
  int st = validate_observed(e, M, K, &plan);
  if (st != FFTENKF_OK) return st;
  if (data == nullptr) return fail(FFTENKF_EINVAL, "data is NULL");
  if (out == nullptr) return fail(FFTENKF_EINVAL, "out is NULL");
  if (misaligned(data, 16) || misaligned(out, 16) || (R_spec != nullptr && misaligned(R_spec, 16)))
    return fail(FFTENKF_EINVAL, "data, R_spec and out must be 16-byte aligned");
  if (R_spec == nullptr) {
    if (r_obs == nullptr) return fail(FFTENKF_EINVAL, "R_spec and r_obs are both NULL");
    for (int o = 0; o < K; ++o) {
      char prefix[48];
      snprintf(prefix, sizeof(prefix), "observed block %d: ", o);
      if ((st = check_r_scalar(r_obs[o], e->dtype, prefix)) != FFTENKF_OK) return st;
    }
  }
  const size_t s = dsize(e->dtype);
  const size_t field = (size_t)e->ny * e->nx * s;
  const size_t ens_b = field * e->n_members * M;
  const size_t rs_b = (size_t)e->ny * (e->nx / 2 + 1) * s * K;
  const Ptr ptrs[] = {{e->members, ens_b, "members"},
                      {data, field * K, "data"},
                      {R_spec, rs_b, "R_spec"},
                      {out, ens_b, "out"},
                      {e->workspace, plan.ws_bytes, "workspace"}};
  for (int i = 0; i < 5; ++i)
    for (int j = i + 1; j < 5; ++j) {
      if (ptrs[i].p == nullptr || ptrs[j].p == nullptr) continue;
      const bool in_place = (i == 0 && j == 3 && ptrs[i].p == ptrs[j].p);
      if (!in_place && overlaps(ptrs[i].p, ptrs[i].bytes, ptrs[j].p, ptrs[j].bytes))
        return fail(FFTENKF_EINVAL, "%s overlaps %s", ptrs[i].name, ptrs[j].name);
    }
  st = check_pointers(ptrs, 5);
  if (st == FFTENKF_OK)
    st = check_spectrum_values(R_spec, (size_t)e->ny * (e->nx / 2 + 1) * K, e->dtype,
                               static_cast<hipStream_t>(e->stream), "R_spec");
  if (st != FFTENKF_OK) return st;
  return run_observed(e, M, K, plan, data, R_spec, r_obs, seed, out);
}

hipError_t launch_k2_batch(const BatchArgs& b, int dtype, hipStream_t s) {
  switch (k2_member_bucket(dtype, b.N) * (dtype == FFTENKF_F32 ? 1 : -1)) {
    case 4: return launch_k2_batch_f32_n4(b, s);
    case 8: return launch_k2_batch_f32_n8(b, s);
    case 12: return launch_k2_batch_f32_n12(b, s);
    case 16: return launch_k2_batch_f32_n16(b, s);
    case 20: return launch_k2_batch_f32_n20(b, s);
    case 24: return launch_k2_batch_f32_n24(b, s);
    case -4: return launch_k2_batch_f64_n4(b, s);
    case -8: return launch_k2_batch_f64_n8(b, s);
    default: return hipErrorInvalidValue;
  }
}

// One filter of a batch: the checks of fftenkf_analyze, host-side ones only.
int validate_filter(const fftenkf_filter& f, int N, int dtype, int i, Plan* plan) {
  if (!pow2_in_range(f.ny) || !pow2_in_range(f.nx))
    return fail(FFTENKF_EUNSUPPORTED, "filter %d: grid %d x %d: each side must be a power of two in [8, 4096]", i,
                f.ny, f.nx);
  *plan = make_plan(N, f.ny, f.nx, dtype);
  if (f.members == nullptr || f.data == nullptr || f.out == nullptr || f.workspace == nullptr)
    return fail(FFTENKF_EINVAL, "filter %d: members, data, out and workspace are required", i);
  if (f.workspace_bytes < plan->ws_bytes)
    return fail(FFTENKF_EINVAL, "filter %d: workspace of %zu bytes, %zu needed", i, f.workspace_bytes, plan->ws_bytes);
  if (misaligned(f.members, 16) || misaligned(f.data, 16) || misaligned(f.out, 16) ||
      (f.R_spec != nullptr && misaligned(f.R_spec, 16)) || misaligned(f.workspace, 256))
    return fail(FFTENKF_EINVAL, "filter %d: pointers must be 16-byte (workspace 256-byte) aligned", i);
  if (f.R_spec == nullptr) {
    char prefix[32];
    snprintf(prefix, sizeof(prefix), "filter %d: ", i);
    const int st = check_r_scalar(f.r_scalar, dtype, prefix);
    if (st != FFTENKF_OK) return st;
  }
  return FFTENKF_OK;
}

// The regions a filter reads (members, data, R_spec) and writes (out, workspace).
void filter_regions(const fftenkf_filter& f, int N, int dtype, const Plan& plan, Ptr* r) {
  const size_t s = dsize(dtype);
  const size_t field = (size_t)f.ny * f.nx * s;
  r[0] = {f.members, field * N, "members"};
  r[1] = {f.data, field, "data"};
  r[2] = {f.R_spec, (size_t)f.ny * (f.nx / 2 + 1) * s, "R_spec"};
  r[3] = {f.out, field * N, "out"};
  r[4] = {f.workspace, plan.ws_bytes, "workspace"};
}

// Streams beside the caller's for the launch chains of a batch, per device,
// made on the first batch that is not being captured (stream and event
// creation stay out of a capture).  Default priority, non-blocking.
constexpr int kSideStreams = 3;
struct SidePool {
  hipStream_t s[kSideStreams];
  hipEvent_t fork, join[kSideStreams];
};
std::mutex g_side_mu;
std::map<int, SidePool> g_side;

// The pool of the current device, or nullptr if there is none and one cannot
// be made now (under capture, or on a creation failure), or if `stream`
// belongs to another device than the current one (the chains then stay on
// `stream`).  g_side_mu held.
const SidePool* side_pool(hipStream_t stream) {
  int dev = 0, sdev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  if (stream != nullptr && hipStreamGetDevice(stream, &sdev) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  if (stream != nullptr && sdev != dev) return nullptr;
  auto it = g_side.find(dev);
  if (it != g_side.end()) return &it->second;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return nullptr;
  SidePool p{};
  bool ok = hipEventCreateWithFlags(&p.fork, hipEventDisableTiming) == hipSuccess;
  for (int k = 0; k < kSideStreams && ok; ++k)
    ok = hipStreamCreateWithFlags(&p.s[k], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&p.join[k], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    return nullptr;  // what was made is kept until the process ends
  }
  return &g_side.emplace(dev, p).first->second;
}

// The three sweeps of every filter: filters on the same grid share launches,
// kMaxBatch at a time, blockIdx.y selecting the filter.  Each such chain of
// three launches is independent of the others; with more than one chain they
// run on side streams forked from `stream` and joined back into it (largest
// chains first, each to the least loaded side stream), so a small grid's
// launches run beside a large grid's rather than after them and the end of one
// launch overlaps the others.  Under stream capture this records the same fork
// and join as graph dependencies.
int run_batch(int N, int dtype, const fftenkf_filter* fs, int n, const std::vector<Plan>& plans, hipStream_t stream) {
  if (t_fail_next != 0) {
    const int st = t_fail_next;
    t_fail_next = 0;
    return fail(st, "failure forced by fftenkf_debug_fail_next");
  }
  const void* tab = nullptr;
  hipError_t err = twiddle_table(dtype, &tab);
  if (err != hipSuccess) return fail(FFTENKF_EDEVICE, "twiddle table: %s", hipGetErrorString(err));
  std::map<std::pair<int, int>, std::vector<int>> groups;
  for (int i = 0; i < n; ++i) groups[std::make_pair(fs[i].ny, fs[i].nx)].push_back(i);
  struct Chain {
    int plan;
    std::vector<int> idx;
    double cost;
  };
  std::vector<Chain> chains;
  for (const auto& g : groups)
    for (size_t c0 = 0; c0 < g.second.size(); c0 += kMaxBatch) {
      Chain c;
      c.plan = g.second[0];
      c.idx.assign(g.second.begin() + c0, g.second.begin() + std::min(g.second.size(), c0 + kMaxBatch));
      c.cost = (double)c.idx.size() * g.first.first * g.first.second;
      chains.push_back(std::move(c));
    }
  std::stable_sort(chains.begin(), chains.end(), [](const Chain& a, const Chain& b) { return a.cost > b.cost; });

  auto launch_chain = [&](const Chain& c, hipStream_t st) -> hipError_t {
    const Plan& plan = plans[c.plan];
    BatchArgs b{};
    b.count = (int)c.idx.size();
    b.N = N;
    b.ny = fs[c.idx[0]].ny;
    b.nx = fs[c.idx[0]].nx;
    b.L = plan.L;
    b.tab = tab;
    K2Args& a2 = b.k2;
    set_k2_geometry(a2, plan, N, b.ny, b.nx, dtype);
    a2.mode = K2_ANALYZE;
    a2.tab = tab;
    for (int k = 0; k < b.count; ++k) {
      const fftenkf_filter& f = fs[c.idx[k]];
      BatchFilter& bf = b.f[k];
      bf.members = f.members;
      bf.data = f.data;
      bf.R_spec = f.R_spec;
      bf.out = f.out;
      bf.ws_main = f.workspace;
      bf.r_scalar = f.r_scalar;
      bf.key0 = (uint32_t)(f.seed & 0xFFFFFFFFu);
      bf.key1 = (uint32_t)(f.seed >> 32);
    }
    hipError_t e = dtype == FFTENKF_F32 ? launch_k1_batch_f32(b, plan.R, st) : launch_k1_batch_f64(b, plan.R, st);
    if (e == hipSuccess) e = launch_k2_batch(b, dtype, st);
    if (e == hipSuccess)
      e = dtype == FFTENKF_F32 ? launch_k3_batch_f32(b, plan.R, st) : launch_k3_batch_f64(b, plan.R, st);
    if (e != hipSuccess) fail(FFTENKF_EDEVICE, "batch launch (%d x %d): %s", b.ny, b.nx, hipGetErrorString(e));
    return e;
  };

  std::lock_guard<std::mutex> lock(g_side_mu);
  const SidePool* pool = chains.size() > 1 ? side_pool(stream) : nullptr;
  if (pool == nullptr) {
    for (const Chain& c : chains)
      if (launch_chain(c, stream) != hipSuccess) return FFTENKF_EDEVICE;
    return FFTENKF_OK;
  }
  const int K = (int)std::min<size_t>(kSideStreams, chains.size());
  err = hipEventRecord(pool->fork, stream);
  for (int k = 0; k < K && err == hipSuccess; ++k) err = hipStreamWaitEvent(pool->s[k], pool->fork, 0);
  if (err != hipSuccess) return fail(FFTENKF_EDEVICE, "batch fork: %s", hipGetErrorString(err));
  double load[kSideStreams] = {};
  int st = FFTENKF_OK;
  for (const Chain& c : chains) {
    int k = 0;
    for (int j = 1; j < K; ++j)
      if (load[j] < load[k]) k = j;
    load[k] += c.cost;
    if (launch_chain(c, pool->s[k]) != hipSuccess) {
      st = FFTENKF_EDEVICE;
      break;
    }
  }
  // always join every side stream that was forked, so a capture can end
  for (int k = 0; k < K; ++k) {
    hipError_t e = hipEventRecord(pool->join[k], pool->s[k]);
    if (e == hipSuccess) e = hipStreamWaitEvent(stream, pool->join[k], 0);
    if (e != hipSuccess && st == FFTENKF_OK) st = fail(FFTENKF_EDEVICE, "batch join: %s", hipGetErrorString(e));
  }
  return st;
}

// The sine-basis analysis uses the periodic analysis' workspace.
size_t dst_ws_bytes(const Plan& plan, int, int, int, int) { return plan.ws_bytes; }

// Sweep 1 through the sine reordering; then, on the shapes it takes, the fused
// sine-basis sweep (k11_dst_fused.hpp) and sweep 3 back through the
// reordering.  Otherwise (and for the coefficient export) the statistics mode of
// sweep 2, the per-bin sine-basis kernel, then (for an analysis) the
// inverse-only mode of sweep 2 and sweep 3.
int run_dst(const fftenkf_ens* e, const Plan& plan, const void* data, const void* R_dst, uint64_t seed, void* out,
            void* dbg_coeffs) {
  if (t_fail_next != 0) {
    const int st = t_fail_next;
    t_fail_next = 0;
    return fail(st, "failure forced by fftenkf_debug_fail_next");
  }
  hipStream_t stream = static_cast<hipStream_t>(e->stream);
  const void* tab = nullptr;
  hipError_t err = twiddle_table(e->dtype, &tab);
  if (err != hipSuccess) return fail(FFTENKF_EDEVICE, "twiddle table: %s", hipGetErrorString(err));
  char* ws = static_cast<char*>(e->workspace);
  void* ws_main = ws;
  const int N = e->n_members, ny = e->ny, nx = e->nx;
  K1Args a1{e->members, data, N, ny, nx, plan.R, plan.L, ws_main, tab, 1};
  err = e->dtype == FFTENKF_F32 ? launch_k1_f32(a1, stream) : launch_k1_f64(a1, stream);
  K9Args a9{ws_main, R_dst, e->r_scalar, N, ny, nx, plan.R, plan.L,
            (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32), dbg_coeffs};
  a9.tab = tab;
  a9.main_bytes = (uint32_t)(plan.main_elems * 2 * dsize(e->dtype));
  if (dbg_coeffs == nullptr && k11_supports(plan.L, nx)) {
    // the spectral part as one sweep: transforms, eq. (2)-(3) on the sine
    // coefficients, inverse transforms
    if (err == hipSuccess) err = launch_k11(a9, e->dtype, stream);
    K3Args a3{ws_main, N, ny, nx, plan.R, plan.L, out, tab, 1};
    if (err == hipSuccess) err = e->dtype == FFTENKF_F32 ? launch_k3_f32(a3, stream) : launch_k3_f64(a3, stream);
    if (err != hipSuccess) return fail(FFTENKF_EDEVICE, "sine-basis analysis launch: %s", hipGetErrorString(err));
    return FFTENKF_OK;
  }
  K2Args a2{};
  a2.ws_main = ws_main;
  a2.r_scalar = 1.0;
  set_k2_geometry(a2, plan, N, ny, nx, e->dtype);
  a2.chat_map = ws + plan.off_chat;
  a2.partials = ws + plan.off_part;
  a2.tab = tab;
  a2.mode = K2_STATS;
  auto k2 = [&]() { return e->dtype == FFTENKF_F32 ? launch_k2_f32(a2, stream) : launch_k2_f64(a2, stream); };
  if (err == hipSuccess) err = k2();
  if (err == hipSuccess) err = launch_dst_quad(a9, e->dtype, stream);
  if (err == hipSuccess && dbg_coeffs == nullptr) {
    a2.mode = K2_INVERSE;
    err = k2();
    K3Args a3{ws_main, N, ny, nx, plan.R, plan.L, out, tab, 1};
    if (err == hipSuccess) err = e->dtype == FFTENKF_F32 ? launch_k3_f32(a3, stream) : launch_k3_f64(a3, stream);
  }
  if (err != hipSuccess) return fail(FFTENKF_EDEVICE, "sine-basis analysis launch: %s", hipGetErrorString(err));
  return FFTENKF_OK;
}

// The eight weight arrays of the perceptron: present and aligned (host-side
// checks), then device memory of the current device.
int check_mlp(const fftenkf_mlp* m, bool device) {
  const Ptr w[] = {{m->W1, 26 * 64 * 4, "mlp.W1"}, {m->b1, 64 * 4, "mlp.b1"}, {m->W2, 64 * 64 * 4, "mlp.W2"},
                   {m->b2, 64 * 4, "mlp.b2"},      {m->W3, 64 * 64 * 4, "mlp.W3"}, {m->b3, 64 * 4, "mlp.b3"},
                   {m->w4, 64 * 4, "mlp.w4"},      {m->b4, 4, "mlp.b4"}};
  for (const Ptr& p : w) {
    if (p.p == nullptr) return fail(FFTENKF_EINVAL, "%s is NULL", p.name);
    if (misaligned(p.p, 4)) return fail(FFTENKF_EINVAL, "%s is not 4-byte aligned", p.name);
  }
  return device ? check_pointers(w, 8) : FFTENKF_OK;
}

// ws_static: the workspace is the library's static scratch array (not a HIP
// allocation, so it is left out of the device-pointer check).
int analyze_impl(const fftenkf_ens* e, const void* data, const void* R_spec, uint64_t seed, const fftenkf_mlp* mlp,
                 const void* lam, void* out, bool ws_static = false) {
  try {
    Plan plan;
    int st = validate_shape(e, &plan);
    if (st != FFTENKF_OK) return st;
    if (data == nullptr) return fail(FFTENKF_EINVAL, "data is NULL");
    if (out == nullptr) return fail(FFTENKF_EINVAL, "out is NULL");
    if (misaligned(data, 16) || misaligned(out, 16) || (R_spec != nullptr && misaligned(R_spec, 16)))
      return fail(FFTENKF_EINVAL, "data, R_spec and out must be 16-byte aligned");
    if (R_spec == nullptr && (st = check_r_scalar(e->r_scalar, e->dtype, "")) != FFTENKF_OK) return st;
    const size_t s = dsize(e->dtype);
    const size_t field = (size_t)e->ny * e->nx * s;
    const size_t ens_b = field * e->n_members;
    const size_t rs_b = (size_t)e->ny * (e->nx / 2 + 1) * s;
    if (lam != nullptr && misaligned(lam, 16)) return fail(FFTENKF_EINVAL, "lam must be 16-byte aligned");
    const Ptr ptrs[] = {{e->members, ens_b, "members"},
                        {data, field, "data"},
                        {R_spec, rs_b, "R_spec"},
                        {out, ens_b, "out"},
                        {e->workspace, plan.ws_bytes, "workspace"},
                        {lam, rs_b, "lam"}};
    const int np = 6;
    for (int i = 0; i < np; ++i)
      for (int j = i + 1; j < np; ++j) {
        if (ptrs[i].p == nullptr || ptrs[j].p == nullptr) continue;
        const bool in_place = (i == 0 && j == 3 && ptrs[i].p == ptrs[j].p);
        if (!in_place && overlaps(ptrs[i].p, ptrs[i].bytes, ptrs[j].p, ptrs[j].bytes))
          return fail(FFTENKF_EINVAL, "%s overlaps %s", ptrs[i].name, ptrs[j].name);
      }
    if (mlp != nullptr) {
      st = check_mlp(mlp, false);
      if (st != FFTENKF_OK) return st;
    }
    Ptr dev_ptrs[np];
    for (int i = 0; i < np; ++i) dev_ptrs[i] = ptrs[i];
    if (ws_static) dev_ptrs[4].p = nullptr;
    st = check_pointers(dev_ptrs, np);
    if (st == FFTENKF_OK && mlp != nullptr) st = check_mlp(mlp, true);
    const size_t plane = (size_t)e->ny * (e->nx / 2 + 1);
    hipStream_t stream = static_cast<hipStream_t>(e->stream);
    if (st == FFTENKF_OK) st = check_spectrum_values(R_spec, plane, e->dtype, stream, "R_spec");
    if (st == FFTENKF_OK) st = check_spectrum_values(lam, plane, e->dtype, stream, "lam");
    if (st != FFTENKF_OK) return st;
    return run(e, plan, data, R_spec, seed, out, K2_ANALYZE, nullptr, nullptr, nullptr, nullptr, mlp, nullptr, nullptr,
               nullptr, lam);
  } catch (...) {
    return fail(FFTENKF_EDEVICE, "internal error");
  }
}

// ---- static scratch of the entry point that allocates nothing
//
// One array of kScratchBytes in static device memory per device, used as the
// workspace of fftenkf_analyze_noalloc.  The array's name is a host-side
// stand-in: its address on a device comes from hipGetSymbolAddress with that
// device current, once per device, and only that address is ever passed on.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kScratchDevices];

}  // namespace
}  // namespace fftenkf

static __device__ __align__(256) unsigned char scratch[fftenkf::kScratchBytes];

namespace fftenkf {
namespace {

// The scratch array's address on the current device (set up on the first call
// on each device, together with that device's twiddle tables).
int scratch_address(void** out) {
  int dev = 0;
  hipError_t err = hipGetDevice(&dev);
  if (err != hipSuccess) return fail(FFTENKF_EDEVICE, "hipGetDevice: %s", hipGetErrorString(err));
  if (dev < 0 || dev >= kScratchDevices) return fail(FFTENKF_EDEVICE, "device %d beyond the scratch table", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_addr[dev] == nullptr) {
    void* p = nullptr;
    err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (err != hipSuccess || p == nullptr)
      return fail(FFTENKF_EDEVICE, "scratch address: %s", hipGetErrorString(err));
    const void* tab = nullptr;
    err = twiddle_table(FFTENKF_F32, &tab);
    if (err == hipSuccess) err = twiddle_table(FFTENKF_F64, &tab);
    if (err != hipSuccess) return fail(FFTENKF_EDEVICE, "twiddle table: %s", hipGetErrorString(err));
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return FFTENKF_OK;
}

}  // namespace
}  // namespace fftenkf

using namespace fftenkf;

extern "C" {

size_t fftenkf_noalloc_max_bytes(void) { return kScratchBytes; }

int fftenkf_analyze_noalloc(const fftenkf_ens* e, const void* data, const void* R_spec, uint64_t seed, void* out) {
  try {
    if (e == nullptr) return fail(FFTENKF_EINVAL, "ens is NULL");
    // shape checks first (host only), with a stand-in workspace of any size
    fftenkf_ens copy = *e;
    copy.workspace = reinterpret_cast<void*>((uintptr_t)256);
    copy.workspace_bytes = (size_t)-1;
    Plan plan;
    int st = validate_shape(&copy, &plan);
    if (st != FFTENKF_OK) return st;
    if (plan.ws_bytes > kScratchBytes)
      return fail(FFTENKF_EINVAL,
                  "%d members on a %d x %d grid need %zu bytes of workspace; the static scratch holds %zu "
                  "(call fftenkf_analyze with a workspace instead)",
                  e->n_members, e->ny, e->nx, plan.ws_bytes, kScratchBytes);
    void* ws = nullptr;
    st = scratch_address(&ws);
    if (st != FFTENKF_OK) return st;
    copy.workspace = ws;
    copy.workspace_bytes = kScratchBytes;
    return analyze_impl(&copy, data, R_spec, seed, nullptr, nullptr, out, true);
  } catch (...) {
    return fail(FFTENKF_EDEVICE, "internal error");
  }
}

int fftenkf_max_members(int dtype) {
  if (dtype == FFTENKF_F32) return kMaxMembersF32;
  if (dtype == FFTENKF_F64) return kMaxMembersF64;
  return 0;
}

size_t fftenkf_workspace_bytes(int n_members, int ny, int nx, int dtype) {
  if ((dtype != FFTENKF_F32 && dtype != FFTENKF_F64) || n_members < 2 || !pow2_in_range(ny) || !pow2_in_range(nx))
    return 0;
  return make_plan(n_members, ny, nx, dtype).ws_bytes;
}

const char* fftenkf_strerror(int status) {
  switch (status) {
    case FFTENKF_OK: return "success";
    case FFTENKF_EINVAL: return "invalid argument";
    case FFTENKF_EUNSUPPORTED: return "unsupported shape";
    case FFTENKF_EDEVICE: return "HIP device error";
    case FFTENKF_ENOMEM: return "out of memory";
    default: return "unknown status";
  }
}

const char* fftenkf_last_error(void) { return t_last_error.c_str(); }

void fftenkf_debug_fail_next(int status) { t_fail_next = status; }

int fftenkf_profile_events(void* const* events, int n) {
  if (n == 0) {
    t_events_on = false;
    return FFTENKF_OK;
  }
  if ((n != 4 && n != 6) || events == nullptr) return fail(FFTENKF_EINVAL, "profile events: need an array of 4 or 6 events");
  for (int i = 0; i < n; ++i) {
    if (events[i] == nullptr) return fail(FFTENKF_EINVAL, "profile events: event %d is NULL", i);
    t_events[i] = static_cast<hipEvent_t>(events[i]);
  }
  t_nevents = n;
  t_events_on = true;
  return FFTENKF_OK;
}

int fftenkf_analyze(const fftenkf_ens* e, const void* data, const void* R_spec, uint64_t seed, void* out) {
  return analyze_impl(e, data, R_spec, seed, nullptr, nullptr, out);
}

int fftenkf_analyze_spectrum(const fftenkf_ens* e, const void* data, const void* R_spec, uint64_t seed, const void* lam,
                             void* out) {
  if (lam == nullptr) return fail(FFTENKF_EINVAL, "lam is NULL");
  return analyze_impl(e, data, R_spec, seed, nullptr, lam, out);
}

int fftenkf_analyze_learned(const fftenkf_ens* e, const void* data, const void* R_spec, uint64_t seed,
                            const fftenkf_mlp* mlp, void* out) {
  if (mlp == nullptr) return fail(FFTENKF_EINVAL, "mlp is NULL");
  if (e != nullptr && e->dtype != FFTENKF_F32) return fail(FFTENKF_EUNSUPPORTED, "the learned covariance is float32 only");
  return analyze_impl(e, data, R_spec, seed, mlp, nullptr, out);
}

int fftenkf_debug_spectra(const fftenkf_ens* e, const void* data, const void* R_spec, void* c_hat, void* gain,
                          void* spectra) {
  try {
    Plan plan;
    int st = validate_shape(e, &plan);
    if (st != FFTENKF_OK) return st;
    if (data == nullptr || c_hat == nullptr || gain == nullptr) return fail(FFTENKF_EINVAL, "data, c_hat and gain are required");
    const size_t s = dsize(e->dtype);
    const size_t plane = (size_t)e->ny * (e->nx / 2 + 1);
    const Ptr ptrs[] = {{e->members, (size_t)e->ny * e->nx * s * e->n_members, "members"},
                        {data, (size_t)e->ny * e->nx * s, "data"},
                        {R_spec, plane * s, "R_spec"},
                        {c_hat, plane * s, "c_hat"},
                        {gain, plane * s, "gain"},
                        {spectra, plane * 2 * s * (e->n_members + 1), "spectra"},
                        {e->workspace, plan.ws_bytes, "workspace"}};
    for (int i = 0; i < 7; ++i)
      for (int j = i + 1; j < 7; ++j)
        if (ptrs[i].p && ptrs[j].p && overlaps(ptrs[i].p, ptrs[i].bytes, ptrs[j].p, ptrs[j].bytes))
          return fail(FFTENKF_EINVAL, "%s overlaps %s", ptrs[i].name, ptrs[j].name);
    st = check_pointers(ptrs, 7);
    if (st != FFTENKF_OK) return st;
    return run(e, plan, data, R_spec, 0, nullptr, K2_DEBUG_SPECTRA, c_hat, gain, spectra, nullptr);
  } catch (...) {
    return fail(FFTENKF_EDEVICE, "internal error");
  }
}

int fftenkf_debug_perturb(const fftenkf_ens* e, const void* data, const void* R_spec, uint64_t seed, void* e_hat) {
  try {
    Plan plan;
    int st = validate_shape(e, &plan);
    if (st != FFTENKF_OK) return st;
    if (data == nullptr || e_hat == nullptr) return fail(FFTENKF_EINVAL, "data and e_hat are required");
    const size_t s = dsize(e->dtype);
    const size_t plane = (size_t)e->ny * (e->nx / 2 + 1);
    const Ptr ptrs[] = {{e->members, (size_t)e->ny * e->nx * s * e->n_members, "members"},
                        {data, (size_t)e->ny * e->nx * s, "data"},
                        {R_spec, plane * s, "R_spec"},
                        {e_hat, plane * 2 * s * e->n_members, "e_hat"},
                        {e->workspace, plan.ws_bytes, "workspace"}};
    for (int i = 0; i < 5; ++i)
      for (int j = i + 1; j < 5; ++j)
        if (ptrs[i].p && ptrs[j].p && overlaps(ptrs[i].p, ptrs[i].bytes, ptrs[j].p, ptrs[j].bytes))
          return fail(FFTENKF_EINVAL, "%s overlaps %s", ptrs[i].name, ptrs[j].name);
    st = check_pointers(ptrs, 5);
    if (st != FFTENKF_OK) return st;
    return run(e, plan, data, R_spec, seed, nullptr, K2_DEBUG_PERTURB, nullptr, nullptr, nullptr, e_hat);
  } catch (...) {
    return fail(FFTENKF_EDEVICE, "internal error");
  }
}

int fftenkf_debug_learned_spectrum(const fftenkf_ens* e, const void* data, const fftenkf_mlp* mlp, void* c_hat,
                                   void* lam_hat, void* mu) {
  try {
    Plan plan;
    int st = validate_shape(e, &plan);
    if (st != FFTENKF_OK) return st;
    if (e->dtype != FFTENKF_F32) return fail(FFTENKF_EUNSUPPORTED, "the learned covariance is float32 only");
    if (mlp == nullptr || data == nullptr || c_hat == nullptr || lam_hat == nullptr || mu == nullptr)
      return fail(FFTENKF_EINVAL, "data, mlp, c_hat, lam_hat and mu are required");
    const size_t plane = (size_t)e->ny * (e->nx / 2 + 1) * 4;
    const Ptr ptrs[] = {{e->members, (size_t)e->ny * e->nx * 4 * e->n_members, "members"},
                        {data, (size_t)e->ny * e->nx * 4, "data"},
                        {c_hat, plane, "c_hat"},
                        {lam_hat, plane, "lam_hat"},
                        {mu, 4, "mu"},
                        {e->workspace, plan.ws_bytes, "workspace"}};
    for (int i = 0; i < 6; ++i)
      for (int j = i + 1; j < 6; ++j)
        if (overlaps(ptrs[i].p, ptrs[i].bytes, ptrs[j].p, ptrs[j].bytes))
          return fail(FFTENKF_EINVAL, "%s overlaps %s", ptrs[i].name, ptrs[j].name);
    st = check_mlp(mlp, false);
    if (st == FFTENKF_OK) st = check_pointers(ptrs, 6);
    if (st == FFTENKF_OK) st = check_mlp(mlp, true);
    if (st != FFTENKF_OK) return st;
    return run(e, plan, data, nullptr, 0, nullptr, K2_STATS, nullptr, nullptr, nullptr, nullptr, mlp, c_hat, lam_hat,
               mu);
  } catch (...) {
    return fail(FFTENKF_EDEVICE, "internal error");
  }
}

int fftenkf_release_caches(void) { return FFTENKF_OK; }

int fftenkf_debug_fft2(const fftenkf_ens* e, int inverse, const void* spectra, void* out) {
  try {
    Plan plan;
    int st = validate_shape(e, &plan);
    if (st != FFTENKF_OK) return st;
    if (inverse != 0 && inverse != 1) return fail(FFTENKF_EINVAL, "inverse must be 0 or 1");
    if (out == nullptr || (inverse && spectra == nullptr)) return fail(FFTENKF_EINVAL, "out (and spectra for the inverse) required");
    if (misaligned(out, 16) || (spectra != nullptr && misaligned(spectra, 16)))
      return fail(FFTENKF_EINVAL, "spectra and out must be 16-byte aligned");
    const size_t s = dsize(e->dtype);
    const size_t fields = (size_t)e->ny * e->nx * s * e->n_members;
    const size_t specs = (size_t)e->ny * (e->nx / 2 + 1) * 2 * s * e->n_members;
    const Ptr ptrs[] = {{inverse ? nullptr : e->members, fields, "members"},
                        {inverse ? spectra : nullptr, specs, "spectra"},
                        {out, inverse ? fields : specs, "out"},
                        {e->workspace, plan.ws_bytes, "workspace"}};
    for (int i = 0; i < 4; ++i)
      for (int j = i + 1; j < 4; ++j)
        if (ptrs[i].p && ptrs[j].p && overlaps(ptrs[i].p, ptrs[i].bytes, ptrs[j].p, ptrs[j].bytes))
          return fail(FFTENKF_EINVAL, "%s overlaps %s", ptrs[i].name, ptrs[j].name);
    st = check_pointers(ptrs, 4);
    if (st != FFTENKF_OK) return st;
    return run_fft2(e, plan, inverse, spectra, out);
  } catch (...) {
    return fail(FFTENKF_EDEVICE, "internal error");
  }
}

int fftenkf_max_members_multi(int dtype) { return max_members_observed(dtype, 1); }

size_t fftenkf_workspace_bytes_multi(int n_members, int n_blocks, int ny, int nx, int dtype) {
  return fftenkf_workspace_bytes_morph(n_members, n_blocks, 1, ny, nx, dtype);
}

int fftenkf_analyze_multi(const fftenkf_ens* e, int n_blocks, const void* data, const void* R_spec, uint64_t seed,
                          void* out) {
  try {
    const double r = e != nullptr ? e->r_scalar : 0.0;
    return analyze_observed(e, n_blocks, 1, data, R_spec, &r, seed, out);
  } catch (...) {
    return fail(FFTENKF_EDEVICE, "internal error");
  }
}

int fftenkf_max_members_morph(int dtype, int n_obs) {
  if (n_obs < 1 || n_obs > kMaxObserved) return 0;
  return max_members_observed(dtype, n_obs);
}

size_t fftenkf_workspace_bytes_morph(int n_members, int n_blocks, int n_obs, int ny, int nx, int dtype) {
  if ((dtype != FFTENKF_F32 && dtype != FFTENKF_F64) || n_members < 2 || n_blocks < 1 || n_blocks > kMaxStateBlocks ||
      n_obs < 1 || n_obs > kMaxObserved || n_obs > n_blocks || !pow2_in_range(ny) || !pow2_in_range(nx))
    return 0;
  return make_plan(n_members * n_blocks + n_obs - 1, ny, nx, dtype).ws_bytes;
}

int fftenkf_analyze_morph(const fftenkf_ens* e, int n_blocks, int n_obs, const void* data, const void* R_spec,
                          const double* r_obs, uint64_t seed, void* out) {
  try {
    return analyze_observed(e, n_blocks, n_obs, data, R_spec, r_obs, seed, out);
  } catch (...) {
    return fail(FFTENKF_EDEVICE, "internal error");
  }
}

int fftenkf_tile_rows_options(int ny, int nx, int dtype, int* rows, int capacity) {
  if ((dtype != FFTENKF_F32 && dtype != FFTENKF_F64) || !pow2_in_range(ny) || !pow2_in_range(nx)) return 0;
  int all[4];
  const int n = tile_rows_options(dtype, nx, all);
  int k = 0;
  for (int i = 0; i < n; ++i)
    if (tile_rows_fit(all[i], ny)) {
      if (rows != nullptr && k < capacity) rows[k] = all[i];
      ++k;
    }
  return k;
}

int fftenkf_tile_rows(int ny, int nx, int dtype) {
  if ((dtype != FFTENKF_F32 && dtype != FFTENKF_F64) || !pow2_in_range(ny) || !pow2_in_range(nx)) return 0;
  return tile_rows(ny, nx, dtype);
}

int fftenkf_set_tile_rows(int ny, int nx, int dtype, int rows) {
  if ((dtype != FFTENKF_F32 && dtype != FFTENKF_F64) || !pow2_in_range(ny) || !pow2_in_range(nx))
    return fail(FFTENKF_EINVAL, "bad grid or dtype");
  std::lock_guard<std::mutex> lock(g_tune_mu);
  const auto key = std::make_tuple(ny, nx, dtype);
  if (rows == 0) {
    g_tune.erase(key);
    return FFTENKF_OK;
  }
  int all[4];
  const int n = tile_rows_options(dtype, nx, all);
  for (int i = 0; i < n; ++i)
    if (all[i] == rows && tile_rows_fit(rows, ny)) {
      g_tune[key] = rows;
      return FFTENKF_OK;
    }
  return fail(FFTENKF_EUNSUPPORTED, "%d tile rows are not compiled for a %d x %d grid of this dtype", rows, ny, nx);
}

int fftenkf_analyze_batch(int n_members, int dtype, const fftenkf_filter* filters, int n_filters, void* stream) {
  try {
    if (dtype != FFTENKF_F32 && dtype != FFTENKF_F64) return fail(FFTENKF_EINVAL, "dtype %d is not 0 or 1", dtype);
    if (n_members < 2) return fail(FFTENKF_EINVAL, "n_members = %d, eq. (2) needs N >= 2", n_members);
    if (k2_member_bucket(dtype, n_members) == 0)
      return fail(FFTENKF_EUNSUPPORTED, "n_members = %d exceeds %d for this dtype", n_members, fftenkf_max_members(dtype));
    if (n_filters < 0 || (n_filters > 0 && filters == nullptr)) return fail(FFTENKF_EINVAL, "filters is NULL");
    if (n_filters == 0) return FFTENKF_OK;
    std::vector<Plan> plans((size_t)n_filters);
    std::vector<Ptr> regions((size_t)n_filters * 5);
    for (int i = 0; i < n_filters; ++i) {
      const int st = validate_filter(filters[i], n_members, dtype, i, &plans[i]);
      if (st != FFTENKF_OK) return st;
      filter_regions(filters[i], n_members, dtype, plans[i], &regions[(size_t)i * 5]);
    }
    // what a filter writes (out, workspace) may overlap nothing else, except out
    // == members of the same filter (in place)
    for (int i = 0; i < n_filters; ++i)
      for (int w = 3; w < 5; ++w) {
        const Ptr& a = regions[(size_t)i * 5 + w];
        for (int j = 0; j < n_filters; ++j)
          for (int r = 0; r < 5; ++r) {
            if (i == j && r == w) continue;
            const Ptr& b = regions[(size_t)j * 5 + r];
            if (b.p == nullptr) continue;
            if (i == j && w == 3 && r == 0 && a.p == b.p) continue;
            if (overlaps(a.p, a.bytes, b.p, b.bytes))
              return fail(FFTENKF_EINVAL, "filter %d's %s overlaps filter %d's %s", i, a.name, j, b.name);
          }
      }
    int st = check_pointers(regions.data(), (int)regions.size());
    if (st != FFTENKF_OK) return st;
    for (int i = 0; i < n_filters && st == FFTENKF_OK; ++i)
      st = check_spectrum_values(filters[i].R_spec, (size_t)filters[i].ny * (filters[i].nx / 2 + 1), dtype,
                                 static_cast<hipStream_t>(stream), "R_spec");
    if (st != FFTENKF_OK) return st;
    return run_batch(n_members, dtype, filters, n_filters, plans, static_cast<hipStream_t>(stream));
  } catch (...) {
    return fail(FFTENKF_EDEVICE, "internal error");
  }
}

size_t fftenkf_workspace_bytes_dst(int n_members, int ny, int nx, int dtype) {
  if ((dtype != FFTENKF_F32 && dtype != FFTENKF_F64) || n_members < 2 || !pow2_in_range(ny) || !pow2_in_range(nx))
    return 0;
  return dst_ws_bytes(make_plan(n_members, ny, nx, dtype), n_members, ny, nx, dtype);
}

// Shared checks of the sine-basis entry points; the workspace includes the v planes.
int validate_dst(const fftenkf_ens* e, Plan* plan) {
  fftenkf_ens copy = *e;
  copy.workspace_bytes = (size_t)-1;  // checked below against the larger size
  int st = validate_shape(&copy, plan);
  if (st != FFTENKF_OK) return st;
  const size_t need = dst_ws_bytes(*plan, e->n_members, e->ny, e->nx, e->dtype);
  if (e->workspace_bytes < need) return fail(FFTENKF_EINVAL, "workspace of %zu bytes, %zu needed", e->workspace_bytes, need);
  return FFTENKF_OK;
}

int fftenkf_analyze_dst(const fftenkf_ens* e, const void* data, const void* R_dst, uint64_t seed, void* out) {
  try {
    if (e == nullptr) return fail(FFTENKF_EINVAL, "ens is NULL");
    Plan plan;
    int st = validate_dst(e, &plan);
    if (st != FFTENKF_OK) return st;
    if (data == nullptr || out == nullptr) return fail(FFTENKF_EINVAL, "data and out are required");
    if (misaligned(data, 16) || misaligned(out, 16) || (R_dst != nullptr && misaligned(R_dst, 16)))
      return fail(FFTENKF_EINVAL, "data, R_dst and out must be 16-byte aligned");
    if (R_dst == nullptr && (st = check_r_scalar(e->r_scalar, e->dtype, "")) != FFTENKF_OK) return st;
    const size_t s = dsize(e->dtype);
    const size_t field = (size_t)e->ny * e->nx * s;
    const size_t ens_b = field * e->n_members;
    const size_t ws_b = dst_ws_bytes(plan, e->n_members, e->ny, e->nx, e->dtype);
    const Ptr ptrs[] = {{e->members, ens_b, "members"},
                        {data, field, "data"},
                        {R_dst, field, "R_dst"},
                        {out, ens_b, "out"},
                        {e->workspace, ws_b, "workspace"}};
    for (int i = 0; i < 5; ++i)
      for (int j = i + 1; j < 5; ++j) {
        if (ptrs[i].p == nullptr || ptrs[j].p == nullptr) continue;
        const bool in_place = (i == 0 && j == 3 && ptrs[i].p == ptrs[j].p);
        if (!in_place && overlaps(ptrs[i].p, ptrs[i].bytes, ptrs[j].p, ptrs[j].bytes))
          return fail(FFTENKF_EINVAL, "%s overlaps %s", ptrs[i].name, ptrs[j].name);
      }
    st = check_pointers(ptrs, 5);
    if (st == FFTENKF_OK)
      st = check_spectrum_values(R_dst, (size_t)e->ny * e->nx, e->dtype, static_cast<hipStream_t>(e->stream), "R_dst");
    if (st != FFTENKF_OK) return st;
    return run_dst(e, plan, data, R_dst, seed, out, nullptr);
  } catch (...) {
    return fail(FFTENKF_EDEVICE, "internal error");
  }
}

int fftenkf_debug_dst_coeffs(const fftenkf_ens* e, const void* data, void* coeffs) {
  try {
    if (e == nullptr) return fail(FFTENKF_EINVAL, "ens is NULL");
    Plan plan;
    int st = validate_dst(e, &plan);
    if (st != FFTENKF_OK) return st;
    if (data == nullptr || coeffs == nullptr) return fail(FFTENKF_EINVAL, "data and coeffs are required");
    const size_t field = (size_t)e->ny * e->nx * dsize(e->dtype);
    const Ptr ptrs[] = {{e->members, field * e->n_members, "members"},
                        {data, field, "data"},
                        {coeffs, field * (e->n_members + 1), "coeffs"},
                        {e->workspace, dst_ws_bytes(plan, e->n_members, e->ny, e->nx, e->dtype), "workspace"}};
    for (int i = 0; i < 4; ++i)
      for (int j = i + 1; j < 4; ++j)
        if (overlaps(ptrs[i].p, ptrs[i].bytes, ptrs[j].p, ptrs[j].bytes))
          return fail(FFTENKF_EINVAL, "%s overlaps %s", ptrs[i].name, ptrs[j].name);
    st = check_pointers(ptrs, 4);
    if (st != FFTENKF_OK) return st;
    return run_dst(e, plan, data, nullptr, 0, nullptr, coeffs);
  } catch (...) {
    return fail(FFTENKF_EDEVICE, "internal error");
  }
}

}  // extern "C"
