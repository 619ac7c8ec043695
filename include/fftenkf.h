/*
 * fftenkf.h -- C ABI of the FFT EnKF analysis step on AMD Instinct MI355X (gfx950).
 *
 * The operation is the FFT EnKF of Mandel, Beezley and Kondratenko, Section 2.1,
 * for one block with H = I (the whole state observed) and a stationary data
 * error covariance R:
 *
 *   step 1   u_hat_k = F u_k for each of the N forecast members, d_hat = F d;
 *   eq. (2)  c_hat_i = 1/(N-1) sum_k |u_hat_ik - mean_k u_hat_ik|^2;
 *   eq. (3)  u_hat_k^a = u_hat_k + c_hat (c_hat + R_spec)^-1 (d_hat + e_hat_k - u_hat_k),
 *            entry by entry (R = r I gives R_spec = r everywhere);
 *   then     u_k^a = F^-1 u_hat_k^a.
 *
 * F is the 2D DFT of a periodic grid, normalised to be unitary, so c_hat and
 * R_spec are both eigenvalues of stationary covariances and the result does not
 * depend on how the FFTs are scaled internally.  The perturbations e_k ~ N(0, R)
 * of eq. (1) are drawn in the frequency domain, e_hat_k = sqrt(R_spec) z_hat_k,
 * with z_hat_k distributed as the unitary DFT of real white noise:
 *   - generic bins: (a + i b) / sqrt(2);
 *   - the four self-conjugate bins (ky in {0, ny/2}, kx in {0, nx/2}): a at
 *     kx = 0 and b at kx = nx/2, both from the draw of the bin (ky, 0);
 *   - bins in the kx = 0 and kx = nx/2 columns with ky > ny/2: the conjugate of
 *     the value drawn for (ny - ky, kx).
 * (a, b) = Box-Muller(u1, u2) with u = (2 * (w >> 9) + 1) * 2^-24 for words w of
 * Philox4x32-10 (Salmon et al., SC'11), key = (seed mod 2^32, seed div 2^32),
 * counter = (gy * (nx/2 + 1) + gx, k div 2, 0, 0) for the generating bin
 * (gy, gx) (gx = 0 for both self-conjugate bins of a row); member k takes
 * words (x0, x1) if k is even, (x2, x3) if odd.
 * The squared deviations of eq. (2) are formed from u_hat_k - u_hat_0, the
 * same sum in exact arithmetic, so c_hat is exactly 0 when all members are
 * equal; the gain is 0 where c_hat + R_spec is below the smallest normal number
 * of the working precision (no spread and no data error: no update).
 *
 * Layouts (row-major, x fastest):
 *   members / out : [N][ny][nx]  real, dtype        (device memory)
 *   data          : [ny][nx]     real, dtype        (device memory)
 *   R_spec        : [ny][nx/2+1] real, dtype        (device memory), or NULL
 *                   to use ens->r_scalar for every bin.  Values must be >= 0
 *                   and finite; in the kx = 0 and kx = nx/2 columns R_spec must
 *                   be even in ky (it is the spectrum of a real symmetric R).
 *                   r_scalar (used when R_spec is NULL) must be >= 0 and finite
 *                   in the working precision, else FFTENKF_EINVAL.
 * All device pointers must be 16-byte aligned; the workspace 256-byte aligned.
 *
 * Ownership: the caller owns every buffer.  The library keeps only per-device
 * twiddle tables in static device memory (no allocation).
 *
 * Errors: arguments are validated before anything is enqueued; on any error
 * nothing is written and the return value is negative.  NaN or Inf in the
 * numeric inputs is not checked and propagates, unless the environment
 * variable FFTENKF_CHECK is "1": then the analysis entry points first wait
 * for ens->stream, copy R_spec (and a prescribed lam) to the host and return
 * FFTENKF_EINVAL if any entry is negative, NaN or infinite.  No C++ exception
 * crosses this interface.  fftenkf_last_error() gives a message for the
 * calling thread.
 *
 * Concurrency: calls are asynchronous on ens->stream, like a kernel launch.
 * Two calls sharing a workspace must be ordered on one stream.
 */
#ifndef FFTENKF_H
#define FFTENKF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  FFTENKF_OK = 0,
  FFTENKF_EINVAL = -1,        /* null pointer, N < 2, bad dtype, aliasing, alignment, small workspace */
  FFTENKF_EUNSUPPORTED = -2,  /* grid not a power of two in [8, 4096], or N beyond the supported range */
  FFTENKF_EDEVICE = -3,       /* a HIP runtime call failed, or a pointer is not device memory */
  FFTENKF_ENOMEM = -4         /* reserved: the library allocates nothing today */
};

enum { FFTENKF_F32 = 0, FFTENKF_F64 = 1 };

typedef struct fftenkf_ens {
  int32_t n_members;      /* N, 2 <= N <= fftenkf_max_members(dtype) */
  int32_t ny, nx;         /* grid, each a power of two in [8, 4096] */
  int32_t dtype;          /* FFTENKF_F32 or FFTENKF_F64: members, data, R_spec and out */
  const void* members;    /* device [N][ny][nx] forecast ensemble u_k */
  void* workspace;        /* device scratch of at least fftenkf_workspace_bytes(...) bytes */
  size_t workspace_bytes; /* size of workspace in bytes */
  void* stream;           /* hipStream_t to enqueue on; NULL means the default stream */
  double r_scalar;        /* R = r_scalar * I when R_spec is NULL */
} fftenkf_ens;

/*
 * One FFT EnKF analysis, eq. (3) with the estimator of eq. (2) (Section 2.1).
 * out may equal ens->members (in place); any other overlap of out, data,
 * R_spec, members and workspace is FFTENKF_EINVAL.  Enqueued on ens->stream;
 * synchronise the stream before reading out.  Same inputs and seed give
 * bitwise-identical output.
 */
int fftenkf_analyze(const fftenkf_ens* ens, const void* data, const void* R_spec, uint64_t seed, void* out);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the analysis
 * of fftenkf_analyze with the same arguments, except that ens->workspace and
 * ens->workspace_bytes are ignored.  The workspace is instead a static device
 * array of fftenkf_noalloc_max_bytes() bytes (64 MiB) that the library holds on
 * every device it runs on until the process ends; its address on a device is
 * looked up on the first call there (with that device current).  Shapes whose
 * fftenkf_workspace_bytes exceeds that size (e.g. more than 13 members on a
 * 1024 x 1024 grid in float32) return FFTENKF_EINVAL without enqueuing
 * anything.  No call allocates: nothing in the array needs to start at zero
 * (sweep 1 writes every element the later sweeps read).  All calls on one GPU
 * share the array, which keeps the last call's contents: two calls that may
 * overlap in time on one GPU (different streams, or different host threads
 * without ordering) race and give undefined results; order them on one stream.
 * Same kernels, so the output is bitwise that of fftenkf_analyze.
 */
int fftenkf_analyze_noalloc(const fftenkf_ens* ens, const void* data, const void* R_spec, uint64_t seed, void* out);

/* Size in bytes of the static scratch array of fftenkf_analyze_noalloc. */
size_t fftenkf_noalloc_max_bytes(void);

/* Bytes of workspace fftenkf_analyze and fftenkf_analyze_learned need: (N+1)
 * spectra of ny*(nx/2+1) complex values, two ny*(nx/2+1) real planes and one
 * float per unit of the spectral sweep, rounded up to 256; 0 if the shape is invalid. */
size_t fftenkf_workspace_bytes(int n_members, int ny, int nx, int dtype);

/*
 * Learned spectral covariance: a per-wavenumber perceptron replaces the
 * estimator of eq. (2) in eq. (3).  For each stored bin it reads
 * x_j = log(c_hat(ky + dy, kx + dx) / mu + 1e-6), (dy, dx) = (j/5 - 2, j%5 - 2),
 * j < 25 (indices on the full periodic spectrum, c_hat even), and
 * x_25 = log(1 + |k|) with |k| = sqrt(min(ky, ny-ky)^2 + kx^2); then
 * h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), h3 = relu(h2 W3 + b3),
 * y = h3 . w4 + b4 and lambda_hat = mu exp(y), mu = mean of c_hat over the
 * ny*(nx/2+1) stored bins.  The gain is lambda_hat / (lambda_hat + R_spec);
 * lambda_hat need not be even in ky, and in the kx = 0 and kx = nx/2 columns
 * the update is that of the mean of the gains at (ky, kx) and (ny - ky, kx),
 * which is what the inverse real transform of the updated half spectrum gives.
 * Inputs, weights and hidden activations are rounded to bfloat16 (nearest,
 * ties to even); products accumulate in float32 on the matrix cores.  Where mu
 * is not a positive normal float (no spread anywhere) the features do not
 * exist and lambda_hat falls back to the plain c_hat.
 * All eight pointers are device float32 arrays, row-major [in][out].
 */
typedef struct fftenkf_mlp {
  const float* W1; /* [26][64] */
  const float* b1; /* [64] */
  const float* W2; /* [64][64] */
  const float* b2; /* [64] */
  const float* W3; /* [64][64] */
  const float* b3; /* [64] */
  const float* w4; /* [64] */
  const float* b4; /* [1] */
} fftenkf_mlp;

/* As fftenkf_analyze, with lambda_hat from the perceptron in place of c_hat
 * (float32 only).  Same arguments, ownership and error behaviour. */
int fftenkf_analyze_learned(const fftenkf_ens* ens, const void* data, const void* R_spec, uint64_t seed,
                            const fftenkf_mlp* mlp, void* out);

/* As fftenkf_analyze, with the covariance eigenvalues prescribed: lam is a
 * device [ny][nx/2+1] array of dtype (unitary DFT scale, the same scale as
 * R_spec) used in eq. (3) in place of the estimate of eq. (2), e.g. the known
 * spectrum of a twin experiment; in the kx = 0 and kx = nx/2 columns the gains
 * at (ky, kx) and (ny - ky, kx) are averaged, as for fftenkf_analyze_learned.
 * Same arguments and error behaviour. */
int fftenkf_analyze_spectrum(const fftenkf_ens* ens, const void* data, const void* R_spec, uint64_t seed,
                             const void* lam, void* out);

/*
 * Multi-block analysis (Section 2.2): every member is a state of M blocks
 * (fields) on one grid and only block 0 is observed (H = [I 0 .. 0]).  Eq. (5)
 * in the frequency domain, eq. (6): for every block j and bin
 *   u_hat^(j)a_k = u_hat^(j)_k + c_hat^(j0) / (c_hat^(00) + R_spec) (d_hat + e_hat_k - u_hat^(0)_k),
 *   c_hat^(j0) = 1/(N-1) sum_k (u_hat^(j)_k - mean^(j)) conj(u_hat^(0)_k - mean^(0)),
 * the spectral cross-covariance of eq. (7) with the conjugate on the observed
 * factor, which makes c_hat^(j0) the eigenvalues of the circulant
 * (lag-averaged) cross-covariance of block j with block 0; the printed form
 * conjugates the other factor, which gives their complex conjugates.  Block 0
 * gets exactly the single-block update of fftenkf_analyze, and e_hat_k follows
 * the same seeded convention.
 *   ens->members, out : [N][M][ny][nx]  (member-major state vectors)
 *   data              : [ny][nx], observes block 0
 *   R_spec            : [ny][nx/2+1] or NULL (ens->r_scalar), as for fftenkf_analyze
 *   workspace         : fftenkf_workspace_bytes_multi(N, M, ny, nx, dtype) bytes
 * 1 <= n_blocks <= 64 and 2 <= N <= fftenkf_max_members_multi(dtype).  Other
 * rules (alignment, overlap, in place, errors) as for fftenkf_analyze.
 */
int fftenkf_analyze_multi(const fftenkf_ens* ens, int n_blocks, const void* data, const void* R_spec, uint64_t seed,
                          void* out);

/* Workspace bytes of fftenkf_analyze_multi; 0 if the arguments are invalid. */
size_t fftenkf_workspace_bytes_multi(int n_members, int n_blocks, int ny, int nx, int dtype);

/* Largest N of fftenkf_analyze_multi for a dtype. */
int fftenkf_max_members_multi(int dtype);

/*
 * The FFT EnKF step of the morphing EnKF (Section 2.2, eq. (9)): the analysis
 * of an extended state of M blocks whose first K (1 <= K <= 3) are observed,
 * each by its own data d_o and stationary error R_o, with the
 * cross-covariances among the observed blocks neglected, so that their
 * covariance is K diagonal matrices in the frequency domain (in the paper,
 * the extended state (T, r(1), .., r(M)) with T_x, T_y and r(1) observed).
 * Per bin:
 *   observed block o:   u^(o)a_k = u^(o)_k + c^(oo) / (c^(oo) + R_o) (d_o + e_ko - u^(o)_k),
 *   unobserved block j: u^(j)a_k = u^(j)_k + sum_o c^(jo) / (c^(oo) + R_o) (d_o + e_ko - u^(o)_k),
 * with c^(oo) from eq. (2) and c^(jo) from eq. (7) (conjugate on the observed
 * factor), and no update from field o where c^(oo) + R_o is below the smallest
 * normal number.  e_ko ~ N(0, R_o), independent across o, follows the
 * convention of fftenkf_analyze with the fourth Philox counter word set to o
 * (so o = 0 draws the single-block stream).  With K = 1 this is
 * fftenkf_analyze_multi.  The registration that produces the extended state
 * and the inverse morphing transform are the caller's.
 *   ens->members, out : [N][M][ny][nx]  (member-major extended states)
 *   data              : [K][ny][nx], block o observed by data[o]
 *   R_spec            : [K][ny][nx/2+1] eigenvalues of each R_o, or NULL to
 *                       use r_obs (host array of K doubles, R_o = r_obs[o] I;
 *                       each >= 0 and finite in the working precision)
 *   workspace         : fftenkf_workspace_bytes_morph(N, M, K, ny, nx, dtype) bytes
 * 2 <= N <= fftenkf_max_members_morph(dtype, K), 1 <= K <= min(3, M) and
 * M <= 64; other rules (alignment, overlap, in place, errors) as for
 * fftenkf_analyze.
 */
int fftenkf_analyze_morph(const fftenkf_ens* ens, int n_blocks, int n_obs, const void* data, const void* R_spec,
                          const double* r_obs, uint64_t seed, void* out);

/* Workspace bytes of fftenkf_analyze_morph; 0 if the arguments are invalid. */
size_t fftenkf_workspace_bytes_morph(int n_members, int n_blocks, int n_obs, int ny, int nx, int dtype);

/* Largest N of fftenkf_analyze_morph for a dtype and number of observed blocks (0 if invalid). */
int fftenkf_max_members_morph(int dtype, int n_obs);

/*
 * A batch of independent analyses (eq. (3) with eq. (2), exactly as
 * fftenkf_analyze, one per filter) with one member count and dtype but grids
 * of any supported sizes.  Filters on the same grid share launches: each of the
 * three sweeps runs once per grid size for up to 40 filters at a time, the
 * filter selected by the second grid dimension, and the per-filter arguments
 * travel by value in the launch, so the whole batch can be captured in a HIP
 * graph (stream capture) and replayed; FFTENKF_CHECK must then be unset, since
 * its check synchronises the stream.  Each filter's output is bitwise equal to
 * fftenkf_analyze on the same arguments.
 */
typedef struct fftenkf_filter {
  int32_t ny, nx;         /* grid of this filter, powers of two in [8, 4096] */
  const void* members;    /* device [N][ny][nx] */
  const void* data;       /* device [ny][nx] */
  const void* R_spec;     /* device [ny][nx/2+1], or NULL for r_scalar */
  void* out;              /* device [N][ny][nx]; may equal members */
  void* workspace;        /* device, fftenkf_workspace_bytes(N, ny, nx, dtype) bytes, 256-byte aligned */
  size_t workspace_bytes;
  double r_scalar;        /* R = r_scalar * I when R_spec is NULL */
  uint64_t seed;          /* perturbations of this filter (the convention of fftenkf_analyze) */
} fftenkf_filter;

/* Enqueues every filter's analysis on `stream` (hipStream_t, NULL = default).
 * Arguments are validated first (as for fftenkf_analyze, per filter; what a
 * filter writes may overlap no other buffer of the batch); on error nothing is
 * enqueued.  When the batch has more than one launch chain (more than one grid
 * size, or more than 40 filters of one), the chains run on up to three
 * library-owned streams of the device, forked from `stream` by an event and
 * joined back into it: work queued on `stream` before the call happens before
 * the batch and work queued after it sees the finished outputs, as with a
 * single stream, and under stream capture the fork and join become graph
 * dependencies.  The streams are made on the first such call outside a
 * capture (until then, and if they cannot be made, the chains run one after
 * another on `stream`) and kept until the process ends; batches issued on
 * different streams share them and so run one after the other. */
int fftenkf_analyze_batch(int n_members, int dtype, const fftenkf_filter* filters, int n_filters, void* stream);

/*
 * Tile schedule.  The y transform is split as ny = R * L between sweeps 1/3 (R
 * rows per tile, a radix-R stage in registers) and sweep 2 (length-L
 * transforms).  fftenkf_tile_rows_options lists the R compiled for a grid and
 * dtype (up to `capacity` of them into `rows`; returns how many there are);
 * fftenkf_set_tile_rows chooses one for every later call on that grid and
 * dtype in this process (0 restores the default; FFTENKF_EUNSUPPORTED if not
 * compiled); fftenkf_tile_rows returns the R in use.  The workspace size
 * depends on R: query it after choosing.  Default: R = 16 for float32 grids
 * 2048 wide, else 8 (float64: 8, or 4 for grids 4096 wide), at most ny.
 */
int fftenkf_tile_rows_options(int ny, int nx, int dtype, int* rows, int capacity);
int fftenkf_set_tile_rows(int ny, int nx, int dtype, int rows);
int fftenkf_tile_rows(int ny, int nx, int dtype);

/*
 * The analysis in the real sine basis (Section 4, whose experiment uses a sine
 * transform so that the analysis leaves the boundary values unchanged).  The
 * transform is the orthonormal 2D DST-II,
 *   S[k][j] = sqrt(2/n) c_k sin(pi (2j + 1)(k + 1) / (2n)),  c_{n-1} = 1/sqrt(2), else 1,
 * per axis, whose basis functions vanish at the cell faces j = -1/2, n - 1/2;
 * eq. (2) and eq. (3) act on its real coefficients:
 *   c_hat = 1/(N-1) sum_k (s_hat_k - mean)^2,
 *   s_hat_k^a = s_hat_k + c_hat / (c_hat + R_dst) (d_hat + e_hat_k - s_hat_k),
 * and the analysis is S^T s_hat_k^a.  e_hat_k = sqrt(R_dst) z with z drawn per
 * sine bin (s1, s2) from Philox4x32-10, key as for fftenkf_analyze, counter
 * (s1 * nx + s2, k div 4, 1, 0): Box-Muller on words (x0, x1) gives members
 * 4q and 4q + 1 (its cosine and its sine output), on words (x2, x3) members
 * 4q + 2 and 4q + 3, where q = k div 4.
 *   R_dst : device [ny][nx] real, the eigenvalues of R in the sine basis (>= 0),
 *           or NULL to use ens->r_scalar;
 *   workspace : fftenkf_workspace_bytes_dst(N, ny, nx, dtype) bytes.
 * Other arguments and rules as for fftenkf_analyze (same N limits).
 */
int fftenkf_analyze_dst(const fftenkf_ens* ens, const void* data, const void* R_dst, uint64_t seed, void* out);

/* Workspace bytes of fftenkf_analyze_dst and fftenkf_debug_dst_coeffs (the
 * same as fftenkf_workspace_bytes); 0 if invalid. */
size_t fftenkf_workspace_bytes_dst(int n_members, int ny, int nx, int dtype);

/* Test-only: the orthonormal sine coefficients [N+1][ny][nx] (members, then
 * data) that fftenkf_analyze_dst works on, into device `coeffs`. */
int fftenkf_debug_dst_coeffs(const fftenkf_ens* ens, const void* data, void* coeffs);

/* Releases cached library state.  The library keeps only its twiddle tables,
 * which are static device arrays filled on first use and live until the
 * process ends, so there is nothing to free: returns FFTENKF_OK. */
int fftenkf_release_caches(void);

/* Largest N the analysis supports for a dtype. */
int fftenkf_max_members(int dtype);

/* Static description of a status code, and the last error message of this thread. */
const char* fftenkf_strerror(int status);
const char* fftenkf_last_error(void);

/*
 * Test-only exports.  They run the same kernels as fftenkf_analyze.
 *
 * fftenkf_debug_spectra: after the forward transforms, writes per bin the
 *   estimator c_hat of eq. (2) and the gain c_hat/(c_hat + R_spec) of eq. (3)
 *   (device [ny][nx/2+1] real each), and, if spectra is not NULL, the unitary
 *   half spectra of the N members followed by d (device [N+1][ny][nx/2+1]
 *   complex, interleaved re/im).  ens->members is not modified.
 * fftenkf_debug_perturb: writes e_hat_k (device [N][ny][nx/2+1] complex), the
 *   unitary-scale spectral perturbations drawn for `seed` (Section 2, eq. (1)).
 * fftenkf_debug_fail_next: the next validated call of this thread returns
 *   `status` without enqueuing anything (forces the device-failure path).
 */
int fftenkf_debug_spectra(const fftenkf_ens* ens, const void* data, const void* R_spec, void* c_hat,
                          void* gain, void* spectra);
int fftenkf_debug_perturb(const fftenkf_ens* ens, const void* data, const void* R_spec, uint64_t seed,
                          void* e_hat);
void fftenkf_debug_fail_next(int status);

/* Test-only: the 2D transform of the analysis on its own (Section 2.1, step 1
 * and the inverse F^-1).  inverse == 0: out (device [N][ny][nx/2+1] complex of
 * dtype) receives the unitary half spectra of ens->members; `spectra` is not
 * read.  inverse == 1: out (device [N][ny][nx] real) receives the real inverse
 * of the unitary half spectra in `spectra` ([N][ny][nx/2+1] complex): the real
 * part of the inverse transform of their Hermitian extension, so the imaginary
 * parts of the kx = 0 and kx = nx/2 bins act through their Hermitian part
 * only; ens->members must be non-NULL but is not read.  Uses the workspace. */
int fftenkf_debug_fft2(const fftenkf_ens* ens, int inverse, const void* spectra, void* out);

/* Test-only: c_hat (eq. (2)) and lambda_hat (the perceptron) per stored bin,
 * device [ny][nx/2+1] float each, and mu (device, one float); float32 only. */
int fftenkf_debug_learned_spectrum(const fftenkf_ens* ens, const void* data, const fftenkf_mlp* mlp, void* c_hat,
                                   void* lam_hat, void* mu);

/*
 * Profiling hook for the calling thread.  With n == 4, the next
 * fftenkf_analyze, fftenkf_analyze_spectrum or fftenkf_analyze_multi records
 * events[0] before sweep 1,
 * events[1] between sweeps 1 and 2, events[2] between sweeps 2 and 3 and
 * events[3] after sweep 3.  With n == 6, the next fftenkf_analyze_learned
 * records them around its five launches (sweep 1, the statistics sweep, the
 * perceptron, the update sweep, sweep 3).  Events are hipEvent_t created by the
 * caller, recorded on ens->stream; the hook is forgotten after that call (or
 * after any call it does not fit).  n == 0 clears it.  Returns FFTENKF_EINVAL
 * for any other n or a NULL array.
 */
int fftenkf_profile_events(void* const* events, int n);

#ifdef __cplusplus
}
#endif

#endif /* FFTENKF_H */
