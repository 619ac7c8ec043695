"""The FFT EnKF analysis step (one block, H = I), and the dense EnKF it equals.

Two independent float64 forms:

O1 -- spectral form, in the paper's order (Section 2.1):
   step 1   u_hat_k = F u_k for every member, and d_hat = F d;
   eq. (2)  c_hat_i = 1/(N-1) sum_k |u_hat_ik - mean_k u_hat_ik|^2;
   eq. (3)  u_hat_k^a = u_hat_k + c_hat (c_hat + r)^-1 (d_hat + e_hat_k - u_hat_k),
            entry by entry, with r generalised to the eigenvalues R_spec of a
            stationary R (R = r I gives R_spec = r everywhere);
   then     u_k^a = F^-1 u_hat_k^a.
   F is the unitary DFT (see dft.py).

O2 -- dense form, eq. (1) with H = I:
   u_k^a = u_k + C_N (C_N + R)^-1 (d + e_k - u_k),
   where C_N is the stationary (circulant) covariance whose first column is the
   lag-averaged sample covariance c(h) = 1/n sum_x S(x + h, x), S the ensemble
   sample covariance.  Dropping the off-diagonal terms of the sample covariance
   in the frequency domain (Section 2.1) is exactly replacing S by this C_N: its
   eigenvalues are the c_hat of eq. (2).  O2 builds C_N by direct lag sums in
   physical space, with no DFT, and solves with a dense factorisation.

Perturbations e_k ~ N(0, R) (Section 2, after eq. (1)) are drawn in the
frequency domain with Philox4x32-10 and Box-Muller; the exact convention is
`spectral_noise`.
"""

from __future__ import annotations

import numpy as np

from . import dft
from .philox import box_muller, philox4x32


# --------------------------------------------------------------------- helpers

def tiny_for(dtype) -> float:
    """Smallest normal number of the input precision: below it the gain is 0."""
    return float(np.finfo(np.dtype(dtype)).tiny)


def special_masks(ny: int, nx: int):
    """Masks over the half spectrum [ny, nx//2+1].

    mirrored: bins in the kx = 0 and kx = nx/2 columns with ky > ny/2, whose
              value is the conjugate of the bin (ny - ky, kx) for a real field;
    selfconj: the four bins (ky, kx) with ky in {0, ny/2}, kx in {0, nx/2},
              which are real for a real field."""
    nh = nx // 2 + 1
    ky = np.arange(ny)[:, None] * np.ones((1, nh), dtype=np.int64)
    kx = np.ones((ny, 1), dtype=np.int64) * np.arange(nh)[None, :]
    edge = (kx == 0) | (kx == nx // 2)
    mirrored = edge & (ky > ny // 2)
    selfconj = edge & ((ky == 0) | (ky == ny // 2))
    return ky, kx, mirrored, selfconj


# ------------------------------------------------------------- perturbations

def spectral_noise(seed: int, N: int, ny: int, nx: int) -> np.ndarray:
    """Unit-variance spectral white noise z_hat[k, ky, kx] (complex128, half spectrum).

    z_hat is distributed as the unitary DFT of real white noise N(0, I):
      * generic bins: (a + i b) / sqrt(2);
      * self-conjugate bins: real, a in the kx = 0 column and b in the
        kx = nx/2 column, both from the kx = 0 bin's draw (the two real bins of
        a row ky in {0, ny/2} share one Box-Muller pair, as the real and
        imaginary parts of a generic bin do);
      * mirrored bins (see special_masks): the conjugate of the generating bin
        (ny - ky, kx), so the field it represents is real.
    (a, b) = Box-Muller of two words of Philox4x32-10 with
      key     = (seed mod 2^32, seed div 2^32),
      counter = (gy * (nx//2 + 1) + gx, k div 2, 0, 0), (gy, gx) the generating
                bin (gx = 0 for both self-conjugate bins of a row);
      member k uses words (x0, x1) when k is even and (x2, x3) when k is odd.
    """
    return _noise(seed, N, ny, nx, 0)


def _noise(seed: int, N: int, ny: int, nx: int, word3: int) -> np.ndarray:
    """spectral_noise with the fourth counter word set to word3."""
    nh = nx // 2 + 1
    ky, kx, mirrored, selfconj = special_masks(ny, nx)
    gy = np.where(mirrored, ny - ky, ky)
    nyq_sc = selfconj & (kx == nx // 2)
    lin = (gy * nh + np.where(nyq_sc, 0, kx)).astype(np.uint64)
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    z = np.empty((N, ny, nh), dtype=np.complex128)
    for k in range(N):
        words = philox4x32((lin, np.uint64(k // 2), np.uint64(0), np.uint64(word3)), key)
        wa, wb = (words[0], words[1]) if k % 2 == 0 else (words[2], words[3])
        a, b = box_muller(wa, wb)
        zk = np.where(selfconj, np.where(nyq_sc, b, a) + 0j, (a + 1j * b) / np.sqrt(2.0))
        z[k] = np.where(mirrored, np.conj(zk), zk)
    return z


def spectral_perturbations(seed: int, N: int, R_spec: np.ndarray, nx: int) -> np.ndarray:
    """e_hat_k = sqrt(R_spec) * z_hat_k: the unitary DFT of e_k ~ N(0, R)."""
    R_spec = np.asarray(R_spec, dtype=np.float64)
    ny = R_spec.shape[0]
    return np.sqrt(R_spec)[None] * spectral_noise(seed, N, ny, nx)


# ------------------------------------------------------------- O1, spectral

def spectral_mean_variance(u_hat: np.ndarray):
    """Eq. (2): mean_i and c_hat_i over the member axis 0 of u_hat[N, ...].

    The squared deviations of eq. (2) are summed over s_k = u_hat_k - u_hat_1,
    the members taken relative to the first one: subtracting a common value
    changes neither the deviations from the mean nor c_hat in exact arithmetic,
    and it makes c_hat exactly zero when every member is the same (a collapsed
    ensemble, whose gain eq. (3) then guards), which the plain mean need not."""
    N = u_hat.shape[0]
    if N < 2:
        raise ValueError("eq. (2) needs N >= 2")
    mean = u_hat.sum(axis=0) / N
    s = u_hat - u_hat[0:1]
    dev = s - s.sum(axis=0, keepdims=True) / N
    c_hat = (dev.real ** 2 + dev.imag ** 2).sum(axis=0) / (N - 1)
    return mean, c_hat


def spectral_gain(c_hat: np.ndarray, R_spec: np.ndarray, tiny: float) -> np.ndarray:
    """c_hat (c_hat + r)^-1 of eq. (3), entry by entry; 0 where c_hat + r < tiny."""
    den = c_hat + R_spec
    safe = np.where(den < tiny, 1.0, den)
    return np.where(den < tiny, 0.0, c_hat / safe)


def analyze_spectral(ens, data, R_spec, e_hat, *, method: str = "matmul", tiny=None,
                     return_parts: bool = False, lam=None):
    """O1 with given spectral perturbations e_hat[N, ny, nx//2+1] (unitary scale).

    lam, if given, is a prescribed covariance spectrum [ny, nx//2+1] used in the
    gain of eq. (3) in place of the estimate of eq. (2) (the filter with the
    known covariance of a twin experiment)."""
    ens = np.asarray(ens)
    N, ny, nx = ens.shape
    if tiny is None:
        tiny = tiny_for(ens.dtype)
    R_spec = np.broadcast_to(np.asarray(R_spec, dtype=np.float64), (ny, nx // 2 + 1))
    u_hat = dft.rdft2(ens.astype(np.float64), method=method)          # step 1
    d_hat = dft.rdft2(np.asarray(data, dtype=np.float64), method=method)
    mean, c_hat = spectral_mean_variance(u_hat)                        # eq. (2)
    cov = c_hat if lam is None else np.asarray(lam, dtype=np.float64)
    K = spectral_gain(cov, R_spec, tiny)                               # eq. (3), gain
    ua_hat = u_hat + K[None] * (d_hat[None] + e_hat - u_hat)           # eq. (3), update
    ua = dft.irdft2(ua_hat, nx, method=method)                         # F^-1
    if return_parts:
        return ua, dict(u_hat=u_hat, d_hat=d_hat, mean=mean, c_hat=c_hat, K=K, e_hat=e_hat, ua_hat=ua_hat)
    return ua


def analyze(ens, data, R_spec, seed: int, *, method: str = "matmul", tiny=None,
            return_parts: bool = False, lam=None):
    """O1: the FFT EnKF analysis with the seeded perturbation convention."""
    ens = np.asarray(ens)
    N, ny, nx = ens.shape
    R_spec = np.broadcast_to(np.asarray(R_spec, dtype=np.float64), (ny, nx // 2 + 1))
    e_hat = spectral_perturbations(seed, N, R_spec, nx)
    return analyze_spectral(ens, data, R_spec, e_hat, method=method, tiny=tiny, return_parts=return_parts, lam=lam)


# --------------------------------------------------------------- O2, dense

def lag_covariance(ens) -> np.ndarray:
    """c[hy, hx] = 1/n sum_x S(x + h, x) by direct sums over the grid (no DFT).

    S = 1/(N-1) sum_k (u_k - u_mean)(u_k - u_mean)^T; lags wrap periodically."""
    ens = np.asarray(ens, dtype=np.float64)
    N, ny, nx = ens.shape
    dev = ens - ens.mean(axis=0, keepdims=True)
    c = np.empty((ny, nx))
    for hy in range(ny):
        shifted_y = np.roll(dev, -hy, axis=1)
        for hx in range(nx):
            c[hy, hx] = np.sum(np.roll(shifted_y, -hx, axis=2) * dev)
    return c / ((N - 1) * ny * nx)


def circulant_matrix(c: np.ndarray) -> np.ndarray:
    """Dense [n, n] matrix C[i, j] = c((y_i - y_j) mod ny, (x_i - x_j) mod nx), i = y*nx + x."""
    ny, nx = c.shape
    y = np.repeat(np.arange(ny), nx)
    x = np.tile(np.arange(nx), ny)
    return c[(y[:, None] - y[None, :]) % ny, (x[:, None] - x[None, :]) % nx]


def sample_covariance(ens) -> np.ndarray:
    """Standard EnKF covariance: the dense ensemble sample covariance S [n, n]."""
    ens = np.asarray(ens, dtype=np.float64)
    N = ens.shape[0]
    D = (ens - ens.mean(axis=0, keepdims=True)).reshape(N, -1)
    return D.T @ D / (N - 1)


def analyze_dense(ens, data, R_dense, e_phys, C: np.ndarray) -> np.ndarray:
    """Eq. (1) with H = I and a given covariance C [n, n]; e_phys[N, ny, nx]."""
    ens = np.asarray(ens, dtype=np.float64)
    N, ny, nx = ens.shape
    n = ny * nx
    U = ens.reshape(N, n).T                                            # [n, N]
    innov = (np.asarray(data, dtype=np.float64).reshape(n, 1) + np.asarray(e_phys).reshape(N, n).T - U)
    R_dense = np.asarray(R_dense, dtype=np.float64)
    if R_dense.ndim == 0:
        R_dense = float(R_dense) * np.eye(n)
    X = np.linalg.solve(C + R_dense, innov)
    return (U + C @ X).T.reshape(N, ny, nx)


def analyze_dense_circulant(ens, data, R_dense, e_phys) -> np.ndarray:
    """O2: eq. (1) with H = I and C_N the circulant lag-averaged sample covariance."""
    return analyze_dense(ens, data, R_dense, e_phys, circulant_matrix(lag_covariance(ens)))


# ---------------------------------------------------- test-support helpers

def physical_perturbations(e_hat: np.ndarray, nx: int, method: str = "matmul") -> np.ndarray:
    """e_k = F^-1 e_hat_k (real fields)."""
    return dft.irdft2(e_hat, nx, method=method)


def stationary_matrix(R_spec: np.ndarray, nx: int) -> np.ndarray:
    """Dense stationary matrix whose eigenvalues are R_spec (half spectrum, even)."""
    R_spec = np.asarray(R_spec, dtype=np.float64)
    ny = R_spec.shape[0]
    first_col = dft.irdft2(R_spec.astype(np.complex128), nx) / np.sqrt(ny * nx)
    return circulant_matrix(first_col)


def mean_rmse(ens, truth) -> float:
    """Root-mean-square error of the ensemble mean against the truth."""
    m = np.asarray(ens, dtype=np.float64).mean(axis=0)
    return float(np.sqrt(np.mean((m - np.asarray(truth, dtype=np.float64)) ** 2)))
