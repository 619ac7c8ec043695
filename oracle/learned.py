"""Learned spectral covariance for the FFT EnKF: the plain reference form.

Test infrastructure only: the library never imports this module.

The estimator of eq. (2) replaced by a per-wavenumber multilayer perceptron:
for each stored bin of the half spectrum it reads the log sample spectrum in a
5 x 5 wavenumber neighbourhood plus |k| and returns an estimate lambda_hat of
the eigenvalue, which is then used in eq. (3) exactly where c_hat was.

Conventions (shared with the HIP kernels by specification only):

* mu = mean of c_hat over the ny * (nx/2+1) stored bins;
* feature j < 25: log(c_hat(ky + dy, kx + dx) / mu + 1e-6), (dy, dx) =
  (j div 5 - 2, j mod 5 - 2), indices taken on the full periodic spectrum, whose
  columns kx > nx/2 are the mirror c_hat(ny - ky, nx - kx) (c_hat is even);
* feature 25: log(1 + |k|), |k| = sqrt(ky'^2 + kx^2), ky' = min(ky, ny - ky);
* layers: h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), h3 = relu(h2 W3 + b3),
  y = h3 . w4 + b4; lambda_hat = mu exp(y);
* fallback: where mu is not a positive normal float32 the features do not
  exist and lambda_hat is the plain c_hat;
* precision: inputs, weights and the hidden activations that feed a product
  are rounded to bfloat16 (round to nearest, ties to even); products are
  accumulated in float64 here (float32 on the GPU); biases stay float32.
"""

from __future__ import annotations

import numpy as np

from . import dft
from .enkf import spectral_gain, spectral_mean_variance, spectral_perturbations, tiny_for

N_FEATURES = 26
EPS = 1e-6
MU_MIN = float(np.finfo(np.float32).tiny)  # smallest positive normal float32
MU_MAX = float(np.finfo(np.float32).max)


def round_bf16(x) -> np.ndarray:
    """Round float values to the nearest bfloat16 (ties to even), returned as float32."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    bits = a.view(np.uint32).astype(np.uint64)
    lsb = (bits >> np.uint64(16)) & np.uint64(1)
    rounded = ((bits + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    out = (rounded & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32)
    return np.where(np.isnan(a), a, out).reshape(np.shape(x))


def full_spectrum_even(c_half: np.ndarray, nx: int) -> np.ndarray:
    """Full [ny, nx] map of an even real spectrum stored as [ny, nx/2+1]."""
    ny, nh = c_half.shape
    full = np.empty((ny, nx), dtype=np.float64)
    full[:, :nh] = c_half
    ky = (-np.arange(ny)) % ny
    for kx in range(nh, nx):
        full[:, kx] = c_half[ky, nx - kx]
    return full


def features(c_half: np.ndarray, nx: int, mu: float | None = None) -> np.ndarray:
    """Input features [ny, nx/2+1, 26] of every stored bin."""
    c_half = np.asarray(c_half, dtype=np.float64)
    ny, nh = c_half.shape
    if mu is None:
        mu = float(c_half.mean())
    full = full_spectrum_even(c_half, nx)
    logc = np.log(full / mu + EPS)
    out = np.empty((ny, nh, N_FEATURES), dtype=np.float64)
    ky = np.arange(ny)[:, None]
    kx = np.arange(nh)[None, :]
    for j in range(25):
        dy, dx = j // 5 - 2, j % 5 - 2
        out[:, :, j] = logc[(ky + dy) % ny, (kx + dx) % nx]
    kyw = np.minimum(ky, ny - ky).astype(np.float64)
    out[:, :, 25] = np.log1p(np.sqrt(kyw * kyw + kx.astype(np.float64) ** 2))
    return out


def mlp(x: np.ndarray, w: dict, bf16: bool = True) -> np.ndarray:
    """The perceptron on features x[..., 26] -> y[...]; w has W1, b1, W2, b2, W3, b3, w4, b4."""
    r = round_bf16 if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    h = np.asarray(r(x), dtype=np.float64)
    for name in ("1", "2", "3"):
        W = np.asarray(r(w["W" + name]), dtype=np.float64)
        b = np.asarray(w["b" + name], dtype=np.float32).astype(np.float64)
        h = np.maximum(h @ W + b, 0.0)
        h = np.asarray(r(h.astype(np.float32)), dtype=np.float64) if bf16 else h
    w4 = np.asarray(r(w["w4"]), dtype=np.float64).reshape(-1)
    return h @ w4 + float(np.asarray(w["b4"], dtype=np.float32).reshape(-1)[0])


def learned_spectrum(c_half: np.ndarray, nx: int, w: dict, bf16: bool = True):
    """(lambda_hat [ny, nx/2+1], mu) from a sample spectrum c_half.

    The features divide by mu, so they exist only for a positive normal mu (in
    float32, the precision of the kernels); otherwise -- an ensemble without
    spread, or an overflowing one -- the estimate falls back to the plain
    sample spectrum, lambda_hat = c_hat."""
    c_half = np.asarray(c_half, dtype=np.float64)
    mu = float(c_half.mean())
    if not (MU_MIN <= mu <= MU_MAX):
        return c_half.copy(), mu
    y = mlp(features(c_half, nx, mu), w, bf16=bf16)
    return mu * np.exp(y), mu


def analyze_learned(ens, data, R_spec, seed: int, w: dict, *, method: str = "matmul", tiny=None,
                    return_parts: bool = False, bf16: bool = True):
    """Eq. (3) with the estimate lambda_hat of the perceptron in place of c_hat."""
    ens = np.asarray(ens)
    N, ny, nx = ens.shape
    if tiny is None:
        tiny = tiny_for(ens.dtype)
    R_spec = np.broadcast_to(np.asarray(R_spec, dtype=np.float64), (ny, nx // 2 + 1))
    u_hat = dft.rdft2(ens.astype(np.float64), method=method)
    d_hat = dft.rdft2(np.asarray(data, dtype=np.float64), method=method)
    _, c_hat = spectral_mean_variance(u_hat)
    lam, mu = learned_spectrum(c_hat, nx, w, bf16=bf16)
    K = spectral_gain(lam, R_spec, tiny)
    e_hat = spectral_perturbations(seed, N, R_spec, nx)
    ua = dft.irdft2(u_hat + K[None] * (d_hat[None] + e_hat - u_hat), nx, method=method)
    if return_parts:
        return ua, dict(c_hat=c_hat, lam=lam, mu=mu, K=K)
    return ua
