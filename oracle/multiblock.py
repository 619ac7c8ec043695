"""Multi-block FFT EnKF (Section 2.2): the plain reference forms.

Test infrastructure only: the library never imports this module.

The state of each member is M blocks (fields on one grid), u_k = [u_k^(1); ..;
u_k^(M)], and only block 1 is observed (H = [I 0 .. 0]).  The EnKF, eq. (1),
becomes eq. (5): every block j moves by C^(j1) (C^(11) + R)^-1 times the
innovation d + e_k - u_k^(1) of block 1.  Two independent float64 forms:

MB1 -- spectral form, eq. (6): per bin i
   c_hat^(j1)_i = 1/(N-1) sum_k (u_hat^(j)_ik - mean^(j)_i) conj(u_hat^(1)_ik - mean^(1)_i),
   u_hat^(j)a_k = u_hat^(j)_k + c_hat^(j1) (c_hat^(11) + R_spec)^-1 (d_hat + e_hat_k - u_hat^(1)_k).
   The conjugate sits on the block-1 factor: these are the eigenvalues of the
   circulant cross-covariance below (for j = 1 the two placements agree, for
   j != 1 the other placement gives the complex conjugate).

MB2 -- dense form, eq. (5): C^(j1) is the circulant matrix whose first column
   is the lag-averaged cross sample covariance
     c^(j1)(h) = 1/n sum_x S^(j1)(x + h, x),
     S^(j1) = 1/(N-1) sum_k (u_k^(j) - mean^(j)) (u_k^(1) - mean^(1))^T,
   assembled by direct lag sums without any DFT, and the system with
   C^(11) + R is solved densely.

Perturbations are those of the single-block analysis (enkf.py), drawn for the
observed block.  Layout: ens [N][M][ny][nx] (member-major state vectors).
"""

from __future__ import annotations

import numpy as np

from . import dft
from .enkf import spectral_gain, spectral_perturbations, tiny_for


def cross_spectrum(u_hat_j: np.ndarray, u_hat_1: np.ndarray) -> np.ndarray:
    """c_hat^(j1) [ny, nx/2+1] from the unitary spectra [N, ny, nx/2+1] of blocks j and 1."""
    N = u_hat_j.shape[0]
    # deviations from the member mean, each block taken relative to its first
    # member first (the same in exact arithmetic; exactly zero for a collapsed block)
    sj = u_hat_j - u_hat_j[0:1]
    s1 = u_hat_1 - u_hat_1[0:1]
    dj = sj - sj.mean(axis=0, keepdims=True)
    d1 = s1 - s1.mean(axis=0, keepdims=True)
    return (dj * np.conj(d1)).sum(axis=0) / (N - 1)


def analyze_multi_spectral(ens, data, R_spec, e_hat, *, method: str = "matmul", tiny=None,
                           return_parts: bool = False):
    """MB1 with given spectral perturbations e_hat [N, ny, nx/2+1] (unitary scale)."""
    ens = np.asarray(ens)
    N, M, ny, nx = ens.shape
    if tiny is None:
        tiny = tiny_for(ens.dtype)
    R_spec = np.broadcast_to(np.asarray(R_spec, dtype=np.float64), (ny, nx // 2 + 1))
    u_hat = dft.rdft2(ens.astype(np.float64), method=method)          # [N, M, ny, nh]
    d_hat = dft.rdft2(np.asarray(data, dtype=np.float64), method=method)
    c11 = cross_spectrum(u_hat[:, 0], u_hat[:, 0]).real
    den = c11 + R_spec
    innov = d_hat[None] + e_hat - u_hat[:, 0]                          # [N, ny, nh]
    out_hat = np.empty_like(u_hat)
    gains = []
    for j in range(M):
        if j == 0:
            G = spectral_gain(c11, R_spec, tiny)                       # eq. (3) for the observed block
        else:
            cj1 = cross_spectrum(u_hat[:, j], u_hat[:, 0])
            # the guard of eq. (3): no update where c_hat^(11) + R underflows
            G = np.where(den < tiny, 0.0, cj1 / np.where(den < tiny, 1.0, den))
        gains.append(G)
        out_hat[:, j] = u_hat[:, j] + G[None] * innov
    ua = dft.irdft2(out_hat, nx, method=method)
    if return_parts:
        return ua, dict(u_hat=u_hat, d_hat=d_hat, c11=c11, gains=np.array(gains), innov=innov)
    return ua


def analyze_multi(ens, data, R_spec, seed: int, *, method: str = "matmul", tiny=None, return_parts: bool = False):
    """MB1 with the seeded perturbation convention of the single-block analysis."""
    ens = np.asarray(ens)
    N, M, ny, nx = ens.shape
    R_spec = np.broadcast_to(np.asarray(R_spec, dtype=np.float64), (ny, nx // 2 + 1))
    e_hat = spectral_perturbations(seed, N, R_spec, nx)
    return analyze_multi_spectral(ens, data, R_spec, e_hat, method=method, tiny=tiny, return_parts=return_parts)


def lag_cross_covariance(ens_j, ens_1) -> np.ndarray:
    """c^(j1)(h) [ny, nx]: lag average of the cross sample covariance, by direct sums."""
    a = np.asarray(ens_j, dtype=np.float64)
    b = np.asarray(ens_1, dtype=np.float64)
    N, ny, nx = a.shape
    a = a - a.mean(axis=0, keepdims=True)
    b = b - b.mean(axis=0, keepdims=True)
    c = np.empty((ny, nx))
    for hy in range(ny):
        for hx in range(nx):
            # sum_x a(x + h) b(x), summed over members
            c[hy, hx] = np.sum(np.roll(a, (-hy, -hx), axis=(1, 2)) * b)
    return c / ((N - 1) * ny * nx)


def circulant(c: np.ndarray) -> np.ndarray:
    """Dense [n, n] matrix M[x', x] = c(x' - x) (periodic), x = (y, x) row-major."""
    ny, nx = c.shape
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    y, x = y.ravel(), x.ravel()
    return c[(y[:, None] - y[None, :]) % ny, (x[:, None] - x[None, :]) % nx]


def analyze_multi_dense(ens, data, R_dense, e_phys) -> np.ndarray:
    """MB2: eq. (5) with the circulant cross-covariances; e_phys [N, ny, nx]."""
    ens = np.asarray(ens, dtype=np.float64)
    N, M, ny, nx = ens.shape
    n = ny * nx
    C11 = circulant(lag_cross_covariance(ens[:, 0], ens[:, 0]))
    R_dense = np.asarray(R_dense, dtype=np.float64)
    if R_dense.ndim == 0:
        R_dense = float(R_dense) * np.eye(n)
    innov = (np.asarray(data, dtype=np.float64).reshape(1, n) + np.asarray(e_phys).reshape(N, n)
             - ens[:, 0].reshape(N, n)).T                              # [n, N]
    X = np.linalg.solve(C11 + R_dense, innov)
    out = np.empty_like(ens)
    for j in range(M):
        Cj1 = circulant(lag_cross_covariance(ens[:, j], ens[:, 0]))
        out[:, j] = (ens[:, j].reshape(N, n).T + Cj1 @ X).T.reshape(N, ny, nx)
    return out
