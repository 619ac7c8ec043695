"""Plain discrete Fourier transforms for the oracle (float64 / complex128).

The paper's step 1 (Section 2.1) applies "an FFT operator F" to each member; the
FFT only computes the DFT faster, so the oracle writes the DFT out as a matrix
product with exact twiddles.  F is taken *unitary* (1/sqrt(n) on both the
forward and the inverse transform): that is the scale on which the spectral
variance of eq. (2) estimates the eigenvalues of a stationary covariance, and on
which it can be added to the eigenvalues of R in eq. (3).

Two interchangeable evaluation methods are offered:

* ``"matmul"`` (default): the DFT matrix W[j, k] = exp(-2 pi i ((j k) mod m) / m),
  integer reduction first so every twiddle is correctly rounded, applied by BLAS.
* ``"fft"``: numpy.fft (pocketfft) as a library primitive, for full-size cases.

Both are checked against closed forms in the tests, and against each other.

Half spectra are stored as [..., ny, nx//2 + 1] (x is the last axis).  The
inverse of a half spectrum S is Re(F^-1 ext(S)) where ext fills the missing
columns kx > nx/2 by Hermitian symmetry, ext(S)[ky, kx] = conj(S[-ky, nx-kx]).
"""

from __future__ import annotations

import numpy as np

_CACHE: dict = {}


def dft_matrix(m: int, sign: int = -1) -> np.ndarray:
    """W[j, k] = exp(sign * 2 pi i ((j*k) mod m) / m), complex128, unnormalised."""
    key = (m, sign)
    if key not in _CACHE:
        j = np.arange(m, dtype=np.int64)
        idx = np.outer(j, j) % m
        ang = (2.0 * np.pi / m) * idx.astype(np.float64)
        _CACHE[key] = np.cos(ang) + 1j * sign * np.sin(ang)
    return _CACHE[key]


def rdft2(u: np.ndarray, method: str = "matmul") -> np.ndarray:
    """Unitary forward 2D DFT of real fields u[..., ny, nx] -> half spectrum [..., ny, nx//2+1]."""
    u = np.asarray(u, dtype=np.float64)
    ny, nx = u.shape[-2:]
    nh = nx // 2 + 1
    scale = 1.0 / np.sqrt(ny * nx)
    if method == "fft":
        return np.fft.rfft2(u, axes=(-2, -1)) * scale
    if method != "matmul":
        raise ValueError(method)
    wx = dft_matrix(nx)[:, :nh]                  # [x, kx]
    wy = dft_matrix(ny)                          # [ky, y]
    # contiguous real and imaginary parts, so the products go to BLAS
    wx_re, wx_im = np.ascontiguousarray(wx.real), np.ascontiguousarray(wx.imag)
    along_x = u @ wx_re + 1j * (u @ wx_im)       # [..., y, kx]
    return (wy @ along_x) * scale                # [..., ky, kx]


def hermitian_extend(S: np.ndarray, nx: int) -> np.ndarray:
    """Full spectrum [..., ny, nx] from a half spectrum [..., ny, nx//2+1]."""
    ny, nh = S.shape[-2:]
    if nh != nx // 2 + 1:
        raise ValueError("half-spectrum width does not match nx")
    full = np.empty(S.shape[:-1] + (nx,), dtype=np.complex128)
    full[..., :nh] = S
    ky = (-np.arange(ny)) % ny
    for kx in range(nh, nx):
        full[..., :, kx] = np.conj(S[..., ky, nx - kx])
    return full


def irdft2(S: np.ndarray, nx: int, method: str = "matmul", return_imag: bool = False):
    """Unitary inverse 2D DFT of a half spectrum: Re(F^-1 ext(S)) as real [..., ny, nx].

    With return_imag=True also returns max |Im| of F^-1 ext(S) (zero when S is
    the half spectrum of a real field, up to rounding)."""
    S = np.asarray(S, dtype=np.complex128)
    ny = S.shape[-2]
    scale = 1.0 / np.sqrt(ny * nx)
    full = hermitian_extend(S, nx)
    if method == "fft":
        z = np.fft.ifft2(full, axes=(-2, -1)) * (ny * nx) * scale
    elif method == "matmul":
        z = (dft_matrix(ny, +1) @ full @ dft_matrix(nx, +1)) * scale
    else:
        raise ValueError(method)
    if return_imag:
        return z.real.copy(), float(np.max(np.abs(z.imag))) if z.size else 0.0
    return z.real.copy()


def dft2_full(u: np.ndarray, sign: int = -1, method: str = "matmul") -> np.ndarray:
    """Unitary full 2D DFT of complex or real fields [..., ny, nx]."""
    u = np.asarray(u, dtype=np.complex128)
    ny, nx = u.shape[-2:]
    scale = 1.0 / np.sqrt(ny * nx)
    if method == "fft":
        if sign < 0:
            return np.fft.fft2(u, axes=(-2, -1)) * scale
        return np.fft.ifft2(u, axes=(-2, -1)) * (ny * nx) * scale
    return (dft_matrix(ny, sign) @ u @ dft_matrix(nx, sign)) * scale
