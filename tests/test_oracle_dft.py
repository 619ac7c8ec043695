"""Pins of the oracle's DFT (step 1 of Section 2.1) against closed forms.

A sign, scale, transpose or index mistake in oracle/dft.py fails at least one
of these: the delta test fixes the sign and the axis order (non-square grid),
the constant test fixes the scale, the cosine test the bin placement, Parseval
the unitary normalisation, the round trip the inverse, the Hermitian test the
half-spectrum storage.
"""

import numpy as np
import pytest

from oracle import dft

SHAPES = [(8, 8), (4, 16), (16, 8), (12, 10), (32, 32)]


@pytest.mark.parametrize("method", ["matmul", "fft"])
@pytest.mark.parametrize("ny,nx", SHAPES)
def test_delta_is_phase_ramp(ny, nx, method):
    y0, x0 = 3 % ny, 5 % nx
    u = np.zeros((ny, nx))
    u[y0, x0] = 1.0
    S = dft.rdft2(u, method=method)
    ky = np.arange(ny)[:, None]
    kx = np.arange(nx // 2 + 1)[None, :]
    expect = np.exp(-2j * np.pi * (ky * y0 / ny + kx * x0 / nx)) / np.sqrt(ny * nx)
    assert np.allclose(S, expect, atol=1e-14, rtol=0)


@pytest.mark.parametrize("method", ["matmul", "fft"])
@pytest.mark.parametrize("ny,nx", SHAPES)
def test_constant_only_dc(ny, nx, method):
    S = dft.rdft2(np.full((ny, nx), 2.5), method=method)
    expect = np.zeros_like(S)
    expect[0, 0] = 2.5 * np.sqrt(ny * nx)
    assert np.allclose(S, expect, atol=1e-13, rtol=0)


@pytest.mark.parametrize("method", ["matmul", "fft"])
def test_cosine_two_bins(method):
    ny, nx, ky0, kx0 = 16, 32, 3, 5
    y = np.arange(ny)[:, None]
    x = np.arange(nx)[None, :]
    u = np.cos(2 * np.pi * (ky0 * y / ny + kx0 * x / nx))
    S = dft.rdft2(u, method=method)
    expect = np.zeros_like(S)
    expect[ky0, kx0] = np.sqrt(ny * nx) / 2       # the -k0 partner lives in the omitted half
    assert np.allclose(S, expect, atol=1e-12, rtol=0)
    # a cosine along y only: both +ky0 and -ky0 are stored in the kx = 0 column
    S2 = dft.rdft2(np.cos(2 * np.pi * ky0 * y / ny) * np.ones((1, nx)), method=method)
    expect2 = np.zeros_like(S2)
    expect2[ky0, 0] = expect2[ny - ky0, 0] = np.sqrt(ny * nx) / 2
    assert np.allclose(S2, expect2, atol=1e-12, rtol=0)


def _half_weights(nx):
    w = np.full(nx // 2 + 1, 2.0)
    w[0] = 1.0
    w[nx // 2] = 1.0
    return w


@pytest.mark.parametrize("ny,nx", SHAPES)
def test_parseval_unitary(ny, nx):
    rng = np.random.default_rng(7)
    u = rng.standard_normal((3, ny, nx))
    S = dft.rdft2(u)
    lhs = np.sum(u ** 2, axis=(1, 2))
    rhs = np.sum(_half_weights(nx)[None, None, :] * np.abs(S) ** 2, axis=(1, 2))
    assert np.allclose(lhs, rhs, rtol=1e-13)


@pytest.mark.parametrize("method", ["matmul", "fft"])
@pytest.mark.parametrize("ny,nx", SHAPES)
def test_round_trip_and_real(ny, nx, method):
    rng = np.random.default_rng(11)
    u = rng.standard_normal((2, ny, nx))
    back, imag = dft.irdft2(dft.rdft2(u, method=method), nx, method=method, return_imag=True)
    assert np.max(np.abs(back - u)) < 1e-13
    assert imag < 1e-12


@pytest.mark.parametrize("ny,nx", SHAPES)
def test_hermitian_edge_columns(ny, nx):
    rng = np.random.default_rng(3)
    S = dft.rdft2(rng.standard_normal((ny, nx)))
    for kx in {0, nx // 2}:
        for ky in range(ny):
            assert abs(S[ky, kx] - np.conj(S[(-ky) % ny, kx])) < 1e-13


def test_matmul_matches_fft_library():
    rng = np.random.default_rng(5)
    u = rng.standard_normal((2, 24, 40))
    assert np.allclose(dft.rdft2(u), np.fft.rfft2(u) / np.sqrt(24 * 40), atol=1e-13)
    S = dft.rdft2(u)
    assert np.allclose(dft.irdft2(S, 40), np.fft.irfft2(S * np.sqrt(24 * 40), s=(24, 40)), atol=1e-13)


def test_inverse_of_non_hermitian_edge_takes_real_part():
    """An inconsistent kx=0 column is read as its Hermitian part (the real part
    of the inverse), which is what a c2r transform does."""
    ny, nx = 8, 8
    S = np.zeros((ny, nx // 2 + 1), dtype=complex)
    S[1, 0] = 1.0 + 0.5j          # partner S[7, 0] left at 0
    full = dft.hermitian_extend(S, nx)
    z = np.fft.ifft2(full) * np.sqrt(ny * nx)
    assert np.allclose(dft.irdft2(S, nx), z.real, atol=1e-15)
    Sh = S.copy()
    Sh[1, 0] = 0.5 * (1.0 + 0.5j)
    Sh[7, 0] = np.conj(Sh[1, 0])
    assert np.allclose(dft.irdft2(S, nx), dft.irdft2(Sh, nx), atol=1e-15)
