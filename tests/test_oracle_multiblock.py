"""Pins of oracle/multiblock.py, the multi-block analysis (Section 2.2).

* MB1 (spectral, eq. (6) with the conjugate on the block-1 factor) equals MB2
  (dense eq. (5) with circulant cross-covariances assembled by lag sums, no DFT);
* with one block it is the single-block analysis of eq. (2)-(3);
* a block that is block 1 shifted by s is updated as block 1's update shifted by s;
* a block equal to a * block 1 + b (a common field b) moves by a times block 1's move;
* the twin generator's blocks have the stated spectra and coherence.
"""

import numpy as np
import pytest

from oracle import dft, enkf, multiblock
from paper_1001_1588_amd import twin


@pytest.mark.parametrize("ny,nx,N,M,R_kind", [(4, 4, 3, 2, "scalar"), (8, 8, 4, 3, "spectral"),
                                              (8, 16, 5, 2, "spectral"), (16, 8, 3, 4, "scalar")])
def test_spectral_equals_dense(ny, nx, N, M, R_kind):
    tw = twin.make_multiblock_twin(ny, nx, N, seed=ny * 10 + M, Ls=(1.0, 2.0, 3.0, 4.0)[:M], dtype=np.float64)
    R_spec = tw.R_spec
    if R_kind == "spectral":
        ky = twin.integer_wavenumbers(ny)[:, None]
        kx = np.arange(nx // 2 + 1)[None, :].astype(np.float64)
        R_spec = 0.02 * (0.5 + 1.5 / (1.0 + ky * ky + kx * kx))
    e_hat = enkf.spectral_perturbations(tw.seed, N, R_spec, nx)
    o1 = multiblock.analyze_multi_spectral(tw.ens, tw.data, R_spec, e_hat)
    R_dense = enkf.stationary_matrix(R_spec, nx)
    o2 = multiblock.analyze_multi_dense(tw.ens, tw.data, R_dense, enkf.physical_perturbations(e_hat, nx))
    assert np.linalg.norm(o1 - o2) / np.linalg.norm(o2) < 1e-10


def test_printed_conjugation_differs_from_dense():
    """Conjugating the block-j factor instead gives the complex-conjugate gain; it is not eq. (5)."""
    tw = twin.make_multiblock_twin(8, 8, 4, seed=3, Ls=(1.0, 2.0), dtype=np.float64)
    u_hat = dft.rdft2(tw.ens.astype(np.float64))
    right = multiblock.cross_spectrum(u_hat[:, 1], u_hat[:, 0])
    swapped = np.conj(right)
    assert np.max(np.abs(right.imag)) > 1e-3 * np.max(np.abs(right))
    dense = multiblock.circulant(multiblock.lag_cross_covariance(tw.ens[:, 1], tw.ens[:, 0]))
    # eigenvalues of the circulant cross-covariance, by applying it to DFT basis vectors
    ny, nx = 8, 8
    for (ky, kx) in [(1, 2), (3, 1), (0, 3)]:
        y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        v = np.exp(2j * np.pi * (ky * y / ny + kx * x / nx)).ravel()
        lam = (dense @ v)[0] / v[0]
        assert abs(lam - right[ky, kx]) < 1e-12
        assert abs(lam - swapped[ky, kx]) > 1e-6


@pytest.mark.parametrize("ny,nx,N", [(16, 16, 4), (8, 32, 5)])
def test_one_block_is_the_single_block_analysis(ny, nx, N):
    tw = twin.random_ensemble(ny, nx, N, seed=ny + nx, dtype=np.float64, R_kind="spectral")
    single = enkf.analyze(tw.ens, tw.data, tw.R_spec, tw.seed)
    multi = multiblock.analyze_multi(tw.ens[:, None], tw.data, tw.R_spec, tw.seed)
    assert np.allclose(multi[:, 0], single, atol=1e-12)


def test_shifted_block_follows_block_one():
    tw = twin.random_ensemble(16, 16, 5, seed=8, dtype=np.float64)
    s = (3, 5)
    ens = np.stack([tw.ens, np.roll(tw.ens, s, axis=(1, 2))], axis=1)
    out = multiblock.analyze_multi(ens, tw.data, tw.R_spec, tw.seed)
    assert np.allclose(out[:, 1], np.roll(out[:, 0], s, axis=(1, 2)), atol=1e-12)


def test_affine_block_moves_proportionally():
    tw = twin.random_ensemble(16, 8, 4, seed=9, dtype=np.float64)
    b = np.random.default_rng(0).standard_normal((16, 8))
    ens = np.stack([tw.ens, -2.5 * tw.ens + b[None]], axis=1)
    out = multiblock.analyze_multi(ens, tw.data, tw.R_spec, tw.seed)
    assert np.allclose(out[:, 1] - ens[:, 1], -2.5 * (out[:, 0] - ens[:, 0]), atol=1e-12)


def test_multiblock_twin_statistics():
    ny = nx = 64
    tw = twin.make_multiblock_twin(ny, nx, 200, seed=1, Ls=(2.0, 8.0), rho=0.6, dtype=np.float64)
    dev = tw.ens - tw.ens.mean(axis=0, keepdims=True)
    u = np.fft.rfft2(dev, norm="ortho")
    p0 = (np.abs(u[:, 0]) ** 2).sum(axis=0) / 199
    p1 = (np.abs(u[:, 1]) ** 2).sum(axis=0) / 199
    x01 = (u[:, 1] * np.conj(u[:, 0])).sum(axis=0) / 199
    lam0, lam1 = tw.lam[0][:, : nx // 2 + 1], tw.lam[1][:, : nx // 2 + 1]
    # averaged over bins: spectra as stated (relative error ~ 1/sqrt(200 * bins)) and coherence 0.6
    assert abs(np.mean(p0 / lam0) - 1) < 0.02 and abs(np.mean(p1 / lam1) - 1) < 0.02
    coh = np.mean(x01.real / np.sqrt(lam0 * lam1))
    assert abs(coh - 0.6) < 0.02
