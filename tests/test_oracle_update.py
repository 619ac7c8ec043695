"""Pins of eq. (3), the entrywise spectral update, and of the whole analysis.

* O1 (spectral, eq. (2)-(3)) equals O2 (dense eq. (1) with the circulant
  lag-averaged covariance, assembled without any DFT) on small grids;
* a single-mode ensemble is updated only in that mode, by the scalar Kalman
  formula; r -> infinity leaves the ensemble; r = 0 replaces the mode by the data;
* translation and scale equivariance, and invariance to a common added field.
"""

import numpy as np
import pytest

from oracle import dft, enkf
from paper_1001_1588_amd import twin

DENSE_CASES = [(4, 4, 2), (8, 16, 4), (16, 8, 3), (16, 16, 5), (32, 32, 5)]


@pytest.mark.parametrize("R_kind", ["scalar", "spectral"])
@pytest.mark.parametrize("ny,nx,N", DENSE_CASES)
def test_spectral_equals_dense_circulant(ny, nx, N, R_kind):
    tw = twin.random_ensemble(ny, nx, N, seed=ny * 100 + nx + N, dtype=np.float64, r=0.05, R_kind=R_kind)
    e_hat = enkf.spectral_perturbations(tw.seed, N, tw.R_spec, nx)
    o1 = enkf.analyze_spectral(tw.ens, tw.data, tw.R_spec, e_hat)
    e_phys = enkf.physical_perturbations(e_hat, nx)
    R_dense = 0.05 if R_kind == "scalar" else enkf.stationary_matrix(tw.R_spec, nx)
    o2 = enkf.analyze_dense_circulant(tw.ens, tw.data, R_dense, e_phys)
    rel = np.linalg.norm(o1 - o2) / np.linalg.norm(o2)
    assert rel < 1e-10


@pytest.mark.slow
def test_spectral_equals_dense_circulant_64():
    tw = twin.workload("small64", seed=2)
    N, ny, nx = tw.ens.shape
    e_hat = enkf.spectral_perturbations(tw.seed, N, tw.R_spec, nx)
    o1 = enkf.analyze_spectral(tw.ens, tw.data, tw.R_spec, e_hat)
    o2 = enkf.analyze_dense_circulant(tw.ens, tw.data, tw.r, enkf.physical_perturbations(e_hat, nx))
    assert np.linalg.norm(o1 - o2) / np.linalg.norm(o2) < 1e-10


def test_seeded_analyze_equals_explicit_perturbations():
    tw = twin.random_ensemble(8, 8, 3, seed=9, dtype=np.float64)
    e_hat = enkf.spectral_perturbations(tw.seed, 3, tw.R_spec, 8)
    assert np.array_equal(enkf.analyze(tw.ens, tw.data, tw.R_spec, tw.seed),
                          enkf.analyze_spectral(tw.ens, tw.data, tw.R_spec, e_hat))


def _mode_case(N=4, ny=16, nx=16, ky0=2, kx0=3, seed=0):
    rng = np.random.default_rng(seed)
    y = np.arange(ny)[:, None]
    x = np.arange(nx)[None, :]
    mode = np.cos(2 * np.pi * (ky0 * y / ny + kx0 * x / nx))
    base = 0.3 * np.sin(2 * np.pi * (y / ny)) + 0.1
    a = rng.standard_normal(N)
    ens = base[None] + a[:, None, None] * mode[None]
    delta = 0.7
    data = base + delta * mode
    return ens, data, a, delta, mode, base


def test_single_mode_scalar_kalman():
    ens, data, a, delta, mode, base = _mode_case()
    N, ny, nx = ens.shape
    r = 0.4
    zero = np.zeros((N, ny, nx // 2 + 1), dtype=complex)
    out = enkf.analyze_spectral(ens, data, r, zero)
    c = np.var(a, ddof=1) * (ny * nx) / 4           # unitary coefficient of a*cos is a*sqrt(n)/2
    K = c / (c + r)
    expect = base[None] + (a + K * (delta - a))[:, None, None] * mode[None]
    assert np.allclose(out, expect, atol=1e-12)


def test_limits_r_infinite_and_zero():
    ens, data, a, delta, mode, base = _mode_case(seed=1)
    N, ny, nx = ens.shape
    zero = np.zeros((N, ny, nx // 2 + 1), dtype=complex)
    out_inf = enkf.analyze_spectral(ens, data, 1e30, zero)
    assert np.allclose(out_inf, ens, atol=1e-12)
    out_0 = enkf.analyze_spectral(ens, data, 0.0, zero)
    assert np.allclose(out_0, np.broadcast_to(data, ens.shape), atol=1e-10)


def test_zero_spread_bin_gets_zero_gain():
    c = np.array([0.0, 0.0, 1.0, 1e-320])
    R = np.array([0.0, 1.0, 0.0, 0.0])
    K = enkf.spectral_gain(c, R, tiny=np.finfo(np.float64).tiny)
    assert np.array_equal(K, [0.0, 0.0, 1.0, 0.0])


def test_translation_equivariance_without_perturbation():
    tw = twin.random_ensemble(16, 32, 4, seed=4, dtype=np.float64)
    zero = np.zeros((4, 16, 17), dtype=complex)
    out = enkf.analyze_spectral(tw.ens, tw.data, tw.R_spec, zero)
    sh = (5, 11)
    out_s = enkf.analyze_spectral(np.roll(tw.ens, sh, axis=(1, 2)), np.roll(tw.data, sh, axis=(0, 1)), tw.R_spec, zero)
    assert np.allclose(out_s, np.roll(out, sh, axis=(1, 2)), atol=1e-12)


def test_scale_equivariance_with_seeded_perturbation():
    tw = twin.random_ensemble(16, 16, 5, seed=5, dtype=np.float64)
    alpha = 3.0
    out = enkf.analyze(tw.ens, tw.data, tw.R_spec, tw.seed)
    out_a = enkf.analyze(alpha * tw.ens, alpha * tw.data, alpha ** 2 * tw.R_spec, tw.seed)
    assert np.allclose(out_a, alpha * out, atol=1e-12)


def test_common_field_passes_through():
    tw = twin.random_ensemble(16, 16, 5, seed=6, dtype=np.float64)
    w = np.random.default_rng(1).standard_normal((16, 16))
    out = enkf.analyze(tw.ens, tw.data, tw.R_spec, tw.seed)
    out_w = enkf.analyze(tw.ens + w[None], tw.data + w, tw.R_spec, tw.seed)
    assert np.allclose(out_w, out + w[None], atol=1e-12)


def test_mean_update_without_perturbation():
    """With e = 0 the analysis mean obeys the same entrywise formula."""
    tw = twin.random_ensemble(8, 16, 6, seed=7, dtype=np.float64)
    zero = np.zeros((6, 8, 9), dtype=complex)
    out, parts = enkf.analyze_spectral(tw.ens, tw.data, tw.R_spec, zero, return_parts=True)
    m_hat = parts["mean"] + parts["K"] * (parts["d_hat"] - parts["mean"])
    assert np.allclose(out.mean(axis=0), dft.irdft2(m_hat, 16), atol=1e-12)


def test_fft_and_matmul_oracles_agree():
    tw = twin.random_ensemble(32, 16, 4, seed=8, dtype=np.float32)
    a = enkf.analyze(tw.ens, tw.data, tw.R_spec, tw.seed)
    b = enkf.analyze(tw.ens, tw.data, tw.R_spec, tw.seed, method="fft")
    assert np.linalg.norm(a - b) / np.linalg.norm(a) < 1e-13


def test_prescribed_spectrum_single_mode():
    """A prescribed flat spectrum lam0 gives the scalar gain lam0 / (lam0 + r) on the mode."""
    ens, data, a, delta, mode, base = _mode_case(seed=3)
    N, ny, nx = ens.shape
    r, lam0 = 0.4, 2.5
    zero = np.zeros((N, ny, nx // 2 + 1), dtype=complex)
    out = enkf.analyze_spectral(ens, data, r, zero, lam=np.full((ny, nx // 2 + 1), lam0))
    K = lam0 / (lam0 + r)
    expect = base[None] + (a + K * (delta - a))[:, None, None] * mode[None]
    assert np.allclose(out, expect, atol=1e-12)


@pytest.mark.parametrize("ny,nx,N", [(8, 8, 3), (16, 8, 4)])
def test_prescribed_spectrum_equals_dense_known_covariance(ny, nx, N):
    """Eq. (1) with the stationary covariance whose eigenvalues are lam, solved densely."""
    tw = twin.random_ensemble(ny, nx, N, seed=40 + ny, dtype=np.float64, r=0.05, R_kind="spectral")
    ky = twin.integer_wavenumbers(ny)[:, None]
    kx = np.arange(nx // 2 + 1)[None, :].astype(np.float64)
    lam = 1.0 / (1.0 + ky * ky + kx * kx)
    e_hat = enkf.spectral_perturbations(tw.seed, N, tw.R_spec, nx)
    o1 = enkf.analyze_spectral(tw.ens, tw.data, tw.R_spec, e_hat, lam=lam)
    o2 = enkf.analyze_dense(tw.ens, tw.data, enkf.stationary_matrix(tw.R_spec, nx),
                            enkf.physical_perturbations(e_hat, nx), enkf.stationary_matrix(lam, nx))
    assert np.linalg.norm(o1 - o2) / np.linalg.norm(o2) < 1e-10
