"""Pins of eq. (2), the spectral sample variance, and of the twin generator.

Closed forms (N = 2, identical members, common shifts), the definition the paper
gives in words (diagonal of the frequency-domain sample covariance, computed by
brute force from the dense sample covariance), the chi-square law of a Gaussian
ensemble, and convergence to the generating spectrum as N grows.
"""

import numpy as np
import pytest

from oracle import dft, enkf
from paper_1001_1588_amd import twin


def test_two_members_closed_form():
    rng = np.random.default_rng(0)
    u = rng.standard_normal((2, 8, 16))
    uh = dft.rdft2(u)
    _, c = enkf.spectral_mean_variance(uh)
    assert np.allclose(c, np.abs(uh[0] - uh[1]) ** 2 / 2, rtol=1e-13, atol=1e-15)


def test_identical_members_zero_and_common_shift_invariance():
    rng = np.random.default_rng(1)
    base = rng.standard_normal((8, 8))
    _, c0 = enkf.spectral_mean_variance(dft.rdft2(np.stack([base] * 4)))
    assert np.max(c0) < 1e-28
    u = rng.standard_normal((5, 8, 8))
    _, c1 = enkf.spectral_mean_variance(dft.rdft2(u))
    _, c2 = enkf.spectral_mean_variance(dft.rdft2(u + base[None]))
    assert np.allclose(c1, c2, rtol=1e-12, atol=1e-14)


def test_mean_is_member_average():
    rng = np.random.default_rng(2)
    u = rng.standard_normal((3, 4, 8))
    m, _ = enkf.spectral_mean_variance(dft.rdft2(u))
    assert np.allclose(m, dft.rdft2(u.mean(axis=0)), atol=1e-14)


def test_equals_diagonal_of_frequency_domain_sample_covariance():
    """Brute force from the words of Section 2.1: take the sample covariance,
    transform it to the frequency domain (F S F*), keep its diagonal."""
    rng = np.random.default_rng(3)
    N, ny, nx = 4, 4, 8
    u = rng.standard_normal((N, ny, nx))
    S = enkf.sample_covariance(u)
    Wy, Wx = dft.dft_matrix(ny), dft.dft_matrix(nx)
    F = np.kron(Wy, Wx) / np.sqrt(ny * nx)          # unitary 2D DFT on y*nx + x ordering
    diag = np.real(np.diag(F @ S @ F.conj().T)).reshape(ny, nx)[:, : nx // 2 + 1]
    _, c = enkf.spectral_mean_variance(dft.rdft2(u))
    assert np.allclose(c, diag, rtol=1e-12, atol=1e-14)


def test_eigenvalues_of_lag_covariance_are_spectral_variance():
    """The circulant C_N of the dense oracle has eigenvalues c_hat (eq. (2))."""
    rng = np.random.default_rng(4)
    u = rng.standard_normal((5, 8, 8))
    c = enkf.lag_covariance(u)
    eig = np.real(dft.rdft2(c)) * np.sqrt(64)        # eigenvalues of a circulant: unnormalised DFT of its column
    _, chat = enkf.spectral_mean_variance(dft.rdft2(u))
    assert np.allclose(eig, chat, rtol=1e-12, atol=1e-14)


def test_chi_square_law_gaussian_ensemble():
    """Gaussian members with spectrum lam: c_hat/lam has mean 1 and variance
    1/(N-1) on generic bins, 2/(N-1) on self-conjugate bins."""
    ny = nx = 16
    N = 6
    lam = twin.spectrum(ny, nx, "matern2", L=3.0)
    lam_h = lam[:, : nx // 2 + 1]
    _, _, _, selfconj = enkf.special_masks(ny, nx)
    rng = np.random.default_rng(5)
    ratios = []
    for _ in range(400):
        u = twin.gaussian_fields(rng, lam, N)
        _, c = enkf.spectral_mean_variance(dft.rdft2(u, method="fft"))
        ratios.append(c / lam_h)
    ratios = np.array(ratios)
    generic = ratios[:, ~selfconj]
    sc = ratios[:, selfconj]
    # ~50k generic bin draws: the standard error of the mean is about 0.002
    assert abs(generic.mean() - 1) < 0.02
    assert abs(generic.var() - 1 / (N - 1)) < 0.02
    assert abs(sc.mean() - 1) < 0.1
    assert abs(sc.var() - 2 / (N - 1)) < 0.1


def test_converges_to_generating_spectrum():
    ny = nx = 16
    lam = twin.spectrum(ny, nx, "matern2", L=2.0)
    lam_h = lam[:, : nx // 2 + 1]
    rng = np.random.default_rng(6)
    errs = []
    for N in (4, 16, 64, 256):
        u = twin.gaussian_fields(rng, lam, N)
        _, c = enkf.spectral_mean_variance(dft.rdft2(u, method="fft"))
        errs.append(np.mean(np.abs(c / lam_h - 1)))
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[3] < 0.12


@pytest.mark.parametrize("kind,kw", [("matern2", {}), ("power", {"a": 3.0})])
def test_twin_unit_variance_and_periodogram(kind, kw):
    ny = nx = 32
    lam = twin.spectrum(ny, nx, kind, **kw)
    assert abs(lam.mean() - 1) < 1e-12
    rng = np.random.default_rng(8)
    u = twin.gaussian_fields(rng, lam, 400)
    assert abs(u.var() - 1) < 0.05
    pg = np.mean(np.abs(np.fft.fft2(u) / np.sqrt(ny * nx)) ** 2, axis=0)
    mask = lam > 0
    assert np.mean(np.abs(pg[mask] / lam[mask] - 1)) < 0.1
    if kind == "power":
        assert np.max(np.abs(pg[0, 0])) < 1e-20


def test_twin_workloads_shapes():
    tw = twin.workload("small64", seed=3)
    assert tw.ens.shape == (5, 64, 64) and tw.ens.dtype == np.float64
    assert tw.R_spec.shape == (64, 33) and np.all(tw.R_spec == 0.01)
    tw2 = twin.workload("small64", seed=3)
    assert np.array_equal(tw.ens, tw2.ens) and tw.seed == tw2.seed
    tw3 = twin.workload("small64", seed=4)
    assert not np.array_equal(tw.ens, tw3.ens)
