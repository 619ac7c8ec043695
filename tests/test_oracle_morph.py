"""Pins of the extended-state (morphing) FFT EnKF oracle (Section 2.2, eq. (9)).

MO1 (per-bin spectral form with three diagonal observed covariances) against
MO2 (dense eq. (1) on the extended state with the observed cross-covariances
set to zero, assembled by lag sums with no DFT); the one-observed-field case
against the multi-block analysis; an all-observed state against single-block
analyses; the perturbation convention against the single-block stream."""

import numpy as np
import pytest

from oracle import enkf, morph, multiblock
from paper_1001_1588_amd import twin


def _case(ny, nx, N, M, K, seed, R_kind):
    tw = twin.make_multiblock_twin(ny, nx, N, seed=seed, Ls=tuple(float(2 + b) for b in range(M)), rho=0.5,
                                   r=0.05, dtype=np.float64)
    rng = np.random.default_rng(seed)
    data = tw.truth[:K] + np.sqrt(0.05) * rng.standard_normal((K, ny, nx))
    if R_kind == "scalar":
        R = np.array([0.05, 0.02, 0.1][:K])
        R_dense = list(R)
        R_spec = np.broadcast_to(R[:, None, None], (K, ny, nx // 2 + 1))
    else:
        ky = twin.integer_wavenumbers(ny)[:, None]
        kx = np.arange(nx // 2 + 1)[None, :].astype(np.float64)
        R_spec = np.stack([(0.02 + 0.01 * o) * (0.5 + 1.5 / (1.0 + (ky * ky + kx * kx) / (4.0 + o)))
                           for o in range(K)])
        R = R_spec
        R_dense = [enkf.stationary_matrix(R_spec[o], nx) for o in range(K)]
    return tw.ens, data, R, R_spec, R_dense, tw.seed


@pytest.mark.parametrize("ny,nx,N,M,K,R_kind", [(8, 8, 4, 4, 3, "scalar"), (8, 16, 5, 5, 3, "spectral"),
                                               (16, 8, 3, 3, 2, "spectral"), (8, 8, 4, 2, 1, "scalar")])
def test_spectral_equals_dense(ny, nx, N, M, K, R_kind):
    ens, data, R, R_spec, R_dense, seed = _case(ny, nx, N, M, K, seed=10 * ny + M, R_kind=R_kind)
    e_hat = morph.observed_perturbations(seed, N, R_spec, nx)
    o1 = morph.analyze_morph_spectral(ens, data, R, e_hat)
    e_phys = enkf.dft.irdft2(e_hat, nx)
    o2 = morph.analyze_morph_dense(ens, data, R_dense, e_phys)
    assert np.linalg.norm(o1 - o2) / np.linalg.norm(o2) < 1e-10


def test_one_observed_field_is_the_multiblock_analysis():
    ens, data, R, R_spec, R_dense, seed = _case(16, 16, 5, 4, 1, seed=3, R_kind="spectral")
    a = morph.analyze_morph(ens, data, R, seed)
    b = multiblock.analyze_multi(ens, data[0], R_spec[0], seed)
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-12


def test_all_observed_blocks_are_single_block_analyses():
    """M = K: every block is observed and, with the cross-covariances neglected,
    analysed on its own with its own data, error and noise stream; field 0
    draws exactly the single-block stream."""
    ens, data, R, R_spec, R_dense, seed = _case(16, 8, 4, 3, 3, seed=5, R_kind="spectral")
    out = morph.analyze_morph(ens, data, R, seed)
    e_hat = morph.observed_perturbations(seed, 4, R_spec, 8)
    for o in range(3):
        ref = enkf.analyze_spectral(ens[:, o], data[o], R_spec[o], e_hat[:, o])
        assert np.linalg.norm(out[:, o] - ref) / np.linalg.norm(ref) < 1e-12
    ref0 = enkf.analyze(ens[:, 0], data[0], R_spec[0], seed)
    assert np.linalg.norm(out[:, 0] - ref0) / np.linalg.norm(ref0) < 1e-12


def test_noise_streams():
    ny, nx, N, K = 32, 32, 6, 3
    z = morph.observed_noise(77, N, K, ny, nx)
    assert np.allclose(z[:, 0], enkf.spectral_noise(77, N, ny, nx), rtol=0, atol=0)
    for o in range(K):
        # unit variance of the unitary DFT of white noise: E|z|^2 = 1
        assert abs(np.mean(np.abs(z[:, o]) ** 2) - 1.0) < 0.05
    c = np.mean(z[:, 1] * np.conj(z[:, 2]))
    assert abs(c) < 0.05


def test_neglected_observed_cross_covariances_are_what_is_computed():
    """With correlated observed fields, keeping their cross-covariances in the
    dense solve gives a different analysis; neglecting them (the paper's three
    diagonal matrices) gives MO1."""
    ens, data, R, R_spec, R_dense, seed = _case(8, 8, 5, 4, 3, seed=21, R_kind="scalar")
    N, M, ny, nx = ens.shape
    n = ny * nx
    e_hat = morph.observed_perturbations(seed, N, R_spec, nx)
    e_phys = enkf.dft.irdft2(e_hat, nx)
    o1 = morph.analyze_morph_spectral(ens, data, R, e_hat)
    # the full joint solve: observed cross blocks kept
    C = np.zeros((M * n, M * n))
    for a in range(M):
        for b in range(M):
            C[a * n:(a + 1) * n, b * n:(b + 1) * n] = multiblock.circulant(
                multiblock.lag_cross_covariance(ens[:, a], ens[:, b]))
    H = np.zeros((3 * n, M * n))
    for o in range(3):
        H[o * n:(o + 1) * n, o * n:(o + 1) * n] = np.eye(n)
    Rb = np.kron(np.diag(R), np.eye(n))
    U = ens.reshape(N, M * n).T
    D = data.reshape(3 * n, 1) + e_phys.reshape(N, 3 * n).T
    full = (U + C @ H.T @ np.linalg.solve(H @ C @ H.T + Rb, D - H @ U)).T.reshape(N, M, ny, nx)
    assert np.linalg.norm(full - o1) / np.linalg.norm(o1) > 1e-3
    o2 = morph.analyze_morph_dense(ens, data, R_dense, e_phys)
    assert np.linalg.norm(o1 - o2) / np.linalg.norm(o2) < 1e-10
