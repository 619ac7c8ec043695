"""Pins of oracle/dst.py, the analysis in the real sine basis (Section 4).

* the DST-II matrix against scipy.fft.dst(type=2, norm="ortho") (an
  independent library implementation), its orthogonality, and the closed form
  of a pure sine mode;
* the basis vanishes half a cell outside the grid (zero change on the boundary);
* eq. (2)-(3) in the sine basis equals the dense EnKF with the sine-diagonal
  covariance; a single-mode ensemble gets the scalar Kalman update; r -> inf
  leaves the ensemble;
* the perturbations: the Philox convention's statistics (white, unit variance)
  and their independence from the periodic analysis' stream.
"""

import numpy as np
import pytest
import scipy.fft as sf

from oracle import dst, enkf
from paper_1001_1588_amd import twin


@pytest.mark.parametrize("n", [1, 2, 5, 8, 16, 33])
def test_matrix_is_scipy_orthonormal_dst2(n):
    S = dst.dst2_matrix(n)
    assert np.allclose(S, sf.dst(np.eye(n), type=2, norm="ortho", axis=0), atol=1e-14)
    assert np.allclose(S @ S.T, np.eye(n), atol=1e-13)


def test_2d_transform_matches_scipy_and_inverts():
    x = np.random.default_rng(1).standard_normal((3, 8, 16))
    assert np.allclose(dst.dst2(x), sf.dstn(x, type=2, norm="ortho", axes=(-2, -1)), atol=1e-13)
    assert np.allclose(dst.idst2(dst.dst2(x)), x, atol=1e-13)


def test_pure_sine_mode_and_boundary():
    ny, nx, k1, k2 = 8, 16, 2, 5
    j1 = np.arange(ny)[:, None] + 0.5
    j2 = np.arange(nx)[None, :] + 0.5
    mode = np.sin(np.pi * j1 * (k1 + 1) / ny) * np.sin(np.pi * j2 * (k2 + 1) / nx)
    s = dst.dst2(mode)
    expect = np.zeros((ny, nx))
    expect[k1, k2] = np.sqrt(ny * nx) / 2
    assert np.allclose(s, expect, atol=1e-12)
    # every basis function is a sine through zero at the faces -1/2 and n - 1/2
    for k in range(ny):
        f = lambda x: np.sin(np.pi * (2 * x + 1) * (k + 1) / (2 * ny))  # noqa: E731
        assert abs(f(-0.5)) < 1e-15 and abs(f(ny - 0.5)) < 1e-12


@pytest.mark.parametrize("ny,nx,N,R_kind", [(4, 4, 3, "scalar"), (8, 8, 4, "spectral"), (8, 16, 5, "scalar")])
def test_sine_basis_update_equals_dense(ny, nx, N, R_kind):
    tw = twin.random_ensemble(ny, nx, N, seed=ny + nx + N, dtype=np.float64, r=0.05)
    R = 0.05 * (1.0 + np.arange(ny * nx).reshape(ny, nx) % 3) if R_kind == "spectral" else 0.05
    ua, parts = dst.analyze_dst(tw.ens, tw.data, R, tw.seed, return_parts=True)
    dense = dst.analyze_dst_dense(tw.ens, tw.data, R, parts["e_hat"])
    assert np.linalg.norm(ua - dense) / np.linalg.norm(dense) < 1e-11


def test_single_sine_mode_scalar_kalman_and_limits():
    ny, nx, N = 8, 8, 5
    rng = np.random.default_rng(3)
    S = np.kron(dst.dst2_matrix(ny), dst.dst2_matrix(nx))
    mode = S[3 * nx + 6].reshape(ny, nx)                          # a unit sine basis field
    base = rng.standard_normal((ny, nx))
    a = rng.standard_normal(N)
    ens = base[None] + a[:, None, None] * mode[None]
    data = base + 0.4 * mode
    r = 0.3
    ua, parts = dst.analyze_dst(ens, data, r, 9, return_parts=True)
    e = parts["e_hat"][:, 3, 6]
    c = np.var(a, ddof=1)
    K = c / (c + r)
    s_other = dst.dst2(ua - base[None])
    s_other[:, 3, 6] -= a + K * (0.4 + e - a)
    # the moving mode follows the scalar Kalman formula; every other bin has zero
    # spread, hence zero gain, and stays
    assert np.allclose(s_other, 0.0, atol=1e-10)
    inf = dst.analyze_dst(ens, data, 1e30, 9)
    assert np.allclose(inf, ens, atol=1e-12)


def test_noise_convention_statistics():
    z = dst.dst_noise(123, 6, 64, 64)
    assert abs(z.mean()) < 0.02 and abs(z.var() - 1) < 0.02
    # members are uncorrelated (0, 1: the two outputs of one Box-Muller pair;
    # 0, 2: the two pairs of one Philox call; 0, 4: different calls) and bins are white
    for j in (1, 2, 3, 4, 5):
        assert abs(np.corrcoef(z[0].ravel(), z[j].ravel())[0, 1]) < 0.03
    assert abs(np.corrcoef(z[0, :, :-1].ravel(), z[0, :, 1:].ravel())[0, 1]) < 0.03
    # a different stream from the periodic analysis' perturbations
    per = enkf.spectral_noise(123, 2, 64, 64)
    assert not np.allclose(z[0, :8, :8], per[0, :8, :8].real * np.sqrt(2))


def test_fft_method_equals_matrices():
    x = np.random.default_rng(7).standard_normal((2, 16, 32))
    assert np.allclose(dst.dst2(x, "fft"), dst.dst2(x), atol=1e-12)
    assert np.allclose(dst.idst2(x, "fft"), dst.idst2(x), atol=1e-12)
    tw = twin.random_ensemble(16, 32, 4, seed=3, dtype=np.float64)
    a = dst.analyze_dst(tw.ens, tw.data, 0.02, 5, method="fft")
    b = dst.analyze_dst(tw.ens, tw.data, 0.02, 5)
    assert np.allclose(a, b, atol=1e-12)
