"""Pins of the oracle on degenerate ensembles: the gain guard of eq. (3).

Reading of the paper: eq. (3) divides by c_hat + r.  Where both vanish -- an
ensemble without spread and no data error at a wavenumber -- the gain is taken
as 0 (no information, no update).  These cases check that reading with closed
forms that hold in exact arithmetic:

* identical members have c_hat = 0 exactly (eq. (2) is summed over deviations
  from the first member), so with R = 0 on some bins and R > 0 elsewhere every
  gain is 0 and the analysis returns the forecast;
* without the guard the same case is 0/0 (NaN), so the guard is load-bearing;
* members that are constant fields c_k and R = 0: only the mean wavenumber has
  spread, so its gain is exactly 1 and every other gain 0, and every member
  becomes the constant mean of the data.  The oracle's matrix DFT leaves
  rounding noise of about 1e-16 in bins that are zero in exact arithmetic, so
  its threshold is raised above that noise (1e-20) to reach the exact answer;
* the multi-block form (Section 2.2) with constant blocks: block j moves by
  cov(b, c) / var(c) times the innovation of block 1 at the mean wavenumber;
* the sine-basis form (Section 4) and the learned covariance on a collapsed
  ensemble return the forecast.
"""

import numpy as np
import pytest

from oracle import dst, enkf, learned, multiblock


def _masked_R(ny, nx, rng):
    """R_spec that is 0 on a subset of bins -- every self-conjugate bin, the
    kx = 0 and kx = nx/2 columns, a random scatter -- and positive elsewhere."""
    nh = nx // 2 + 1
    R = rng.uniform(0.01, 0.1, (ny, nh))
    R[:, 0] = 0.0
    R[:, nh - 1] = 0.0
    R[rng.random((ny, nh)) < 0.3] = 0.0
    # keep R even in ky on the edge columns (already zero there)
    return R


@pytest.mark.parametrize("N", [2, 3, 5])
def test_identical_members_have_exactly_zero_spread(N):
    rng = np.random.default_rng(N)
    base = rng.standard_normal((16, 32))
    ens = np.stack([base] * N)
    _, c = enkf.spectral_mean_variance(enkf.dft.rdft2(ens))
    assert np.all(c == 0.0)
    s = dst.dst2(ens)
    rel = s - s[0:1]
    assert np.all(((rel - rel.mean(axis=0)) ** 2).sum(axis=0) == 0.0)
    uh = enkf.dft.rdft2(ens)
    assert np.all(multiblock.cross_spectrum(uh, uh) == 0.0)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_collapsed_ensemble_with_zero_R_returns_forecast(dtype):
    rng = np.random.default_rng(7)
    ny, nx, N = 16, 32, 4
    base = rng.standard_normal((ny, nx)).astype(dtype)
    ens = np.stack([base] * N)
    data = rng.standard_normal((ny, nx)).astype(dtype)
    R = _masked_R(ny, nx, rng)
    out, parts = enkf.analyze(ens, data, R, seed=3, return_parts=True)
    assert np.all(parts["K"] == 0.0)
    assert np.max(np.abs(out - ens)) < 1e-12
    # without the guard the zero-R bins are 0/0
    with np.errstate(invalid="ignore", divide="ignore"):
        bad = enkf.analyze(ens, data, R, seed=3, tiny=0.0)
    assert np.isnan(bad).any()


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_constant_members_zero_R_take_the_data_mean(dtype):
    rng = np.random.default_rng(8)
    ny, nx = 16, 8
    c = np.array([0.5, -1.25, 2.0, 0.75, -0.25])
    ens = (c[:, None, None] * np.ones((1, ny, nx))).astype(dtype)
    data = rng.standard_normal((ny, nx)).astype(dtype)
    out, parts = enkf.analyze(ens, data, 0.0, seed=5, tiny=1e-20, return_parts=True)
    K = parts["K"]
    assert K[0, 0] == 1.0
    K0 = K.copy()
    K0[0, 0] = 0.0
    assert np.all(K0 == 0.0)
    expect = np.full(ens.shape, data.astype(np.float64).mean())
    assert np.max(np.abs(out - expect)) < 1e-12


def test_multiblock_constant_blocks_closed_form():
    rng = np.random.default_rng(9)
    ny, nx, N = 8, 16, 4
    c = np.array([0.5, -1.0, 1.5, 0.25])             # observed block
    b = np.array([[2.0, 0.0, -1.0, 1.0], [0.25, 0.5, 0.75, -0.5]])
    blocks = [c] + list(b)
    ens = np.stack([np.stack([blk[k] * np.ones((ny, nx)) for blk in blocks]) for k in range(N)])
    data = rng.standard_normal((ny, nx))
    out = multiblock.analyze_multi(ens, data, 0.0, seed=2, tiny=1e-20)
    dm = data.mean()
    for j, blk in enumerate(blocks):
        g = np.cov(blk, c)[0, 1] / np.var(c, ddof=1)
        expect = blk[:, None, None] + g * (dm - c)[:, None, None]
        assert np.max(np.abs(out[:, j] - expect)) < 1e-12


def test_multiblock_collapsed_with_zero_R_returns_forecast():
    rng = np.random.default_rng(10)
    ny, nx, N, M = 8, 8, 3, 3
    base = rng.standard_normal((M, ny, nx))
    ens = np.stack([base] * N)
    data = rng.standard_normal((ny, nx))
    out = multiblock.analyze_multi(ens, data, _masked_R(ny, nx, rng), seed=4)
    assert np.max(np.abs(out - ens)) < 1e-12


def test_sine_basis_collapsed_with_zero_R_returns_forecast():
    rng = np.random.default_rng(11)
    ny, nx, N = 8, 16, 5
    base = rng.standard_normal((ny, nx))
    ens = np.stack([base] * N)
    data = rng.standard_normal((ny, nx))
    R = rng.uniform(0.01, 0.1, (ny, nx))
    R[rng.random((ny, nx)) < 0.5] = 0.0
    out, parts = dst.analyze_dst(ens, data, R, seed=6, return_parts=True)
    assert np.all(parts["K"] == 0.0)
    assert np.max(np.abs(out - ens)) < 1e-12


def test_learned_covariance_falls_back_on_a_collapsed_ensemble():
    """mu = 0: the features do not exist, lambda_hat is the plain c_hat (0), so
    the gain is 0 and the analysis returns the forecast."""
    rng = np.random.default_rng(12)
    ny, nx, N = 16, 16, 5
    w = {"W1": rng.standard_normal((26, 64)), "b1": rng.standard_normal(64), "W2": rng.standard_normal((64, 64)),
         "b2": rng.standard_normal(64), "W3": rng.standard_normal((64, 64)), "b3": rng.standard_normal(64),
         "w4": rng.standard_normal(64), "b4": rng.standard_normal(1)}
    base = rng.standard_normal((ny, nx)).astype(np.float32)
    ens = np.stack([base] * N)
    data = rng.standard_normal((ny, nx)).astype(np.float32)
    out, parts = learned.analyze_learned(ens, data, 0.05, 3, w, return_parts=True)
    assert parts["mu"] == 0.0
    assert np.all(parts["lam"] == 0.0) and np.all(parts["K"] == 0.0)
    assert np.max(np.abs(out - ens)) < 1e-12
    lam, mu = learned.learned_spectrum(np.full((4, 5), 1e-39), 8, w)
    assert np.all(lam == 1e-39)
