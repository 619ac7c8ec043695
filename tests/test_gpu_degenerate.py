"""The gain guard of eq. (3) on the GPU: degenerate ensembles (needs an MI355X).

Reading of the paper: where c_hat + R is below the smallest normal number of
the working precision there is neither spread nor data error, and the gain is
0.  The spread of identical members is exactly zero on both sides (eq. (2) is
summed over deviations from member 0), so these cases reach the guarded
division itself, with R = 0 on bins that include the self-conjugate bins, the
kx = 0 and kx = nx/2 columns (the packed column of the spectral sweep):

* identical members, R zero on a subset of bins: every gain is 0 and the
  analysis returns the forecast (single block, multi-block, sine basis; the
  learned covariance with R > 0, whose mean spectrum mu is then 0);
* members that are constant fields c_k, R = 0: the spread sits at the mean
  wavenumber only (the transforms of a constant are exact), its gain is 1 and
  every other gain 0, so every member becomes the constant mean of the data;
  blocks of the multi-block state move by cov(b, c) / var(c) times block 0's
  innovation.  The oracle's matrix DFT leaves noise of about 1e-16 in bins
  that are zero in exact arithmetic; it is run with its threshold above that
  noise (1e-20) and matches the closed form.

Each case compares element by element with the oracle (relative L2 <= 1e-5
for float32, <= 1e-10 for float64) and with the closed form.
"""

import numpy as np
import pytest
import torch

from oracle import dst, enkf, learned, multiblock
from paper_1001_1588_amd import _lib

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = {np.float32: 1e-5, np.float64: 1e-10}


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def masked_R(ny, nx, rng, dtype):
    """R_spec zero on every self-conjugate bin, the kx = 0 and kx = nx/2
    columns and a random 30% of the rest; positive elsewhere."""
    nh = nx // 2 + 1
    R = rng.uniform(0.01, 0.1, (ny, nh))
    R[:, 0] = 0.0
    R[:, nh - 1] = 0.0
    R[rng.random((ny, nh)) < 0.3] = 0.0
    return R.astype(dtype)


# (ny, nx, N, dtype): several tiles of every sweep and packed kx = 0 rows, both precisions
SHAPES = [(16, 16, 3, np.float32), (64, 128, 5, np.float32), (256, 64, 20, np.float32),
          (2048, 64, 7, np.float32), (32, 32, 4, np.float64), (128, 64, 8, np.float64)]


def sid(c):
    return f"{c[0]}x{c[1]}-N{c[2]}-{np.dtype(c[3]).name}"


@pytest.mark.parametrize("case", SHAPES, ids=sid)
def test_collapsed_ensemble_zero_R_returns_forecast(case):
    ny, nx, N, dt = case
    rng = np.random.default_rng(ny + nx + N)
    base = rng.standard_normal((ny, nx)).astype(dt)
    ens = np.ascontiguousarray(np.broadcast_to(base, (N, ny, nx)))
    data = rng.standard_normal((ny, nx)).astype(dt)
    R = masked_R(ny, nx, rng, dt)
    c_hat, gain, _ = _lib.debug_spectra(dev(ens), dev(data), dev(R), with_spectra=False)
    out = _lib.analyze(dev(ens), dev(data), dev(R), 77)
    torch.cuda.synchronize()
    assert bool((c_hat == 0).all()) and bool((gain == 0).all())
    got = out.cpu().numpy()
    assert np.isfinite(got).all()
    ref = enkf.analyze(ens, data, R, 77)
    assert rel_l2(got, ref) < TOL[dt]
    assert rel_l2(got, ens) < TOL[dt]


@pytest.mark.parametrize("case", SHAPES, ids=sid)
def test_constant_members_zero_R_take_the_data_mean(case):
    ny, nx, N, dt = case
    rng = np.random.default_rng(3 * ny + nx + N)
    c = rng.integers(-4, 5, N) * 0.25                      # dyadic: every transform of them is exact
    if np.all(c == c[0]):
        c[0] += 1.0
    ens = np.ascontiguousarray((c[:, None, None] * np.ones((1, ny, nx))).astype(dt))
    # data with a mean of order one, like the members: the analysis mean is then
    # not small against the forecast, whose float32 rounding it inherits
    data = (1.0 + 0.3 * rng.standard_normal((ny, nx))).astype(dt)
    _, gain, _ = _lib.debug_spectra(dev(ens), dev(data), 0.0, with_spectra=False)
    out = _lib.analyze(dev(ens), dev(data), 0.0, 5)
    torch.cuda.synchronize()
    g = gain.cpu().numpy()
    assert g[0, 0] == 1.0
    g[0, 0] = 0.0
    assert np.all(g == 0.0)
    got = out.cpu().numpy()
    expect = np.full(ens.shape, data.astype(np.float64).mean())
    assert rel_l2(got, expect) < TOL[dt]
    ref = enkf.analyze(ens, data, 0.0, 5, tiny=1e-20)
    assert rel_l2(got, ref) < TOL[dt]


MULTI = [(16, 32, 3, 3, np.float32), (256, 128, 10, 4, np.float32), (64, 64, 4, 2, np.float64)]


@pytest.mark.parametrize("case", MULTI, ids=lambda c: f"{c[0]}x{c[1]}-N{c[2]}-M{c[3]}-{np.dtype(c[4]).name}")
def test_multiblock_collapsed_and_constant_blocks(case):
    ny, nx, N, M, dt = case
    rng = np.random.default_rng(ny * M + N)
    # collapsed state, R zero on a subset of bins: no block moves
    base = rng.standard_normal((M, ny, nx)).astype(dt)
    ens = np.ascontiguousarray(np.broadcast_to(base, (N, M, ny, nx)))
    data = rng.standard_normal((ny, nx)).astype(dt)
    R = masked_R(ny, nx, rng, dt)
    out = _lib.analyze_multi(dev(ens), dev(data), dev(R), 9)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.isfinite(got).all()
    assert rel_l2(got, multiblock.analyze_multi(ens, data, R, 9)) < TOL[dt]
    assert rel_l2(got, ens) < TOL[dt]
    # constant blocks, R = 0: the closed form at the mean wavenumber
    consts = (rng.integers(-4, 5, (M, N)) * 0.25).astype(np.float64)
    consts[0, 0] = consts[0, 1] + 1.0                      # block 0 has spread
    data = (1.0 + 0.3 * rng.standard_normal((ny, nx))).astype(dt)
    ens = np.ascontiguousarray(
        np.stack([np.stack([consts[j, k] * np.ones((ny, nx)) for j in range(M)]) for k in range(N)]).astype(dt))
    out = _lib.analyze_multi(dev(ens), dev(data), 0.0, 9)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    c0, dm = consts[0], data.astype(np.float64).mean()
    expect = np.empty(ens.shape)
    for j in range(M):
        gj = np.cov(consts[j], c0)[0, 1] / np.var(c0, ddof=1)
        expect[:, j] = (consts[j] + gj * (dm - c0))[:, None, None]
    assert rel_l2(got, expect) < TOL[dt]
    assert rel_l2(got, multiblock.analyze_multi(ens, data, 0.0, 9, tiny=1e-20)) < TOL[dt]


@pytest.mark.parametrize("case", [(16, 32, 5, np.float32), (128, 256, 12, np.float32), (64, 32, 3, np.float64)],
                         ids=sid)
def test_sine_basis_collapsed_zero_R_returns_forecast(case):
    ny, nx, N, dt = case
    rng = np.random.default_rng(abs(ny - nx) + N)
    base = rng.standard_normal((ny, nx)).astype(dt)
    ens = np.ascontiguousarray(np.broadcast_to(base, (N, ny, nx)))
    data = rng.standard_normal((ny, nx)).astype(dt)
    R = rng.uniform(0.01, 0.1, (ny, nx))
    R[rng.random((ny, nx)) < 0.4] = 0.0
    R[0, :] = 0.0
    R[:, nx - 1] = 0.0
    R = R.astype(dt)
    out = _lib.analyze_dst(dev(ens), dev(data), dev(R), 21)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.isfinite(got).all()
    assert rel_l2(got, dst.analyze_dst(ens, data, R, 21)) < TOL[dt]
    assert rel_l2(got, ens) < TOL[dt]


def test_learned_covariance_collapsed_ensemble_falls_back():
    """N = 5, R > 0, identical members: mu = 0, so the perceptron's features do
    not exist; the estimate falls back to the plain c_hat = 0 and nothing moves."""
    from paper_1001_1588_amd import evaluate

    w = evaluate.load_weights()
    wd = _lib.mlp_weights(w, DEV)
    ny, nx, N = 64, 128, 5
    rng = np.random.default_rng(5)
    base = rng.standard_normal((ny, nx)).astype(np.float32)
    ens = np.ascontiguousarray(np.broadcast_to(base, (N, ny, nx)))
    data = rng.standard_normal((ny, nx)).astype(np.float32)
    c_hat, lam, mu = _lib.debug_learned_spectrum(dev(ens), dev(data), wd)
    out = _lib.analyze_learned(dev(ens), dev(data), 0.05, 8, wd)
    torch.cuda.synchronize()
    assert float(mu.item()) == 0.0
    assert bool((lam == 0).all()) and bool((c_hat == 0).all())
    got = out.cpu().numpy()
    assert np.isfinite(got).all()
    ref = learned.analyze_learned(ens, data, 0.05, 8, {k: w[k] for k in _lib.MLP_SHAPES})
    assert rel_l2(got, ref) < 1e-5
    assert rel_l2(got, ens) < 1e-5
