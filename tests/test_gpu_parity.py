"""HIP path against the float64 oracle, through the C ABI (needs an MI355X).

Bar: relative L2 over all members and grid points <= 1e-5 for float32 inputs,
<= 1e-10 for float64; the oracle consumes the same (upcast) inputs.  Every case
spans several tiles of each sweep and includes the kx = 0 / nx/2 columns and
self-conjugate bins.
"""

import numpy as np
import pytest
import torch

from oracle import dft, enkf
from paper_1001_1588_amd import _lib, twin

pytestmark = pytest.mark.gpu

TOL = {np.float32: 1e-5, np.float64: 1e-10}
DEV = "cuda:0"


def rel_l2(a, b):
    a = np.asarray(a)
    a = a.astype(np.complex128) if np.iscomplexobj(a) else a.astype(np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def gpu_analyze(tw, R_as="array", seed=None, out=None):
    ens, data = to_dev(tw.ens), to_dev(tw.data)
    R = to_dev(tw.R_spec) if R_as == "array" else float(tw.r)
    res = _lib.analyze(ens, data, R, tw.seed if seed is None else seed, out=out)
    torch.cuda.synchronize()
    return res.cpu().numpy()


def case_id(c):
    ny, nx, N, dt = c[:4]
    return f"{ny}x{nx}-N{N}-{np.dtype(dt).name}"


# (ny, nx, N, dtype, R kind)
CASES = [
    (8, 8, 2, np.float32, "scalar"),
    (8, 8, 3, np.float64, "spectral"),
    (16, 16, 5, np.float32, "spectral"),
    (16, 32, 7, np.float64, "scalar"),
    (32, 16, 4, np.float32, "scalar"),
    (64, 64, 5, np.float64, "scalar"),
    (64, 64, 5, np.float32, "spectral"),
    (128, 64, 20, np.float32, "scalar"),
    (64, 128, 11, np.float32, "spectral"),
    (256, 256, 20, np.float32, "spectral"),
    (256, 128, 24, np.float32, "scalar"),
    (128, 256, 8, np.float64, "spectral"),
    (512, 64, 13, np.float32, "scalar"),
    (32, 1024, 3, np.float32, "scalar"),
    (1024, 32, 17, np.float32, "spectral"),
    (8, 2048, 2, np.float32, "scalar"),
    (2048, 8, 6, np.float64, "scalar"),
    # the extreme aspect ratios and sizes: 4096-wide rows (8-row tiles), 4096
    # tall columns, the largest float32 bucket on a tall grid
    (8, 4096, 3, np.float32, "spectral"),
    (4096, 8, 4, np.float64, "scalar"),
    (4096, 16, 24, np.float32, "spectral"),
    (16, 4096, 8, np.float64, "spectral"),
    # length-128 and length-64 columns in float32 (1024 and 512 tall, 8-row
    # tiles): the wave-level transforms in several member buckets, and grids too
    # narrow for their 8- and 16-column units (the Stockham form then)
    (1024, 64, 4, np.float32, "scalar"),
    (1024, 16, 9, np.float32, "spectral"),
    (1024, 8, 5, np.float32, "scalar"),
    (512, 32, 8, np.float32, "spectral"),
    (512, 16, 6, np.float32, "scalar"),
    (1024, 32, 23, np.float32, "scalar"),
    (1024, 16, 7, np.float32, "spectral"),
]


@pytest.mark.parametrize("case", CASES, ids=case_id)
def test_forward_spectra_and_statistics(case):
    """Sweep 1 plus the forward half of sweep 2: unitary spectra, eq. (2), gain."""
    ny, nx, N, dt, rk = case
    tw = twin.random_ensemble(ny, nx, N, seed=ny + 7 * nx + N, dtype=dt, R_kind=rk)
    ens, data = to_dev(tw.ens), to_dev(tw.data)
    c_hat, gain, spec = _lib.debug_spectra(ens, data, to_dev(tw.R_spec))
    torch.cuda.synchronize()
    _, parts = enkf.analyze(tw.ens, tw.data, tw.R_spec, tw.seed, method="fft", return_parts=True)
    spec = spec.cpu().numpy()
    spec = spec[..., 0] + 1j * spec[..., 1]
    ref = np.concatenate([parts["u_hat"], parts["d_hat"][None]])
    tol = TOL[dt]
    assert rel_l2(spec, ref) < tol
    assert rel_l2(c_hat.cpu().numpy(), parts["c_hat"]) < 10 * tol
    assert rel_l2(gain.cpu().numpy(), parts["K"]) < 10 * tol


@pytest.mark.parametrize("case", CASES[:8], ids=case_id)
def test_perturbations_match_convention(case):
    ny, nx, N, dt, rk = case
    tw = twin.random_ensemble(ny, nx, N, seed=3, dtype=dt, R_kind=rk)
    e = _lib.debug_perturb(to_dev(tw.ens), to_dev(tw.data), to_dev(tw.R_spec), tw.seed)
    torch.cuda.synchronize()
    e = e.cpu().numpy()
    e = e[..., 0] + 1j * e[..., 1]
    ref = enkf.spectral_perturbations(tw.seed, N, tw.R_spec, nx)
    assert rel_l2(e, ref) < (2e-6 if dt == np.float32 else 1e-13)


@pytest.mark.parametrize("case", CASES, ids=case_id)
def test_analysis_matches_oracle(case):
    ny, nx, N, dt, rk = case
    tw = twin.random_ensemble(ny, nx, N, seed=ny * 31 + nx + N, dtype=dt, R_kind=rk)
    got = gpu_analyze(tw, R_as="array" if rk == "spectral" else "scalar")
    ref = enkf.analyze(tw.ens, tw.data, tw.R_spec, tw.seed, method="matmul" if ny * nx <= 65536 else "fft")
    assert rel_l2(got, ref) < TOL[dt]


def test_config_small64_float64():
    """The 64x64, N=5, float64 workload (R = 0.01 I)."""
    tw = twin.workload("small64", seed=11)
    got = gpu_analyze(tw, R_as="scalar")
    ref = enkf.analyze(tw.ens, tw.data, tw.R_spec, tw.seed)
    assert rel_l2(got, ref) < 1e-10
    # and it improves on the forecast, as the oracle does
    assert enkf.mean_rmse(got, tw.truth) < enkf.mean_rmse(tw.ens, tw.truth)


def test_config_large2048_float32():
    """The 2048x2048, N=20, float32 workload, checked in full against the oracle
    in its plain form (the DFT written out as matrices, about ten seconds)."""
    tw = twin.workload("large2048", seed=5)
    got = gpu_analyze(tw, R_as="array")
    ref = enkf.analyze(tw.ens, tw.data, tw.R_spec, tw.seed, method="matmul")
    assert rel_l2(got, ref) < 1e-5


def test_max_grid_roundtrip_and_sampled_spectrum():
    """4096x4096 (largest grid): with R huge the gain vanishes and the analysis
    returns the forecast; c_hat at sampled bins equals the direct DFT sum."""
    ny = nx = 4096
    N = 3
    rng = np.random.default_rng(0)
    ens = rng.standard_normal((N, ny, nx)).astype(np.float32)
    data = rng.standard_normal((ny, nx)).astype(np.float32)
    e, d = to_dev(ens), to_dev(data)
    out = _lib.analyze(e, d, 1e30, 123)
    torch.cuda.synchronize()
    assert rel_l2(out.cpu().numpy(), ens.astype(np.float64)) < 1e-5
    c_hat, gain, _ = _lib.debug_spectra(e, d, 0.5, with_spectra=False)
    c_hat = c_hat.cpu().numpy()
    y = np.arange(ny)[:, None]
    x = np.arange(nx)[None, :]
    for (ky, kx) in [(0, 0), (1, 0), (4095, 0), (2048, 2048), (17, 2048), (3000, 5), (123, 1024)]:
        ph = np.exp(-2j * np.pi * (((ky * y) % ny) / ny + ((kx * x) % nx) / nx))
        uh = np.array([np.sum(ens[k].astype(np.float64) * ph) for k in range(N)]) / np.sqrt(ny * nx)
        ref = np.sum(np.abs(uh - uh.mean()) ** 2) / (N - 1)
        assert abs(c_hat[ky, kx] - ref) <= 1e-4 * ref + 1e-6


def test_max_members():
    tw = twin.random_ensemble(64, 32, 24, seed=1, dtype=np.float32)
    assert rel_l2(gpu_analyze(tw, R_as="scalar"), enkf.analyze(tw.ens, tw.data, tw.R_spec, tw.seed)) < 1e-5
    tw = twin.random_ensemble(32, 64, 8, seed=2, dtype=np.float64)
    assert rel_l2(gpu_analyze(tw, R_as="scalar"), enkf.analyze(tw.ens, tw.data, tw.R_spec, tw.seed)) < 1e-10


def test_determinism_seed_and_in_place():
    tw = twin.random_ensemble(256, 128, 9, seed=4, dtype=np.float32)
    a = gpu_analyze(tw)
    b = gpu_analyze(tw)
    assert np.array_equal(a, b)
    c = gpu_analyze(tw, seed=tw.seed + 1)
    assert not np.array_equal(a, c)
    ens = to_dev(tw.ens)
    res = _lib.analyze(ens, to_dev(tw.data), to_dev(tw.R_spec), tw.seed, out=ens)
    torch.cuda.synchronize()
    assert res.data_ptr() == ens.data_ptr()
    assert np.array_equal(ens.cpu().numpy(), a)


def test_scalar_and_array_R_agree():
    tw = twin.random_ensemble(64, 64, 6, seed=8, dtype=np.float32)
    assert np.array_equal(gpu_analyze(tw, R_as="scalar"), gpu_analyze(tw, R_as="array"))


def test_single_mode_scalar_kalman_on_gpu():
    """Closed form: an ensemble differing in one cosine mode is updated in that
    mode only, by the scalar Kalman gain (perturbations off: R = 0 there is
    excluded, so use the mode case with R tiny against a large spread)."""
    ny, nx, N = 32, 64, 4
    y = np.arange(ny)[:, None]
    x = np.arange(nx)[None, :]
    mode = np.cos(2 * np.pi * (3 * y / ny + 5 * x / nx))
    a = np.array([1.0, -0.5, 0.25, 2.0])
    ens = (0.2 + a[:, None, None] * mode[None]).astype(np.float64)
    data = (0.2 + 0.7 * mode).astype(np.float64)
    r = 0.3
    tw = twin.Twin(ens=ens, data=data, R_spec=np.full((ny, nx // 2 + 1), r), r=r, seed=9, truth=data, lam=None)
    got = gpu_analyze(tw, R_as="scalar")
    ref = enkf.analyze(ens, data, r, 9)
    assert rel_l2(got, ref) < 1e-10


def test_rejects_host_memory_without_writing():
    tw = twin.random_ensemble(16, 16, 3, seed=1, dtype=np.float32)
    ens = to_dev(tw.ens)
    host_data = torch.from_numpy(tw.data)
    out = torch.full_like(ens, 7.0)
    with pytest.raises(RuntimeError):
        _lib.analyze(ens, host_data, 0.05, 1, out=out)
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())


def test_forced_failure_path_writes_nothing():
    tw = twin.random_ensemble(16, 16, 3, seed=1, dtype=np.float32)
    ens = to_dev(tw.ens)
    out = torch.full_like(ens, 7.0)
    _lib.debug_fail_next(_lib.EDEVICE)
    with pytest.raises(RuntimeError, match="forced"):
        _lib.analyze(ens, to_dev(tw.data), 0.05, 1, out=out)
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
    # the next call works normally
    _lib.analyze(ens, to_dev(tw.data), 0.05, 1, out=out)
    torch.cuda.synchronize()
    assert not bool((out == 7.0).all())
