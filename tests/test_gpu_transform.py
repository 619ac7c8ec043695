"""The 2D transform of the analysis on its own (fftenkf_debug_fft2), through the
C ABI, against the oracle's matrix DFT; and the optional synchronous check of
R_spec (FFTENKF_CHECK=1).

Bars: relative L2 <= 1e-5 in float32 (about 2 log2(n) roundings of unit size per
output, far below it) and <= 1e-10 in float64, as for the whole analysis.  The
inverse takes arbitrary half spectra: the kx = 0 and kx = nx/2 columns need not
be Hermitian, and both sides then return the real part of the inverse of the
Hermitian extension."""

import os

import numpy as np
import pytest
import torch

from oracle import dft, enkf
from paper_1001_1588_amd import _lib, twin

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = {np.float32: 1e-5, np.float64: 1e-10}

CASES = [(8, 8, 2, np.float32), (16, 32, 3, np.float64), (64, 128, 5, np.float32), (256, 64, 4, np.float64),
         (32, 2048, 2, np.float32), (512, 512, 20, np.float32), (2048, 2048, 2, np.float32),
         (4096, 64, 3, np.float32), (64, 4096, 2, np.float64)]


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - b) / np.linalg.norm(b))


def method(ny, nx):
    return "matmul" if ny * nx <= 65536 else "fft"


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}-N{c[2]}-{np.dtype(c[3]).name}")
def test_forward_transform(case):
    ny, nx, N, dt = case
    x = np.random.default_rng(ny * 7 + nx + N).standard_normal((N, ny, nx)).astype(dt)
    spec = _lib.debug_rfft2(torch.from_numpy(x).to(DEV))
    torch.cuda.synchronize()
    s = spec.cpu().numpy().astype(np.float64)
    got = s[..., 0] + 1j * s[..., 1]
    ref = dft.rdft2(x.astype(np.float64), method=method(ny, nx))
    assert rel_l2(got, ref) <= TOL[dt]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}-N{c[2]}-{np.dtype(c[3]).name}")
def test_inverse_transform_of_arbitrary_half_spectra(case):
    ny, nx, N, dt = case
    rng = np.random.default_rng(ny + nx * 3 + N)
    S = rng.standard_normal((N, ny, nx // 2 + 1, 2)).astype(dt)
    out = _lib.debug_irfft2(torch.from_numpy(S).to(DEV), nx)
    torch.cuda.synchronize()
    ref = dft.irdft2(S[..., 0].astype(np.float64) + 1j * S[..., 1].astype(np.float64), nx, method=method(ny, nx))
    assert rel_l2(out.cpu().numpy().astype(np.float64), ref) <= TOL[dt]


def test_round_trip_and_analysis_unchanged():
    tw = twin.random_ensemble(128, 256, 6, seed=12, dtype=np.float32)
    ens = torch.from_numpy(tw.ens).to(DEV)
    back = _lib.debug_irfft2(_lib.debug_rfft2(ens), 256)
    torch.cuda.synchronize()
    assert rel_l2(back.cpu().numpy().astype(np.float64), tw.ens.astype(np.float64)) <= 1e-6
    # the transform exports share the workspace layout with the analysis, not its results
    a = _lib.analyze(ens, torch.from_numpy(tw.data).to(DEV), 0.01, tw.seed)
    torch.cuda.synchronize()
    ref = enkf.analyze(tw.ens, tw.data, 0.01, tw.seed, method="fft")
    assert rel_l2(a.cpu().numpy().astype(np.float64), ref) <= 1e-5


def test_check_mode_rejects_bad_spectra():
    tw = twin.random_ensemble(32, 32, 4, seed=3, dtype=np.float32)
    ens, data = torch.from_numpy(tw.ens).to(DEV), torch.from_numpy(tw.data).to(DEV)
    R = torch.from_numpy(tw.R_spec).to(DEV)
    good = _lib.analyze(ens, data, R, tw.seed)
    bad_neg, bad_nan = R.clone(), R.clone()
    bad_neg[3, 4] = -1e-3
    bad_nan[5, 0] = float("nan")
    os.environ["FFTENKF_CHECK"] = "1"
    try:
        for bad, what in ((bad_neg, "R_spec"), (bad_nan, "R_spec")):
            with pytest.raises(RuntimeError, match=what):
                _lib.analyze(ens, data, bad, tw.seed)
        lam = torch.ones_like(R)
        lam[0, 0] = float("inf")
        with pytest.raises(RuntimeError, match="lam"):
            _lib.analyze_spectrum(ens, data, R, tw.seed, lam)
        checked = _lib.analyze(ens, data, R, tw.seed)
    finally:
        del os.environ["FFTENKF_CHECK"]
    unchecked_bad = _lib.analyze(ens, data, bad_neg, tw.seed)   # not checked: accepted, garbage in
    torch.cuda.synchronize()
    assert torch.equal(good, checked)
    assert unchecked_bad.shape == good.shape
