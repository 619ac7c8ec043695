"""Pins of the perturbation generator e_k ~ N(0, R) (Section 2, after eq. (1)).

Philox4x32-10 against the published known-answer values; Box-Muller against its
closed form; the spectral noise against what it must be -- the DFT of real white
noise: Hermitian (its inverse is real), unit variance per point, white, and
independent across members and seeds.
"""

import os

import numpy as np
import pytest
from scipy import stats

from oracle import dft, enkf
from oracle.philox import box_muller, philox4x32, uniform_open

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        v = [int(t, 16) for t in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(ctr, key, expect):
    out = philox4x32([np.uint64(c) for c in ctr], key)
    assert [int(o) for o in out] == expect


def test_philox_vectorised_matches_scalar():
    ctr0 = np.arange(50, dtype=np.uint64)
    out = philox4x32((ctr0, np.uint64(7), np.uint64(0), np.uint64(0)), (123, 456))
    for i in (0, 17, 49):
        s = philox4x32((np.uint64(i), np.uint64(7), np.uint64(0), np.uint64(0)), (123, 456))
        assert [int(o[i]) for o in out] == [int(x) for x in s]


def test_uniform_exact_in_binary32_and_open_interval():
    bits = np.array([0, 1, 511, 512, 2**31, 2**32 - 1], dtype=np.uint32)
    u = uniform_open(bits)
    assert np.all(u > 0) and np.all(u < 1)
    assert np.array_equal(u.astype(np.float32).astype(np.float64), u)
    assert u[0] == 2.0 ** -24 and u[-1] == 1 - 2.0 ** -24


def test_box_muller_closed_form():
    a, b = box_muller(np.array([2**31], dtype=np.uint32), np.array([0], dtype=np.uint32))
    u1 = uniform_open(np.array([2**31], dtype=np.uint32))[0]
    u2 = 2.0 ** -24
    rho = np.sqrt(-2 * np.log(u1))
    assert np.isclose(a[0], rho * np.cos(2 * np.pi * u2)) and np.isclose(b[0], rho * np.sin(2 * np.pi * u2))


def test_box_muller_is_standard_normal():
    w = philox4x32((np.arange(20000, dtype=np.uint64), np.uint64(0), np.uint64(0), np.uint64(0)), (1, 2))
    a, b = box_muller(w[0], w[1])
    for s in (a, b):
        assert stats.kstest(s, "norm").pvalue > 1e-3
    assert abs(np.corrcoef(a, b)[0, 1]) < 0.03


@pytest.mark.parametrize("ny,nx", [(16, 16), (8, 32), (32, 8)])
def test_spectral_noise_is_dft_of_real_white_noise(ny, nx):
    N = 6
    z = enkf.spectral_noise(12345, N, ny, nx)
    _, _, mirrored, selfconj = enkf.special_masks(ny, nx)
    assert np.all(z[:, selfconj].imag == 0)
    for kx in {0, nx // 2}:
        for ky in range(ny // 2 + 1, ny):
            assert np.array_equal(z[:, ky, kx], np.conj(z[:, ny - ky, kx]))
    phys, imag = dft.irdft2(z, nx, return_imag=True)
    assert imag < 1e-12
    assert np.allclose(dft.rdft2(phys), z, atol=1e-12)


def test_spectral_noise_statistics():
    ny = nx = 64
    N = 8
    z = enkf.spectral_noise(99, N, ny, nx)
    e = dft.irdft2(z, nx, method="fft")
    assert abs(e.var() - 1) < 0.02                 # unit variance per point
    lag1 = np.mean(e * np.roll(e, 1, axis=2))
    assert abs(lag1) < 0.02                        # white
    c = np.corrcoef(e.reshape(N, -1))
    assert np.max(np.abs(c - np.eye(N))) < 0.05    # independent members
    assert stats.kstest(e.ravel(), "norm").pvalue > 1e-3


def test_self_conjugate_bins_are_independent_unit_normals():
    """The four real bins of the spectrum: each N(0, 1) across members and the
    four mutually uncorrelated (the two of a row share one Box-Muller pair, whose
    halves are independent); a mistake that reused one half for both bins of a
    row would give correlation 1."""
    ny, nx, N = 8, 8, 4000
    z = enkf.spectral_noise(2024, N, ny, nx)
    vals = np.stack([z[:, ky, kx].real for ky in (0, ny // 2) for kx in (0, nx // 2)])
    assert np.all(np.abs(vals.var(axis=1) - 1) < 0.08)
    c = np.corrcoef(vals)
    assert np.max(np.abs(c - np.eye(4))) < 0.08
    for v in vals:
        assert stats.kstest(v, "norm").pvalue > 1e-3


def test_perturbation_scaled_by_R_and_seed_dependent():
    ny = nx = 32
    R = np.full((ny, nx // 2 + 1), 0.05)
    e1 = enkf.physical_perturbations(enkf.spectral_perturbations(1, 4, R, nx), nx)
    assert abs(e1.var() - 0.05) < 0.005
    z1 = enkf.spectral_noise(1, 4, ny, nx)
    z2 = enkf.spectral_noise(2, 4, ny, nx)
    z3 = enkf.spectral_noise(1 + (1 << 32), 4, ny, nx)   # high key word matters too
    assert not np.allclose(z1, z2) and not np.allclose(z1, z3)
    assert np.array_equal(z1, enkf.spectral_noise(1, 4, ny, nx))
    # member k does not depend on N
    assert np.array_equal(z1[:3], enkf.spectral_noise(1, 3, ny, nx))
