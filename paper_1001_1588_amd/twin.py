"""Seeded synthetic twin experiments: the inputs of one FFT EnKF analysis.

This module only draws inputs. It holds none of the analysis arithmetic and is
shared by the tests, the benchmark and the smoke check; the CPU oracle and the
HIP path both receive what it returns.

Random fields follow the paper's generator of random smooth functions (Section
2.2): a Fourier series with random coefficients whose size decays with the
wavenumber.  Concretely, a stationary Gaussian field with spectrum lambda(k)
(the eigenvalues of its circulant covariance) is white noise filtered by
sqrt(lambda) in the unitary Fourier basis.

Workloads (the paper measures on no public dataset; these stand in for its
WRF-Fire ideal problem, Section 4):

* ``small64``  -- periodic 64x64, float64, N=5, lambda = (1+|k|^2)^-2,
  d = truth + N(0, 0.01 I), R = 0.01 I.
* ``large2048`` -- periodic 2048x2048, float32, N=20, lambda = |k|^-3 (k != 0),
  lambda(0) = 0, d = truth + N(0, 0.05 I), R = 0.05 I.
* batch (``batch_sides`` + ``device_twin``) -- 256 independent filters, square
  sides drawn uniformly from {64, 128, 256, 512, 1024}, float32, N=16, lambda =
  (1+|k|^2)^-2, R = 0.01 I; drawn on the device with torch (same law as
  ``make_twin``) because numpy would take minutes at that size.
* multi-block (``make_multiblock_twin``) -- 4 fields of 1024x1024, float32,
  N=10, lambda_b = (1 + |k|^2 / L_b^2)^-2 with L_b in {8, 16, 32, 64}, spectral
  coherence 0.6 between blocks through a shared latent field, d observes block
  0 with R = 0.02 I (Section 2.2).

In both, members = truth + independent draws from the same field law.

``about="centre"`` builds the twin the way the paper's experiment does
(Section 4: ensemble and data both made by random perturbation of one state):
a centre field u, members u + r_k and truth u + r_0 with r_0, r_k independent
draws of the same law, so the truth is exchangeable with the members and the
forecast mean's error has spectrum lambda (1 + 1/N).  With the default
``about="truth"`` the forecast mean sits on the truth, its error spectrum is
lambda / N, and the spread overstates it N-fold.
"""

from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np


def integer_wavenumbers(n: int) -> np.ndarray:
    """|k| along one periodic axis of length n: min(j, n - j)."""
    j = np.arange(n)
    return np.minimum(j, n - j).astype(np.float64)


def spectrum(ny: int, nx: int, kind: str, **kw) -> np.ndarray:
    """Full-grid spectrum lambda[ky, kx] normalised to mean 1 (unit pointwise variance).

    kind = "matern2": (1 + |k|^2 / L^2)^-2 (L = kw.get("L", 1)).
    kind = "power":   |k|^-a for k != 0 and 0 at k = 0 (a = kw.get("a", 3)).
    """
    ky = integer_wavenumbers(ny)[:, None]
    kx = integer_wavenumbers(nx)[None, :]
    k2 = ky * ky + kx * kx
    if kind == "matern2":
        L = float(kw.get("L", 1.0))
        lam = (1.0 + k2 / (L * L)) ** -2
    elif kind == "power":
        a = float(kw.get("a", 3.0))
        with np.errstate(divide="ignore"):
            lam = np.where(k2 > 0, k2 ** (-a / 2.0), 0.0)
    else:
        raise ValueError(f"unknown spectrum kind {kind!r}")
    return lam / lam.mean()


def gaussian_fields(rng: np.random.Generator, lam: np.ndarray, count: int) -> np.ndarray:
    """`count` independent stationary Gaussian fields with spectrum `lam` (float64)."""
    ny, nx = lam.shape
    amp = np.sqrt(lam[:, : nx // 2 + 1])
    out = np.empty((count, ny, nx), dtype=np.float64)
    for c in range(count):
        w = rng.standard_normal((ny, nx))
        out[c] = np.fft.irfft2(np.fft.rfft2(w, norm="ortho") * amp, s=(ny, nx), norm="ortho")
    return out


@dataclasses.dataclass
class Twin:
    """One analysis problem: forecast ensemble, data, R eigenvalues, seed, and the truth."""

    ens: np.ndarray        # [N, ny, nx]
    data: np.ndarray       # [ny, nx]
    R_spec: np.ndarray     # [ny, nx//2 + 1], eigenvalues of the stationary R
    r: float               # R = r I
    seed: int              # seed of the analysis perturbations
    truth: np.ndarray      # [ny, nx]
    lam: np.ndarray        # generating spectrum [ny, nx]
    name: str = ""


WORKLOADS = {
    "small64": dict(ny=64, nx=64, N=5, dtype=np.float64, kind="matern2", kw={}, r=0.01),
    "large2048": dict(ny=2048, nx=2048, N=20, dtype=np.float32, kind="power", kw={"a": 3.0}, r=0.05),
}


def make_twin(ny: int, nx: int, N: int, *, seed: int, dtype=np.float32, kind: str = "matern2",
              kw: Optional[dict] = None, r: float = 0.01, name: str = "", about: str = "truth") -> Twin:
    """Twin experiment from one master seed (numpy SeedSequence spawned four ways:
    truth, member draws, data noise, analysis seed; a fifth, the truth's own
    draw, when about="centre")."""
    kw = kw or {}
    ss = np.random.SeedSequence(seed)
    s_truth, s_mem, s_obs, s_an = ss.spawn(4)
    lam = spectrum(ny, nx, kind, **kw)
    centre = gaussian_fields(np.random.default_rng(s_truth), lam, 1)[0]
    ens = centre[None] + gaussian_fields(np.random.default_rng(s_mem), lam, N)
    if about == "truth":
        truth = centre
    elif about == "centre":
        truth = centre + gaussian_fields(np.random.default_rng(ss.spawn(1)[0]), lam, 1)[0]
    else:
        raise ValueError(f"about must be 'truth' or 'centre', not {about!r}")
    data = truth + np.sqrt(r) * np.random.default_rng(s_obs).standard_normal((ny, nx))
    an_seed = int(np.random.default_rng(s_an).integers(0, 2**63 - 1, dtype=np.int64))
    R_spec = np.full((ny, nx // 2 + 1), r, dtype=np.float64)
    return Twin(ens=ens.astype(dtype), data=data.astype(dtype), R_spec=R_spec.astype(dtype), r=r,
                seed=an_seed, truth=truth.astype(dtype), lam=lam, name=name)


def workload(name: str, seed: int = 0, **override) -> Twin:
    """One of the named workloads (see module docstring); fields may be overridden."""
    cfg = dict(WORKLOADS[name])
    cfg.update(override)
    return make_twin(cfg["ny"], cfg["nx"], cfg["N"], seed=seed, dtype=cfg["dtype"], kind=cfg["kind"],
                     kw=cfg["kw"], r=cfg["r"], name=name)


def random_ensemble(ny: int, nx: int, N: int, *, seed: int, dtype=np.float32, r: float = 0.05,
                    R_kind: str = "scalar") -> Twin:
    """Generic seeded case for parity tests: smooth members plus data, R either
    constant (R_kind="scalar") or a positive even spectrum (R_kind="spectral")."""
    tw = make_twin(ny, nx, N, seed=seed, dtype=dtype, kind="matern2", kw={"L": max(1.0, min(ny, nx) / 16)}, r=r)
    if R_kind == "spectral":
        ky = integer_wavenumbers(ny)[:, None]
        kx = np.arange(nx // 2 + 1)[None, :].astype(np.float64)
        R = r * (0.5 + 1.5 / (1.0 + (ky * ky + kx * kx) / 16.0))
        tw.R_spec = R.astype(dtype)
    return tw


@dataclasses.dataclass
class MultiTwin:
    """Multi-block analysis problem: M fields per member, block 0 observed."""

    ens: np.ndarray        # [N, M, ny, nx] member-major state vectors
    data: np.ndarray       # [ny, nx], observes block 0
    R_spec: np.ndarray     # [ny, nx//2 + 1]
    r: float
    seed: int
    truth: np.ndarray      # [M, ny, nx]
    lam: np.ndarray        # [M, ny, nx] spectra of the blocks
    rho: float             # spectral coherence between blocks


def coherent_fields(rng: np.random.Generator, lams: np.ndarray, rho: float, count: int) -> np.ndarray:
    """`count` draws of M jointly Gaussian stationary fields [count, M, ny, nx]:
    block b filters sqrt(rho) w_shared + sqrt(1 - rho) w_b by sqrt(lambda_b), so
    every pair of blocks has spectral coherence rho at every wavenumber."""
    M, ny, nx = lams.shape
    amp = np.sqrt(lams[:, :, : nx // 2 + 1])
    out = np.empty((count, M, ny, nx), dtype=np.float64)
    for c in range(count):
        shared = rng.standard_normal((ny, nx))
        for b in range(M):
            w = np.sqrt(rho) * shared + np.sqrt(1.0 - rho) * rng.standard_normal((ny, nx))
            out[c, b] = np.fft.irfft2(np.fft.rfft2(w, norm="ortho") * amp[b], s=(ny, nx), norm="ortho")
    return out


def make_multiblock_twin(ny: int, nx: int, N: int, *, seed: int, Ls=(8.0, 16.0, 32.0, 64.0), rho: float = 0.6,
                         r: float = 0.02, dtype=np.float32, about: str = "truth") -> MultiTwin:
    """Multi-block twin: blocks with spectra (1 + |k|^2 / L_b^2)^-2 (mean 1),
    coherence rho through a shared latent white noise, members = truth + draws
    (about="truth") or truth and members both draws about a centre
    (about="centre"); data = block 0 of the truth + N(0, r I)."""
    ss = np.random.SeedSequence(seed)
    s_truth, s_mem, s_obs, s_an = ss.spawn(4)
    lams = np.stack([spectrum(ny, nx, "matern2", L=L) for L in Ls])
    centre = coherent_fields(np.random.default_rng(s_truth), lams, rho, 1)[0]
    ens = centre[None] + coherent_fields(np.random.default_rng(s_mem), lams, rho, N)
    if about == "truth":
        truth = centre
    elif about == "centre":
        truth = centre + coherent_fields(np.random.default_rng(ss.spawn(1)[0]), lams, rho, 1)[0]
    else:
        raise ValueError(f"about must be 'truth' or 'centre', not {about!r}")
    data = truth[0] + np.sqrt(r) * np.random.default_rng(s_obs).standard_normal((ny, nx))
    an_seed = int(np.random.default_rng(s_an).integers(0, 2**63 - 1, dtype=np.int64))
    R_spec = np.full((ny, nx // 2 + 1), r, dtype=np.float64)
    return MultiTwin(ens=ens.astype(dtype), data=data.astype(dtype), R_spec=R_spec.astype(dtype), r=r,
                     seed=an_seed, truth=truth.astype(dtype), lam=lams, rho=rho)


def batch_sides(n_filters: int, seed: int, choices=(64, 128, 256, 512, 1024)) -> list:
    """Square grid sides of a batch of independent filters, uniform over `choices`."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 4]))
    return [int(c) for c in rng.choice(np.asarray(choices), size=n_filters)]


def device_twin(ny: int, nx: int, N: int, *, seed: int, r: float = 0.01, kind: str = "matern2", kw=None,
                device="cuda:0"):
    """A twin like make_twin (members = truth + draws, d = truth + N(0, r I)),
    float32, drawn on the device with torch's generator; returns (ens, data,
    analysis seed).  The fields are white noise filtered by sqrt(lambda) in the
    unitary Fourier basis, as gaussian_fields does."""
    import torch

    kw = kw or {}
    g = torch.Generator(device=device).manual_seed(seed)
    amp = torch.from_numpy(np.sqrt(spectrum(ny, nx, kind, **kw)[:, : nx // 2 + 1])).to(device, torch.float32)

    def fields(count):
        w = torch.randn((count, ny, nx), generator=g, device=device, dtype=torch.float32)
        return torch.fft.irfft2(torch.fft.rfft2(w, norm="ortho") * amp, s=(ny, nx), norm="ortho")

    truth = fields(1)[0]
    ens = (truth[None] + fields(N)).contiguous()
    data = (truth + np.sqrt(r) * torch.randn((ny, nx), generator=g, device=device, dtype=torch.float32)).contiguous()
    an_seed = int(torch.randint(0, 2**62, (1,), generator=g, device=device).item())
    return ens, data, an_seed
