"""CPU oracle for the FFT EnKF analysis step -- TEST INFRASTRUCTURE ONLY.

A plain, slow, float64 implementation of what the HIP path computes, written
from Mandel, Beezley and Kondratenko, "Fast Fourier Transform Ensemble Kalman
Filter with application to a coupled atmosphere-wildland fire model":

* dft.py    -- the DFT written out as matrices with exact twiddles (step 1 of
               Section 2.1), unitary scale;
* philox.py -- Philox4x32-10 and Box-Muller from their published definitions,
               for the perturbations e_k ~ N(0, R) of eq. (1);
* enkf.py   -- O1, the spectral form (eq. (2) and eq. (3)), and O2, the dense
               form (eq. (1) with the circulant lag-averaged sample covariance);
* learned.py -- the learned spectral covariance: a per-wavenumber perceptron
               whose estimate replaces the c_hat of eq. (2) in eq. (3);
* multiblock.py -- the multi-block state of Section 2.2, block 1 observed;
* morph.py  -- the extended state of the morphing EnKF (Section 2.2, eq. (9)):
               several observed fields with the cross-covariances among
               them neglected;
* dst.py    -- the analysis in the real sine basis (Section 4).

Only the tests, the smoke check and the benchmark's CPU baseline may import
this package.  It shares no code with the HIP path and imports nothing from it.
Every function is pinned by tests against closed forms, invariants, brute force
or published known-answer values; nothing here is parity-unpinned except the
choice of perturbation convention itself (spectral_noise), whose statistics and
generator are pinned but whose exact draw is a convention.
"""

from . import dft, enkf, philox  # noqa: F401
from .enkf import (analyze, analyze_dense, analyze_dense_circulant, analyze_spectral,  # noqa: F401
                   lag_covariance, sample_covariance, spectral_gain, spectral_mean_variance,
                   spectral_noise, spectral_perturbations)
