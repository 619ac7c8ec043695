"""The paper's qualitative claim (Sections 4 and 5), as a test of the oracle.

With a very small ensemble (5 members) the FFT EnKF moves the ensemble towards
the data and truth, while the standard EnKF (dense sample covariance, eq. (1))
cannot: on stationary twins the FFT EnKF analysis-mean RMSE is below both the
forecast RMSE and the standard EnKF's.
"""

import numpy as np
import pytest

from oracle import enkf
from paper_1001_1588_amd import twin


@pytest.mark.slow
def test_fft_enkf_beats_standard_enkf_at_five_members():
    fft_rmse, std_rmse, fc_rmse = [], [], []
    for seed in range(3):
        tw = twin.make_twin(32, 32, 5, seed=seed, dtype=np.float64, kind="matern2", kw={"L": 3.0}, r=0.01)
        N, ny, nx = tw.ens.shape
        e_hat = enkf.spectral_perturbations(tw.seed, N, tw.R_spec, nx)
        out_fft = enkf.analyze_spectral(tw.ens, tw.data, tw.R_spec, e_hat)
        e_phys = enkf.physical_perturbations(e_hat, nx)
        out_std = enkf.analyze_dense(tw.ens, tw.data, tw.r, e_phys, enkf.sample_covariance(tw.ens))
        fft_rmse.append(enkf.mean_rmse(out_fft, tw.truth))
        std_rmse.append(enkf.mean_rmse(out_std, tw.truth))
        fc_rmse.append(enkf.mean_rmse(tw.ens, tw.truth))
    assert np.mean(fft_rmse) < np.mean(std_rmse)
    assert np.mean(fft_rmse) < 0.5 * np.mean(fc_rmse)
