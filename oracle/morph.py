"""FFT EnKF on the extended state of the morphing EnKF (Section 2.2, eq. (9)).

Test infrastructure only: the library never imports this module.

The morphing transform turns each member into the extended state of eq. (9),
(T, r^(1), .., r^(M)): the two components T_x, T_y of the registration mapping
and the residual fields.  Its observation operator keeps (T, r^(1)), so K = 3
fields are observed, and the paper neglects the cross-covariances among them:
the observed part's covariance C^(11) is three diagonal matrices.  Generalised
here to K observed fields (blocks 0 .. K-1 of an M-block state, member-major
[N][M][ny][nx]), each with its own data d_o and stationary data error R_o.

With C^(11) block diagonal, eq. (5) becomes, per bin of the frequency domain:

* an observed block o moves by its own gain, as in the single-block eq. (3):
    u_hat^(o)a_k = u_hat^(o)_k + c_hat^(oo) / (c_hat^(oo) + R_o) (d_hat_o + e_hat_ko - u_hat^(o)_k);
* an unobserved block j moves by the sum of one such term per observed field:
    u_hat^(j)a_k = u_hat^(j)_k + sum_o c_hat^(jo) / (c_hat^(oo) + R_o) (d_hat_o + e_hat_ko - u_hat^(o)_k),
  c_hat^(jo) the spectral cross-covariance of eq. (7) (conjugate on the
  observed factor, as in multiblock.py).

Two independent float64 forms:

MO1 -- the spectral form above.
MO2 -- dense eq. (1) on the extended state: H selects the K observed blocks,
   C is assembled from circulant lag-averaged (cross-)covariances, by direct
   lag sums with no DFT, with the blocks between different observed fields set
   to zero, R = blockdiag(R_o), and the system is solved densely.

Perturbations: e_hat_ko ~ N(0, R_o) independently per observed field, drawn
with the convention of enkf.spectral_noise, except that the fourth Philox
counter word is o (so field 0 draws exactly the single-block stream).
"""

from __future__ import annotations

import numpy as np

from . import dft
from .enkf import _noise, spectral_gain, tiny_for
from .multiblock import circulant, cross_spectrum, lag_cross_covariance


def observed_noise(seed: int, N: int, K: int, ny: int, nx: int) -> np.ndarray:
    """Unit-variance spectral white noise z_hat[k, o, ky, kx] (half spectrum) for
    member k and observed field o: enkf.spectral_noise's convention with the
    fourth counter word o."""
    nh = nx // 2 + 1
    z = np.empty((N, K, ny, nh), dtype=np.complex128)
    for o in range(K):
        z[:, o] = _noise(seed, N, ny, nx, o)
    return z


def observed_perturbations(seed: int, N: int, R_obs: np.ndarray, nx: int) -> np.ndarray:
    """e_hat[k, o] = sqrt(R_obs[o]) z_hat[k, o], R_obs [K, ny, nx/2+1]."""
    R_obs = np.asarray(R_obs, dtype=np.float64)
    K, ny = R_obs.shape[:2]
    return np.sqrt(R_obs)[None] * observed_noise(seed, N, K, ny, nx)


def _R_obs(R, K, ny, nx):
    """R per observed field as [K, ny, nx/2+1]: an array, or K scalars."""
    R = np.asarray(R, dtype=np.float64)
    if R.ndim == 1:
        R = R[:, None, None]
    return np.broadcast_to(R, (K, ny, nx // 2 + 1))


def analyze_morph_spectral(ens, data, R, e_hat, *, method: str = "matmul", tiny=None, return_parts: bool = False):
    """MO1 with given perturbations e_hat [N, K, ny, nx/2+1] (unitary scale).

    ens [N, M, ny, nx], blocks 0 .. K-1 observed by data [K, ny, nx]; R is
    [K, ny, nx/2+1] eigenvalues or K scalars."""
    ens = np.asarray(ens)
    N, M, ny, nx = ens.shape
    data = np.asarray(data, dtype=np.float64)
    K = data.shape[0]
    if tiny is None:
        tiny = tiny_for(ens.dtype)
    R = _R_obs(R, K, ny, nx)
    u_hat = dft.rdft2(ens.astype(np.float64), method=method)          # [N, M, ny, nh]
    d_hat = dft.rdft2(data, method=method)                             # [K, ny, nh]
    c_oo = np.stack([cross_spectrum(u_hat[:, o], u_hat[:, o]).real for o in range(K)])
    den = c_oo + R                                                     # [K, ny, nh]
    innov = d_hat[None] + e_hat - u_hat[:, :K]                         # [N, K, ny, nh]
    out_hat = np.empty_like(u_hat)
    for j in range(M):
        if j < K:
            G = spectral_gain(c_oo[j], R[j], tiny)                     # eq. (3) for an observed block
            out_hat[:, j] = u_hat[:, j] + G[None] * innov[:, j]
        else:
            upd = np.zeros_like(u_hat[:, j])
            for o in range(K):
                cjo = cross_spectrum(u_hat[:, j], u_hat[:, o])
                G = np.where(den[o] < tiny, 0.0, cjo / np.where(den[o] < tiny, 1.0, den[o]))
                upd = upd + G[None] * innov[:, o]
            out_hat[:, j] = u_hat[:, j] + upd
    ua = dft.irdft2(out_hat, nx, method=method)
    if return_parts:
        return ua, dict(u_hat=u_hat, d_hat=d_hat, c_oo=c_oo, innov=innov)
    return ua


def analyze_morph(ens, data, R, seed: int, *, method: str = "matmul", tiny=None, return_parts: bool = False):
    """MO1 with the seeded perturbation convention (observed_noise)."""
    ens = np.asarray(ens)
    N, M, ny, nx = ens.shape
    K = np.asarray(data).shape[0]
    e_hat = observed_perturbations(seed, N, _R_obs(R, K, ny, nx), nx)
    return analyze_morph_spectral(ens, data, R, e_hat, method=method, tiny=tiny, return_parts=return_parts)


def analyze_morph_dense(ens, data, R_dense, e_phys) -> np.ndarray:
    """MO2: eq. (1) on the extended state, dense.

    R_dense: list of K dense [n, n] matrices (or scalars); e_phys [N, K, ny, nx].
    C has blocks C^(ab) = circulant(lag-averaged cross-covariance of a and b)
    except C^(ab) = 0 for observed a != b (the neglected cross-covariances)."""
    ens = np.asarray(ens, dtype=np.float64)
    N, M, ny, nx = ens.shape
    data = np.asarray(data, dtype=np.float64)
    K = data.shape[0]
    n = ny * nx
    C = np.zeros((M * n, M * n))
    for a in range(M):
        for b in range(M):
            if a != b and a < K and b < K:
                continue
            C[a * n:(a + 1) * n, b * n:(b + 1) * n] = circulant(lag_cross_covariance(ens[:, a], ens[:, b]))
    H = np.zeros((K * n, M * n))
    for o in range(K):
        H[o * n:(o + 1) * n, o * n:(o + 1) * n] = np.eye(n)
    Rb = np.zeros((K * n, K * n))
    for o in range(K):
        Ro = np.asarray(R_dense[o], dtype=np.float64)
        Rb[o * n:(o + 1) * n, o * n:(o + 1) * n] = Ro * np.eye(n) if Ro.ndim == 0 else Ro
    U = ens.reshape(N, M * n).T                                        # [M n, N]
    D = data.reshape(K * n, 1) + np.asarray(e_phys, dtype=np.float64).reshape(N, K * n).T
    S = H @ C @ H.T + Rb
    X = np.linalg.solve(S, D - H @ U)
    return (U + C @ H.T @ X).T.reshape(N, M, ny, nx)
