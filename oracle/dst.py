"""FFT EnKF with the real sine transform (Section 4): the plain reference form.

Test infrastructure only: the library never imports this module.

In its experiment (Section 4) the paper uses a real sine transform in place of
the periodic DFT, so that the analysis leaves the boundary values unchanged.
Here that transform is the
orthonormal DST-II on an n-point grid,

   S[k, j] = sqrt(2/n) c_k sin(pi (2 j + 1) (k + 1) / (2 n)),   c_{n-1} = 1/sqrt(2), else 1,

whose basis functions vanish at the cell faces j = -1/2 and j = n - 1/2; in 2D
it acts separably, s_hat = S_y u S_x^T, inverse u = S_y^T s_hat S_x.  The
analysis is eq. (2)-(3) in that basis with real coefficients:

   c_hat_i = 1/(N-1) sum_k (s_hat_ik - mean_k s_hat_ik)^2,
   s_hat_k^a = s_hat_k + c_hat / (c_hat + R_dst) (d_hat + e_hat_k - s_hat_k),

R_dst the eigenvalues of R in the sine basis (R = r I gives r everywhere) and
e_hat_k = sqrt(R_dst) z_k with z real standard normals (the sine transform of
white noise is white).  z for DST bin (s1, s2) and member k comes from
Philox4x32-10 with key = (seed lo, seed hi) and counter = (s1 * nx + s2,
k div 4, 1, 0): Box-Muller on words (x0, x1) gives members 4q and 4q + 1 (its
cosine and sine outputs), on (x2, x3) members 4q + 2 and 4q + 3.
"""

from __future__ import annotations

import numpy as np

from .enkf import spectral_gain, tiny_for
from .philox import box_muller, philox4x32


def dst2_matrix(n: int) -> np.ndarray:
    """Orthonormal DST-II matrix [n, n], S[k, j], written out from its definition."""
    k = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    S = np.sqrt(2.0 / n) * np.sin(np.pi * (2 * j + 1) * (k + 1) / (2 * n))
    S[n - 1] /= np.sqrt(2.0)
    return S


def dst2(u: np.ndarray, method: str = "matmul") -> np.ndarray:
    """Orthonormal 2D DST-II of real fields [..., ny, nx]; method "fft" is the
    same transform by scipy.fft (for large grids; pinned against the matrices)."""
    u = np.asarray(u, dtype=np.float64)
    ny, nx = u.shape[-2:]
    if method == "fft":
        import scipy.fft as sf
        return sf.dstn(u, type=2, norm="ortho", axes=(-2, -1))
    return dst2_matrix(ny) @ u @ dst2_matrix(nx).T


def idst2(s: np.ndarray, method: str = "matmul") -> np.ndarray:
    """Inverse of dst2 (the transpose: the matrices are orthogonal)."""
    s = np.asarray(s, dtype=np.float64)
    ny, nx = s.shape[-2:]
    if method == "fft":
        import scipy.fft as sf
        return sf.idstn(s, type=2, norm="ortho", axes=(-2, -1))
    return dst2_matrix(ny).T @ s @ dst2_matrix(nx)


def dst_noise(seed: int, N: int, ny: int, nx: int) -> np.ndarray:
    """Standard normals z [N, ny, nx] per member and DST bin (the convention above)."""
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    bins = np.arange(ny * nx, dtype=np.uint64)
    z = np.empty((N, ny * nx))
    for k in range(N):
        w = philox4x32((bins, np.uint64(k // 4), np.uint64(1), np.uint64(0)), key)
        wa, wb = (w[0], w[1]) if k % 4 < 2 else (w[2], w[3])
        z[k] = box_muller(wa, wb)[k % 2]
    return z.reshape(N, ny, nx)


def analyze_dst(ens, data, R_dst, seed: int, *, tiny=None, return_parts: bool = False, method: str = "matmul"):
    """Eq. (2)-(3) in the sine basis, with the seeded real perturbations."""
    ens = np.asarray(ens)
    N, ny, nx = ens.shape
    if tiny is None:
        tiny = tiny_for(ens.dtype)
    R_dst = np.broadcast_to(np.asarray(R_dst, dtype=np.float64), (ny, nx))
    s_hat = dst2(ens.astype(np.float64), method)
    d_hat = dst2(np.asarray(data, dtype=np.float64), method)
    # eq. (2) on the coefficients taken relative to the first member (the same
    # in exact arithmetic, exactly zero for a collapsed ensemble)
    rel = s_hat - s_hat[0:1]
    c_hat = ((rel - rel.mean(axis=0)) ** 2).sum(axis=0) / (N - 1)
    K = spectral_gain(c_hat, R_dst, tiny)
    e_hat = np.sqrt(R_dst)[None] * dst_noise(seed, N, ny, nx)
    sa = s_hat + K[None] * (d_hat[None] + e_hat - s_hat)
    ua = idst2(sa, method)
    if return_parts:
        return ua, dict(s_hat=s_hat, d_hat=d_hat, c_hat=c_hat, K=K, e_hat=e_hat)
    return ua


def analyze_dst_dense(ens, data, R_dst, e_hat) -> np.ndarray:
    """Eq. (1) with the covariance S^T diag(c) S, c_i = (S Sigma S^T)_ii the
    diagonal of the sample covariance Sigma in the sine basis (each entry
    e_i^T Sigma e_i), and R = S^T diag(R_dst) S; dense solve.  e_hat [N, ny, nx]
    are the perturbations' sine coefficients."""
    ens = np.asarray(ens, dtype=np.float64)
    N, ny, nx = ens.shape
    n = ny * nx
    S = np.kron(dst2_matrix(ny), dst2_matrix(nx))          # acts on row-major fields
    U = ens.reshape(N, n).T
    D = U - U.mean(axis=1, keepdims=True)
    Sigma = D @ D.T / (N - 1)
    c = np.einsum("ij,jk,ik->i", S, Sigma, S)
    C = S.T @ np.diag(c) @ S
    Rd = S.T @ np.diag(np.broadcast_to(np.asarray(R_dst, dtype=np.float64), (ny, nx)).ravel()) @ S
    e_phys = (S.T @ np.asarray(e_hat).reshape(N, n).T)
    innov = np.asarray(data, dtype=np.float64).reshape(n, 1) + e_phys - U
    return (U + C @ np.linalg.solve(C + Rd, innov)).T.reshape(N, ny, nx)
