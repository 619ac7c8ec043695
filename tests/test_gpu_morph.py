"""The extended-state analysis of the morphing EnKF (Section 2.2, eq. (9)) on the
GPU, through the C ABI, against the float64 oracle (oracle/morph.py).

K blocks of the state are observed (T_x, T_y and r(1) in the paper: K = 3),
each with its own data and R, their cross-covariances neglected.  Bar:
relative L2 over all members, blocks and points <= 1e-5 in float32 and
<= 1e-10 in float64, as for the other analyses: every block's update is the
same float32 arithmetic (transforms, sums over members, one division per bin
and observed field)."""

import ctypes

import numpy as np
import pytest
import torch

from oracle import morph
from paper_1001_1588_amd import _lib, twin

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = {np.float32: 1e-5, np.float64: 1e-10}


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def make_case(ny, nx, N, M, K, dt, seed, R_as):
    tw = twin.make_multiblock_twin(ny, nx, N, seed=seed, Ls=tuple(float(2 ** (1 + b % 5)) for b in range(M)),
                                   rho=0.6, r=0.02, dtype=dt)
    rng = np.random.default_rng(seed)
    r_obs = [0.02, 0.05, 0.01][:K]
    data = (tw.truth[:K] + np.sqrt(np.array(r_obs))[:, None, None] * rng.standard_normal((K, ny, nx))).astype(dt)
    if R_as == "array":
        ky = twin.integer_wavenumbers(ny)[:, None]
        kx = np.arange(nx // 2 + 1)[None, :].astype(np.float64)
        R = np.stack([r_obs[o] * (0.5 + 1.5 / (1.0 + (ky * ky + kx * kx) / (8.0 + 4 * o))) for o in range(K)]).astype(dt)
    else:
        R = np.array(r_obs)
    return tw.ens, data, R, tw.seed


# (ny, nx, N, M, K, dtype, R as)
CASES = [(16, 16, 4, 3, 3, np.float32, "scalar"), (32, 64, 5, 5, 3, np.float32, "array"),
         (64, 32, 8, 4, 3, np.float32, "scalar"), (128, 128, 5, 6, 3, np.float32, "array"),
         (64, 64, 3, 3, 2, np.float32, "array"), (8, 16, 4, 4, 3, np.float64, "array"),
         (64, 64, 2, 5, 3, np.float64, "scalar"), (32, 32, 4, 3, 2, np.float64, "scalar"),
         (256, 512, 6, 4, 3, np.float32, "scalar")]


def case_id(c):
    return f"{c[0]}x{c[1]}-N{c[2]}-M{c[3]}-K{c[4]}-{np.dtype(c[5]).name}-{c[6]}"


def run(ens, data, R, seed, out=None):
    Rd = dev(R) if R.ndim == 3 else [float(x) for x in R]
    res = _lib.analyze_morph(dev(ens), dev(data), Rd, seed, out=out)
    torch.cuda.synchronize()
    return res


@pytest.mark.parametrize("case", CASES, ids=case_id)
def test_morph_matches_oracle(case):
    ny, nx, N, M, K, dt, R_as = case
    ens, data, R, seed = make_case(ny, nx, N, M, K, dt, seed=ny + nx + 7 * N + 3 * M + K, R_as=R_as)
    got = run(ens, data, R, seed).cpu().numpy()
    ref = morph.analyze_morph(ens, data, R, seed, method="matmul" if ny * nx <= 65536 else "fft")
    assert rel_l2(got, ref) <= TOL[dt]
    for j in range(M):   # every block, observed and not
        assert rel_l2(got[:, j], ref[:, j]) <= 10 * TOL[dt]


def test_paper_shaped_state_at_512():
    """Five members (the paper's experiment) on a 512 x 512 grid with the
    extended state (T_x, T_y, r(1), r(2), r(3), r(4)) and three observed fields."""
    ens, data, R, seed = make_case(512, 512, 5, 6, 3, np.float32, seed=42, R_as="array")
    got = run(ens, data, R, seed).cpu().numpy()
    ref = morph.analyze_morph(ens, data, R, seed, method="fft")
    for j in range(6):
        assert rel_l2(got[:, j], ref[:, j]) <= 1e-5


def test_one_observed_field_is_the_multiblock_analysis():
    ens, data, R, seed = make_case(64, 128, 6, 4, 1, np.float32, seed=5, R_as="array")
    a = run(ens, data, R, seed)
    b = _lib.analyze_multi(dev(ens), dev(data[0]), dev(R[0]), seed)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_in_place_deterministic_and_seed():
    ens, data, R, seed = make_case(64, 64, 5, 4, 3, np.float32, seed=8, R_as="scalar")
    a = run(ens, data, R, seed)
    b = run(ens, data, R, seed)
    assert torch.equal(a, b)
    c = run(ens, data, R, seed + 1)
    assert not torch.equal(a, c)
    e = dev(ens)
    res = _lib.analyze_morph(e, dev(data), [float(x) for x in R], seed, out=e)
    torch.cuda.synchronize()
    assert res.data_ptr() == e.data_ptr() and torch.equal(e, a)


def test_collapsed_state_with_zero_R_returns_forecast():
    """Identical members, R_o zero on a subset of bins (the guarded division of
    eq. (3) for every observed field): no block moves."""
    ny, nx, N, M, K = 32, 64, 4, 5, 3
    rng = np.random.default_rng(3)
    base = rng.standard_normal((M, ny, nx)).astype(np.float32)
    ens = np.ascontiguousarray(np.broadcast_to(base, (N, M, ny, nx)))
    data = rng.standard_normal((K, ny, nx)).astype(np.float32)
    R = rng.uniform(0.01, 0.1, (K, ny, nx // 2 + 1))
    R[:, :, 0] = 0.0
    R[:, :, -1] = 0.0
    R[rng.random(R.shape) < 0.3] = 0.0
    R = R.astype(np.float32)
    got = run(ens, data, R, 4).cpu().numpy()
    assert np.isfinite(got).all()
    assert rel_l2(got, ens) <= 1e-5
    assert rel_l2(got, morph.analyze_morph(ens, data, R, 4)) <= 1e-5


def test_argument_errors():
    lib = _lib.lib()
    ens = torch.zeros((4, 3, 16, 16), device=DEV)
    data = torch.zeros((3, 16, 16), device=DEV)
    out = torch.full_like(ens, 7.0)
    with pytest.raises(RuntimeError, match="n_obs"):   # three observed fields, two blocks
        _lib.analyze_morph(torch.zeros((4, 2, 16, 16), device=DEV), data, [0.1] * 3, 1)
    with pytest.raises(RuntimeError, match="r_scalar"):
        _lib.analyze_morph(ens, data, [0.1, float("inf"), 0.1], 1, out=out)
    big = torch.zeros((9, 3, 16, 16), device=DEV)
    with pytest.raises(RuntimeError, match="exceeds"):
        _lib.analyze_morph(big, data, [0.1] * 3, 1)
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
    assert lib.fftenkf_max_members_morph(0, 3) == 8 and lib.fftenkf_max_members_morph(1, 3) == 4
    assert lib.fftenkf_max_members_morph(0, 1) == 12 and lib.fftenkf_max_members_morph(0, 4) == 0
    assert lib.fftenkf_workspace_bytes_morph(5, 6, 3, 512, 512, 0) == lib.fftenkf_workspace_bytes(32, 512, 512, 0)
    assert ctypes.sizeof(ctypes.c_double) == 8
