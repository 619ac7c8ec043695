"""Pins of oracle/learned.py, the learned spectral covariance.

Each pin comes from something other than the oracle's own formula:

* bfloat16 rounding against torch's float32 -> bfloat16 conversion, and against
  hand-worked ties;
* the full even spectrum against |fft2|^2 of a real field (no mirroring);
* the features against a per-bin brute force on the full FFT spectrum;
* the perceptron against closed forms (constant output, an identity network
  that returns the log spectrum) and against torch.nn layers in float64;
* the learned analysis with the identity network against the plain analysis
  of eq. (2)-(3), since lambda_hat = c_hat + 1e-6 mu then.
"""

import numpy as np
import pytest
import torch

from oracle import dft, enkf, learned
from paper_1001_1588_amd import twin


def test_round_bf16_hand_ties():
    one = 1.0
    ulp = 2.0 ** -7                           # bfloat16 has 7 stored mantissa bits
    x = np.array([one, one + ulp / 2, one + 1.5 * ulp, one + ulp / 2 + 2.0 ** -20, -3.0, 0.0, 2.0 ** -130])
    want = np.array([one, one, one + 2 * ulp, one + ulp, -3.0, 0.0, 2.0 ** -130], dtype=np.float32)
    got = learned.round_bf16(x)
    assert np.array_equal(got, want)


def test_round_bf16_matches_torch():
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-6, 6, 20000),
                        rng.uniform(-1, 1, 1000).astype(np.float32)]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(learned.round_bf16(x), ref)


@pytest.mark.parametrize("ny,nx", [(8, 8), (16, 8), (8, 32)])
def test_full_spectrum_even_is_the_fft_power(ny, nx):
    rng = np.random.default_rng(ny + nx)
    f = rng.standard_normal((ny, nx))
    full = np.abs(np.fft.fft2(f)) ** 2
    half = full[:, : nx // 2 + 1]
    assert np.allclose(learned.full_spectrum_even(half, nx), full, rtol=1e-12, atol=1e-12)


def test_features_brute_force():
    ny, nx = 16, 8
    rng = np.random.default_rng(9)
    fields = rng.standard_normal((3, ny, nx))
    full = np.var(np.fft.fft2(fields, norm="ortho"), axis=0, ddof=1)  # even, from real fields
    half = full[:, : nx // 2 + 1]
    mu = half.mean()
    feats = learned.features(half, nx)
    for ky in range(ny):
        for kx in range(nx // 2 + 1):
            for j in range(25):
                dy, dx = j // 5 - 2, j % 5 - 2
                want = np.log(full[(ky + dy) % ny, (kx + dx) % nx] / mu + 1e-6)
                assert feats[ky, kx, j] == pytest.approx(want, rel=1e-12, abs=1e-12)
            kyw = min(ky, ny - ky)
            assert feats[ky, kx, 25] == pytest.approx(np.log(1.0 + np.hypot(kyw, kx)), rel=1e-14)
    # the centre feature is the bin itself
    assert np.allclose(feats[:, :, 12], np.log(half / mu + 1e-6))


def zero_weights():
    return dict(W1=np.zeros((26, 64)), b1=np.zeros(64), W2=np.zeros((64, 64)), b2=np.zeros(64),
                W3=np.zeros((64, 64)), b3=np.zeros(64), w4=np.zeros(64), b4=np.zeros(1))


def identity_weights():
    """A network whose output is feature 12 (the log of the bin's own spectrum)."""
    w = zero_weights()
    w["W1"][12, 0], w["W1"][12, 1] = 1.0, -1.0
    w["W2"][0, 0], w["W2"][1, 1] = 1.0, 1.0
    w["W3"][0, 0], w["W3"][1, 1] = 1.0, 1.0
    w["w4"][0], w["w4"][1] = 1.0, -1.0
    return w


def test_constant_network():
    w = zero_weights()
    w["b4"][0] = np.log(2.0)
    c = np.random.default_rng(1).uniform(0.1, 3.0, (8, 5))
    lam, mu = learned.learned_spectrum(c, 8, w, bf16=False)
    assert mu == pytest.approx(c.mean())
    assert np.allclose(lam, 2.0 * c.mean(), rtol=1e-14)
    # ReLU blocks negative pre-activations: a large negative bias leaves only b4
    w["b1"][:] = -5.0
    w["W1"][:] = 0.1
    w["w4"][:] = 7.0
    lam, _ = learned.learned_spectrum(c, 8, w, bf16=False)
    assert np.allclose(lam, 2.0 * c.mean(), rtol=1e-14)


def test_identity_network_returns_the_spectrum():
    c = np.random.default_rng(2).uniform(0.01, 5.0, (16, 9))
    lam, mu = learned.learned_spectrum(c, 16, identity_weights(), bf16=False)
    assert np.allclose(lam, c + 1e-6 * mu, rtol=1e-12)
    # in bfloat16 the input log is rounded once: a relative error below 2^-8 |log|
    lam16, _ = learned.learned_spectrum(c, 16, identity_weights(), bf16=True)
    x = np.log(c / mu + 1e-6)
    assert np.all(np.abs(np.log(lam16 / mu) - x) <= np.abs(x) * 2.0 ** -8 + 1e-12)


def test_mlp_matches_torch_layers():
    rng = np.random.default_rng(3)
    w = dict(W1=rng.standard_normal((26, 64)) * 0.3, b1=rng.standard_normal(64) * 0.1,
             W2=rng.standard_normal((64, 64)) * 0.2, b2=rng.standard_normal(64) * 0.1,
             W3=rng.standard_normal((64, 64)) * 0.2, b3=rng.standard_normal(64) * 0.1,
             w4=rng.standard_normal(64) * 0.2, b4=rng.standard_normal(1) * 0.1)
    x = rng.standard_normal((300, 26))
    net = torch.nn.Sequential(torch.nn.Linear(26, 64), torch.nn.ReLU(), torch.nn.Linear(64, 64), torch.nn.ReLU(),
                              torch.nn.Linear(64, 64), torch.nn.ReLU(), torch.nn.Linear(64, 1)).double()
    with torch.no_grad():
        for layer, (W, b) in zip([net[0], net[2], net[4], net[6]],
                                 [("W1", "b1"), ("W2", "b2"), ("W3", "b3"), ("w4", "b4")]):
            # biases are held in float32 by the network's definition
            layer.weight.copy_(torch.from_numpy(np.asarray(w[W]).reshape(-1, layer.out_features).T.copy()))
            layer.bias.copy_(torch.from_numpy(np.asarray(w[b], dtype=np.float32).astype(np.float64).reshape(-1)))
        ref = net(torch.from_numpy(x)).numpy()[:, 0]
    assert np.allclose(learned.mlp(x, w, bf16=False), ref, rtol=1e-12, atol=1e-12)
    # bfloat16 form: the same layers with torch's bfloat16 rounding at each product input
    rb = lambda a: torch.from_numpy(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).double()  # noqa: E731
    h = rb(x)
    for W, b in [("W1", "b1"), ("W2", "b2"), ("W3", "b3")]:
        h = torch.relu(h @ rb(w[W]) + torch.from_numpy(np.asarray(w[b], dtype=np.float32)).double())
        h = rb(h.float().numpy())
    ref16 = (h @ rb(w["w4"]) + float(np.float32(w["b4"][0]))).numpy()
    assert np.allclose(learned.mlp(x, w, bf16=True), ref16, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("ny,nx,N", [(16, 16, 4), (32, 16, 5)])
def test_identity_network_analysis_is_the_plain_analysis(ny, nx, N):
    tw = twin.random_ensemble(ny, nx, N, seed=ny + nx + N, dtype=np.float64, r=0.05, R_kind="spectral")
    plain = enkf.analyze(tw.ens, tw.data, tw.R_spec, tw.seed)
    ua, parts = learned.analyze_learned(tw.ens, tw.data, tw.R_spec, tw.seed, identity_weights(), bf16=False,
                                        return_parts=True)
    _, c_hat = enkf.spectral_mean_variance(dft.rdft2(tw.ens.astype(np.float64)))
    assert np.allclose(parts["lam"], c_hat + 1e-6 * c_hat.mean(), rtol=1e-10)
    # the gain moves by at most 1e-6 mu / (c_hat + R); the update by that times the innovation
    assert np.linalg.norm(ua - plain) / np.linalg.norm(plain) < 1e-5
    # a constant network gives the filter with a flat spectrum mu * e^b4
    w = zero_weights()
    w["b4"][0] = 0.5
    ua2, parts2 = learned.analyze_learned(tw.ens, tw.data, tw.R_spec, tw.seed, w, bf16=False, return_parts=True)
    lam = np.exp(0.5) * c_hat.mean()
    assert np.allclose(parts2["K"], lam / (lam + tw.R_spec), rtol=1e-12)
