"""The trainer forms the kernel's features and exports weights the kernel reads.

Checked against the oracle's definitions (oracle/learned.py) and the twin
generator, on the CPU."""

import json

import numpy as np
import pytest
import torch

from oracle import learned
from paper_1001_1588_amd import train_spectral_mlp as tr
from paper_1001_1588_amd import twin


@pytest.mark.parametrize("a", [2.0, 3.3, 4.0])
def test_power_spectrum_is_the_twin_spectrum(a):
    k2 = tr.squared_wavenumbers(32, 16, "cpu")
    assert np.allclose(tr.power_spectrum(k2, a).numpy(), twin.spectrum(32, 16, "power", a=a), rtol=1e-12)


def test_features_are_the_oracle_features():
    ny, nx = 16, 32
    gen = torch.Generator().manual_seed(0)
    lam = tr.power_spectrum(tr.squared_wavenumbers(ny, nx, "cpu"), 2.5)
    c = tr.sample_spectrum(lam, 5, gen)
    c_half = c[:, : nx // 2 + 1].numpy()
    ref = learned.features(c_half, nx)
    ky, kx = torch.meshgrid(torch.arange(ny), torch.arange(nx // 2 + 1), indexing="ij")
    f, mu = tr.bin_features(c, ky.reshape(-1), kx.reshape(-1))
    assert float(mu) == pytest.approx(c_half.mean(), rel=1e-12)
    # the trainer reads the full spectrum, the oracle mirrors the stored half: the
    # float32 draws make the full spectrum even to float32 rounding only
    assert np.allclose(f.numpy().reshape(ny, nx // 2 + 1, 26), ref, rtol=1e-5, atol=1e-5)


def test_sample_spectrum_is_unbiased():
    gen = torch.Generator().manual_seed(1)
    lam = tr.power_spectrum(tr.squared_wavenumbers(16, 16, "cpu"), 2.0)
    c = torch.stack([tr.sample_spectrum(lam, 4, gen) for _ in range(400)]).mean(dim=0)
    # mean of 400 draws of lam * chi^2_6 / 6 (3 complex dof): relative sd 0.029 at generic bins
    ok = lam > 0
    assert torch.all(torch.abs(c[ok] / lam[ok] - 1) < 0.25)
    assert abs(float((c[ok] / lam[ok]).mean()) - 1) < 0.01


def test_sampled_bins_are_stored_bins():
    gen = torch.Generator().manual_seed(2)
    ky, kx = tr.sample_bins(5000, 64, 32, gen, "cpu")
    assert int(ky.min()) >= 0 and int(ky.max()) < 64 and int(kx.min()) >= 0 and int(kx.max()) <= 16
    # the log-uniform half puts many more samples at low |k| than uniform sampling (~3% at |k| <= 4)
    k = (torch.minimum(ky, 64 - ky) ** 2 + kx ** 2).double().sqrt()
    assert float((k <= 4).double().mean()) > 0.15


def test_export_folds_standardisation_into_the_first_layer():
    torch.manual_seed(0)
    net = tr.make_net().double()
    x = torch.randn(200, 26, dtype=torch.float64) * 3 + 1
    mean, std = x.mean(dim=0), x.std(dim=0)
    w = tr.export(net, mean, std)
    with torch.no_grad():
        ref = net((x - mean) / std)[:, 0].numpy()
    got = learned.mlp(x.numpy(), w, bf16=False)
    assert np.allclose(got, ref, rtol=2e-5, atol=2e-5)   # exported weights are float32
    # and the bfloat16 emulation the trainer reports matches the oracle's bfloat16 form
    pred = tr.predict_bf16(w, x.float()).numpy()
    assert np.allclose(pred, learned.mlp(x.numpy().astype(np.float32), w, bf16=True), rtol=1e-4, atol=1e-4)


def test_tiny_training_run(tmp_path):
    out = tmp_path / "w.npz"
    tr.main(["--out", str(out), "--twins", "6", "--val-twins", "2", "--bins", "256", "--size", "32",
             "--epochs", "1", "--batch", "256", "--device", "cpu"])
    d = np.load(out)
    for k, shape in [("W1", (26, 64)), ("W2", (64, 64)), ("W3", (64, 64)), ("w4", (64,)), ("b4", (1,))]:
        assert d[k].shape == shape and d[k].dtype == np.float32
    meta = json.loads(str(d["meta"]))
    assert meta["members"] == 5 and np.isfinite(meta["val_mse_bf16"])


def test_autotune_pick_and_table_roundtrip(tmp_path, monkeypatch):
    from paper_1001_1588_amd import autotune
    assert autotune.pick({8: 1.0, 16: 0.5}) == 16
    assert autotune.pick({8: 0.5, 16: 0.5}) == 8           # ties: fewer rows
    calls = []
    monkeypatch.setattr(autotune._lib, "set_tile_rows", lambda ny, nx, dt, r: calls.append((ny, nx, dt, r)))
    table = {"256x256:float32": {"rows": 8}, "64x4096:float64": {"rows": 4}}
    p = tmp_path / "t.json"
    p.write_text(__import__("json").dumps(table))
    autotune.load(str(p))
    assert calls == [(256, 256, torch.float32, 8), (64, 4096, torch.float64, 4)]


def test_batch_sides_are_seeded_and_uniform():
    a = twin.batch_sides(256, 1)
    assert a == twin.batch_sides(256, 1) and a != twin.batch_sides(256, 2)
    assert set(a) == {64, 128, 256, 512, 1024}
    assert all(20 < a.count(s) < 85 for s in set(a))
