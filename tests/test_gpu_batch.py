"""Batched uneven filters (fftenkf_analyze_batch) on the GPU.

Every filter's output must be bitwise equal to fftenkf_analyze on the same
arguments (the same kernels run, with the filter chosen by the launch's second
grid dimension), and within the single-filter bar (1e-5 relative L2 in float32,
1e-10 in float64) of the float64 oracle.  A captured graph replayed several
times, with eager work between the replays, reproduces the eager result every
time.  Launch chains of different grids run on side streams forked from and
joined into the caller's, which orders the batch with the caller's own work.
The tile schedule chosen by the tuner changes the rounding only."""

import numpy as np
import pytest
import torch

from oracle import enkf
from paper_1001_1588_amd import _lib, twin

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def make_batch(shapes, N, dtype, seed, R_as=("array", "scalar")):
    tws = [twin.random_ensemble(ny, nx, N, seed=seed + i, dtype=dtype, r=0.01,
                                R_kind="spectral" if i % 2 == 0 else "scalar") for i, (ny, nx) in enumerate(shapes)]
    ens = [dev(t.ens) for t in tws]
    data = [dev(t.data) for t in tws]
    R = [dev(t.R_spec) if R_as[i % len(R_as)] == "array" else float(t.r) for i, t in enumerate(tws)]
    return tws, ens, data, R


@pytest.mark.parametrize("dtype", [np.float32, np.float64], ids=["float32", "float64"])
def test_batch_equals_single_and_oracle(dtype):
    shapes = [(64, 64), (16, 32), (64, 64), (128, 64), (8, 8), (256, 256), (16, 32), (64, 64), (32, 1024)]
    N = 6
    tws, ens, data, R = make_batch(shapes, N, dtype, seed=100)
    seeds = [t.seed for t in tws]
    b = _lib.Batch(ens, data, R, seeds)
    outs = b.run()
    singles = [_lib.analyze(ens[i], data[i], R[i], seeds[i]) for i in range(len(shapes))]
    torch.cuda.synchronize()
    tol = 1e-5 if dtype == np.float32 else 1e-10
    for i, (t, o, s) in enumerate(zip(tws, outs, singles)):
        assert torch.equal(o, s), f"filter {i} differs from the single-filter analysis"
        ny, nx = shapes[i]
        ref = enkf.analyze(t.ens, t.data, t.R_spec, t.seed, method="matmul" if ny * nx <= 65536 else "fft")
        assert rel_l2(o.cpu().numpy(), ref) <= tol, f"filter {i}"


def test_more_filters_of_one_size_than_one_launch_holds():
    shapes = [(32, 32)] * 45 + [(64, 128)] * 3
    tws, ens, data, R = make_batch(shapes, 4, np.float32, seed=300)
    b = _lib.Batch(ens, data, R, [t.seed for t in tws])
    outs = b.run()
    torch.cuda.synchronize()
    for i in (0, 39, 40, 44, 46):
        single = _lib.analyze(ens[i], data[i], R[i], tws[i].seed)
        torch.cuda.synchronize()
        assert torch.equal(outs[i], single), f"filter {i}"


def test_graph_replays_match_eager():
    shapes = [(64, 64), (128, 128), (64, 64), (256, 128), (32, 32)]
    tws, ens, data, R = make_batch(shapes, 8, np.float32, seed=500)
    b = _lib.Batch(ens, data, R, [t.seed for t in tws])
    eager = [o.clone() for o in b.run()]
    torch.cuda.synchronize()
    b.capture()
    for rep in range(4):
        for o in b.out:
            o.zero_()
        junk = torch.randn(1 << 20, device=DEV) * 3          # eager work between replays
        torch.cuda.synchronize()
        outs = b.replay()
        torch.cuda.synchronize()
        for i in range(len(shapes)):
            assert torch.equal(outs[i], eager[i]), f"replay {rep}, filter {i}"
        del junk


def test_batch_orders_with_the_callers_stream():
    """Filters of several grid sizes run on streams forked from the caller's
    and joined back into it: inputs written on the caller's stream just before
    the batch are the ones analysed, and work queued on that stream right after
    it reads the finished outputs (no device synchronisation in between)."""
    shapes = [(1024, 1024), (64, 64), (256, 256), (128, 128), (512, 512)]
    tws, ens, data, R = make_batch(shapes, 8, np.float32, seed=650)
    refs = [_lib.analyze(ens[i], data[i], R[i], tws[i].seed).clone() for i in range(len(shapes))]
    torch.cuda.synchronize()
    src = [e.clone() for e in ens]
    b = _lib.Batch(ens, data, R, [t.seed for t in tws])
    for rep in range(3):
        for e in ens:
            e.fill_(7.0)                     # overwritten below on the same stream
        torch.cuda.synchronize()
        for e, s in zip(ens, src):
            e.copy_(s)                       # queued, not waited for
        outs = b.run()
        after = [o.clone() for o in outs]    # queued behind the batch's join
        for o in outs:
            o.zero_()
        torch.cuda.synchronize()
        for i in range(len(shapes)):
            assert torch.equal(after[i], refs[i]), f"rep {rep}, filter {i} ({shapes[i]})"


def test_in_place_batch():
    shapes = [(64, 64), (32, 128)]
    tws, ens, data, R = make_batch(shapes, 5, np.float32, seed=700)
    ref = [_lib.analyze(ens[i], data[i], R[i], tws[i].seed) for i in range(2)]
    b = _lib.Batch(ens, data, R, [t.seed for t in tws], out=ens)
    b.run()
    torch.cuda.synchronize()
    for i in range(2):
        assert torch.equal(ens[i], ref[i])


def test_tile_rows_change_rounding_only():
    tw = twin.random_ensemble(256, 256, 8, seed=11, dtype=np.float32)
    e, d = dev(tw.ens), dev(tw.data)
    opts = _lib.tile_rows_options(256, 256, torch.float32)
    assert opts == [4, 8, 16]
    outs = []
    try:
        for r in opts:
            _lib.set_tile_rows(256, 256, torch.float32, r)
            assert _lib.tile_rows(256, 256, torch.float32) == r
            outs.append(_lib.analyze(e, d, 0.01, tw.seed).cpu().numpy())
    finally:
        _lib.set_tile_rows(256, 256, torch.float32, 0)
    ref = enkf.analyze(tw.ens, tw.data, 0.01, tw.seed, method="fft")
    for o in outs:
        assert rel_l2(o, ref) <= 1e-5
    with pytest.raises(RuntimeError):
        _lib.set_tile_rows(256, 256, torch.float32, 32)


def test_autotuner_sets_a_compiled_choice():
    from paper_1001_1588_amd import autotune
    grids = [(128, 128), (64, 256)]
    try:
        table = autotune.tune(grids, 8, torch.float32, reps=3)
        for ny, nx in grids:
            rec = table[autotune.key(ny, nx, torch.float32)]
            assert rec["rows"] in _lib.tile_rows_options(ny, nx, torch.float32)
            assert _lib.tile_rows(ny, nx, torch.float32) == rec["rows"]
            assert all(t > 0 for t in rec["ms"].values())
    finally:
        for ny, nx in grids:
            _lib.set_tile_rows(ny, nx, torch.float32, 0)


def test_device_twin_statistics():
    """The device generator of the batched workload draws the stated law."""
    ens, data, seed = twin.device_twin(128, 128, 16, seed=4, r=0.01, device=DEV)
    lam = twin.spectrum(128, 128, "matern2")[:, :65]
    dev_ = ens - ens.mean(dim=0, keepdim=True)
    c = (torch.fft.rfft2(dev_.double(), norm="ortho").abs() ** 2).sum(dim=0) / 15
    ratio = float((c.cpu().numpy() / lam).mean())
    assert abs(ratio - 1) < 0.02
    # data = truth + N(0, r I): at high wavenumbers the fields carry almost no
    # power, so d - mean(ens) has the unitary power r of the white noise there
    resid = torch.fft.rfft2((data - ens.mean(dim=0)).double(), norm="ortho").abs() ** 2
    ky = torch.minimum(torch.arange(128), 128 - torch.arange(128))[:, None].double()
    kx = torch.arange(65)[None, :].double()
    high = ((ky ** 2 + kx ** 2) > 40 ** 2).to(DEV)
    assert abs(float(resid[high].mean()) / 0.01 - 1) < 0.05


def test_batch_at_the_benchmark_shape():
    """The batched workload's own law: N = 16, float32, square sides from
    {64, 128, 256, 512, 1024} (two of each, shuffled), spectrum (1+|k|^2)^-2,
    R = 0.01 I, tile rows chosen by the autotuner.  Every filter is checked
    against the oracle (the library FFT form from 512 up, which the oracle's
    tests pin to its matrix form) and bitwise against a single-filter call, and
    the captured graph reproduces the eager batch."""
    from paper_1001_1588_amd import autotune

    sides = [512, 64, 1024, 128, 256, 1024, 64, 512, 256, 128]
    N = 16
    tws = [twin.make_twin(s, s, N, seed=900 + i, dtype=np.float32, kind="matern2", r=0.01)
           for i, s in enumerate(sides)]
    grids = sorted({(s, s) for s in sides})
    try:
        autotune.tune(grids, N, torch.float32, reps=2)
        ens = [dev(t.ens) for t in tws]
        data = [dev(t.data) for t in tws]
        b = _lib.Batch(ens, data, [0.01] * len(sides), [t.seed for t in tws])
        outs = [o.clone() for o in b.run()]
        torch.cuda.synchronize()
        for i, t in enumerate(tws):
            single = _lib.analyze(ens[i], data[i], 0.01, t.seed)
            torch.cuda.synchronize()
            assert torch.equal(outs[i], single), f"filter {i} ({sides[i]}^2) differs from the single-filter analysis"
            ref = enkf.analyze(t.ens, t.data, 0.01, t.seed, method="matmul" if sides[i] <= 256 else "fft")
            assert rel_l2(outs[i].cpu().numpy(), ref) <= 1e-5, f"filter {i} ({sides[i]}^2)"
        b.capture()
        for rep in range(2):
            for o in b.out:
                o.zero_()
            torch.cuda.synchronize()
            replay = b.replay()
            torch.cuda.synchronize()
            for i in range(len(sides)):
                assert torch.equal(replay[i], outs[i]), f"replay {rep}, filter {i}"
    finally:
        for g in grids:
            _lib.set_tile_rows(g[0], g[1], torch.float32, 0)
