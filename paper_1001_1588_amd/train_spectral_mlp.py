"""Training of the learned spectral covariance used by fftenkf_analyze_learned.

Twin experiments are drawn on the device.  For each one, a ~ U(a_lo, a_hi) and
lambda = |k|^-a (lambda(0) = 0, normalised to mean 1) is the covariance
spectrum of a stationary Gaussian field; N independent draws of that field give
the sample spectrum c_hat of eq. (2) on the unitary scale (the truth a forecast
ensemble is centred on cancels in eq. (2), so draws suffice).  The inputs are
the ones the kernel forms -- log(c_hat / mu + 1e-6) over the 5 x 5 wavenumber
neighbourhood of the bin on the full periodic spectrum and log(1 + |k|), with mu
the mean of c_hat over the stored half-spectrum bins -- and the target is
log(lambda / mu + 1e-6), so that mu exp(y) estimates lambda.  Bins are sampled
half uniformly over the half spectrum and half log-uniformly in |k|, so the
few low wavenumbers that hold most of the variance are seen often.  The loss is
the mean squared error of y.

The input standardisation used while training is folded into the first layer
on export: the saved weights take the raw features, as the kernel does.

    python -m paper_1001_1588_amd.train_spectral_mlp --out spectral_mlp_n5.npz
"""

from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np
import torch

N_FEATURES = 26
WIDTH = 64
EPS = 1e-6


def power_spectrum(k2: torch.Tensor, a: float) -> torch.Tensor:
    """|k|^-a on the full grid (0 at k = 0), normalised to mean 1."""
    lam = torch.where(k2 > 0, k2.clamp_min(1.0).pow(-a / 2.0), torch.zeros_like(k2))
    return lam / lam.mean()


def squared_wavenumbers(ny: int, nx: int, device) -> torch.Tensor:
    ky = torch.arange(ny, device=device, dtype=torch.float64)
    kx = torch.arange(nx, device=device, dtype=torch.float64)
    ky = torch.minimum(ky, ny - ky)[:, None]
    kx = torch.minimum(kx, nx - kx)[None, :]
    return ky * ky + kx * kx


def sample_spectrum(lam: torch.Tensor, N: int, gen: torch.Generator) -> torch.Tensor:
    """c_hat (unitary, full [ny, nx] grid) of N draws of the field with spectrum lam."""
    ny, nx = lam.shape
    w = torch.randn((N, ny, nx), generator=gen, device=lam.device, dtype=torch.float32)
    z = torch.fft.fft2(w, norm="ortho") * lam.sqrt().to(torch.float32)
    d = z - z.mean(dim=0, keepdim=True)
    return (d.real.square() + d.imag.square()).sum(dim=0).double() / (N - 1)


def sample_bins(n: int, ny: int, nx: int, gen: torch.Generator, device):
    """n stored bins (ky, kx), half uniform and half log-uniform in |k|."""
    nh = nx // 2 + 1
    h = n // 2
    ky_u = torch.randint(0, ny, (h,), generator=gen, device=device)
    kx_u = torch.randint(0, nh, (h,), generator=gen, device=device)
    m = n - h
    rmax = math.hypot(ny / 2, nx / 2)
    r = torch.exp(torch.rand(m, generator=gen, device=device, dtype=torch.float64) * math.log(rmax))
    th = (torch.rand(m, generator=gen, device=device, dtype=torch.float64) - 0.5) * math.pi
    kx_l = torch.round(r * torch.cos(th)).long().clamp(0, nx // 2)
    ky_l = torch.round(r * torch.sin(th)).long().clamp(-(ny // 2), ny // 2) % ny
    return torch.cat([ky_u, ky_l]), torch.cat([kx_u, kx_l])


def bin_features(c: torch.Tensor, ky: torch.Tensor, kx: torch.Tensor):
    """Features [n, 26] of the bins (ky, kx) from the full sample spectrum c, and mu."""
    ny, nx = c.shape
    mu = c[:, : nx // 2 + 1].mean()
    logc = torch.log(c / mu + EPS)
    cols = []
    for j in range(25):
        dy, dx = j // 5 - 2, j % 5 - 2
        cols.append(logc[(ky + dy) % ny, (kx + dx) % nx])
    kyw = torch.minimum(ky, ny - ky).double()
    cols.append(torch.log1p(torch.sqrt(kyw * kyw + kx.double() ** 2)))
    return torch.stack(cols, dim=1), mu


def make_dataset(twins: int, bins: int, ny: int, nx: int, N: int, a_range, seed: int, device):
    """(X [twins * bins, 26], Y [twins * bins]) in float32 on the device."""
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    k2 = squared_wavenumbers(ny, nx, device)
    X = torch.empty((twins * bins, N_FEATURES), device=device, dtype=torch.float32)
    Y = torch.empty((twins * bins,), device=device, dtype=torch.float32)
    for t in range(twins):
        a = a_range[0] + (a_range[1] - a_range[0]) * float(torch.rand(1, generator=gen, device=device))
        lam = power_spectrum(k2, a)
        c = sample_spectrum(lam, N, gen)
        ky, kx = sample_bins(bins, ny, nx, gen, device)
        f, mu = bin_features(c, ky, kx)
        X[t * bins:(t + 1) * bins] = f.float()
        Y[t * bins:(t + 1) * bins] = torch.log(lam[ky, kx] / mu + EPS).float()
    return X, Y


def make_net() -> torch.nn.Sequential:
    return torch.nn.Sequential(torch.nn.Linear(N_FEATURES, WIDTH), torch.nn.ReLU(), torch.nn.Linear(WIDTH, WIDTH),
                               torch.nn.ReLU(), torch.nn.Linear(WIDTH, WIDTH), torch.nn.ReLU(),
                               torch.nn.Linear(WIDTH, 1))


def export(net: torch.nn.Sequential, mean: torch.Tensor, std: torch.Tensor) -> dict:
    """Weights on the raw features: x_std = (x - mean) / std folded into layer 1."""
    W1 = net[0].weight.detach().double().T / std.double()[:, None]          # [26, 64]
    b1 = net[0].bias.detach().double() - (mean.double() / std.double()) @ (net[0].weight.detach().double().T)
    out = dict(W1=W1, b1=b1, W2=net[2].weight.detach().double().T, b2=net[2].bias.detach().double(),
               W3=net[4].weight.detach().double().T, b3=net[4].bias.detach().double(),
               w4=net[6].weight.detach().double().reshape(-1), b4=net[6].bias.detach().double().reshape(1))
    return {k: v.cpu().numpy().astype(np.float32) for k, v in out.items()}


def bf16(t: torch.Tensor) -> torch.Tensor:
    return t.to(torch.bfloat16).to(torch.float32)


def predict_bf16(w: dict, X: torch.Tensor) -> torch.Tensor:
    """The kernel's arithmetic: bfloat16 inputs, weights and activations, float32 sums."""
    dev = X.device
    t = {k: torch.as_tensor(v, device=dev, dtype=torch.float32) for k, v in w.items()}
    h = bf16(X)
    for n in ("1", "2", "3"):
        h = bf16(torch.relu(h @ bf16(t["W" + n]) + t["b" + n]))
    return h @ bf16(t["w4"]) + t["b4"][0]


def train(args) -> dict:
    device = torch.device(args.device)
    t0 = time.time()
    X, Y = make_dataset(args.twins, args.bins, args.size, args.size, args.members, (args.a_lo, args.a_hi),
                        args.seed, device)
    Xv, Yv = make_dataset(args.val_twins, args.bins, args.size, args.size, args.members, (args.a_lo, args.a_hi),
                          args.seed + 7919, device)
    print(f"data: {X.shape[0]} train / {Xv.shape[0]} validation samples in {time.time() - t0:.1f}s", flush=True)
    mean, std = X.mean(dim=0), X.std(dim=0).clamp_min(1e-3)
    torch.manual_seed(args.seed)
    net = make_net().to(device)
    opt = torch.optim.Adam(net.parameters(), lr=args.lr)
    steps_per_epoch = X.shape[0] // args.batch
    total = steps_per_epoch * args.epochs
    sched = torch.optim.lr_scheduler.OneCycleLR(opt, max_lr=args.lr, total_steps=total, pct_start=0.1)
    gen = torch.Generator(device=device)
    gen.manual_seed(args.seed + 1)
    Xs, Xvs = (X - mean) / std, (Xv - mean) / std
    for ep in range(args.epochs):
        perm = torch.randperm(X.shape[0], generator=gen, device=device)
        net.train()
        run = 0.0
        for s in range(steps_per_epoch):
            idx = perm[s * args.batch:(s + 1) * args.batch]
            loss = torch.mean((net(Xs[idx])[:, 0] - Y[idx]) ** 2)
            opt.zero_grad(set_to_none=True)
            loss.backward()
            opt.step()
            sched.step()
            run += float(loss.detach()) if s % 50 == 0 else 0.0
        net.eval()
        with torch.no_grad():
            val = float(torch.mean((net(Xvs)[:, 0] - Yv) ** 2))
        print(f"epoch {ep + 1}/{args.epochs}: train~{run / max(1, (steps_per_epoch + 49) // 50):.4f} "
              f"val {val:.4f} ({time.time() - t0:.0f}s)", flush=True)
    w = export(net, mean, std)
    with torch.no_grad():
        val_bf16 = float(torch.mean((predict_bf16(w, Xv) - Yv) ** 2))
        val_plain = float(torch.mean((Xv[:, 12] - Yv) ** 2))   # log c_hat itself, the plain estimate
    meta = dict(twins=args.twins, val_twins=args.val_twins, bins_per_twin=args.bins, grid=args.size,
                members=args.members, a_range=[args.a_lo, args.a_hi], epochs=args.epochs, seed=args.seed,
                val_mse_fp32=val, val_mse_bf16=val_bf16, val_mse_plain=val_plain)
    print(json.dumps(meta), flush=True)
    return dict(w, meta=np.array(json.dumps(meta)))


def main(argv=None) -> None:
    p = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    p.add_argument("--out", required=True)
    p.add_argument("--twins", type=int, default=10000)
    p.add_argument("--val-twins", type=int, default=200)
    p.add_argument("--bins", type=int, default=2048, help="sampled bins per twin")
    p.add_argument("--size", type=int, default=2048)
    p.add_argument("--members", type=int, default=5)
    p.add_argument("--a-lo", type=float, default=2.0)
    p.add_argument("--a-hi", type=float, default=4.0)
    p.add_argument("--epochs", type=int, default=12)
    p.add_argument("--batch", type=int, default=8192)
    p.add_argument("--lr", type=float, default=3e-3)
    p.add_argument("--seed", type=int, default=20100109)
    p.add_argument("--device", default="cuda")
    args = p.parse_args(argv)
    res = train(args)
    np.savez(args.out, **res)
    print(f"wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
