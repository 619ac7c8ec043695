"""Analysis RMSE of the plain, learned and known-spectrum filters on twin experiments.

For a twin (truth, forecast ensemble, data; twin.py) each filter's analysis
ensemble comes from the library's kernels; the score is the root mean square,
over the grid, of the analysis ensemble mean minus the truth.  The twins are
built as in the paper's experiment (Section 4): members and truth are
independent random perturbations of one state, so the truth is exchangeable
with the members.  The plain filter estimates the covariance spectrum by
eq. (2), the learned one by the perceptron, and the exact-covariance filter
uses the generating spectrum itself: the reference the two estimates are
measured against (for finite N it is close to, not exactly, the best gain for
the mean, whose error spectrum is lambda (1 + 1/N)).
"""

from __future__ import annotations

import os
from typing import Iterable, Optional

import numpy as np
import torch

from . import _lib, twin

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "spectral_mlp_n5.npz")


def load_weights(path: Optional[str] = None) -> dict:
    """The trained perceptron (float32 arrays W1 .. b4) and its training record."""
    d = np.load(path or WEIGHTS)
    w = {k: d[k] for k in _lib.MLP_SHAPES}
    w["meta"] = str(d["meta"]) if "meta" in d.files else ""
    return w


def mean_rmse(ens: torch.Tensor, truth: torch.Tensor) -> float:
    return float(torch.sqrt(torch.mean((ens.double().mean(dim=0) - truth.double()) ** 2)))


def rmse_case(tw: twin.Twin, weights_dev: dict, device="cuda:0") -> dict:
    """RMSE of the forecast and of the three analyses for one twin."""
    ens = torch.from_numpy(tw.ens).to(device)
    data = torch.from_numpy(tw.data).to(device)
    truth = torch.from_numpy(tw.truth).to(device)
    R = torch.from_numpy(np.ascontiguousarray(tw.R_spec)).to(device)
    nh = tw.ens.shape[2] // 2 + 1
    lam = torch.from_numpy(np.ascontiguousarray(tw.lam[:, :nh]).astype(tw.ens.dtype)).to(device)
    plain = _lib.analyze(ens, data, R, tw.seed)
    learned = _lib.analyze_learned(ens, data, R, tw.seed, weights_dev)
    known = _lib.analyze_spectrum(ens, data, R, tw.seed, lam)
    torch.cuda.synchronize(device)
    return dict(forecast=mean_rmse(ens, truth), plain=mean_rmse(plain, truth), learned=mean_rmse(learned, truth),
                known=mean_rmse(known, truth))


def rmse_study(seeds: Iterable[int], a_values: Iterable[float], *, size: int = 2048, members: int = 5,
               r: float = 0.05, weights: Optional[dict] = None, about: str = "centre", workers: int = 8,
               device="cuda:0") -> list:
    """rmse_case over held-out twins with spectrum |k|^-a, one per (seed, a).

    about="centre": truth and members are independent perturbations of one
    state (the paper's experiment); about="truth": the members are the truth
    plus independent draws (the twin of the throughput workloads).  The twins
    are generated on the host (numpy, SeedSequence; never the perceptron's
    training generator) by a pool of threads, a few ahead of the GPU."""
    import concurrent.futures as cf

    w = weights or load_weights()
    wd = _lib.mlp_weights(w, device)
    cases = [(seed, a) for seed in seeds for a in a_values]

    def make(case):
        seed, a = case
        return twin.make_twin(size, size, members, seed=seed, dtype=np.float32, kind="power", kw={"a": a}, r=r,
                              about=about)

    rows = []
    with cf.ThreadPoolExecutor(max(1, workers)) as ex:
        for k0 in range(0, len(cases), workers):
            chunk = cases[k0:k0 + workers]
            for (seed, a), tw in zip(chunk, ex.map(make, chunk)):
                rows.append(dict(seed=seed, a=a, **rmse_case(tw, wd, device)))
    return rows


def paired_summary(rows: list, test: str = "learned", ref: str = "plain") -> dict:
    """The paired comparison of two filters over the cases: wins of `test`,
    and the mean and standard error of the difference test - ref (absolute,
    and relative to ref)."""
    d = np.array([r[test] - r[ref] for r in rows], dtype=np.float64)
    rel = np.array([(r[test] - r[ref]) / r[ref] for r in rows], dtype=np.float64)
    n = len(d)
    se = (lambda x: float(x.std(ddof=1) / np.sqrt(n)) if n > 1 else float("nan"))
    return {"cases": n, "wins": int((d < 0).sum()), "mean_diff": float(d.mean()), "se_diff": se(d),
            "mean_rel_diff": float(rel.mean()), "se_rel_diff": se(rel)}
