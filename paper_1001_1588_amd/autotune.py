"""Autotuner of the tile schedule: for each grid, the split ny = R * L of the y
transform between sweeps 1/3 (R rows per tile) and sweep 2 (length-L column
transforms).

Each compiled choice of R (fftenkf_tile_rows_options) is timed on the device
with HIP events around whole analyses of a synthetic ensemble of the given
size; the fastest is set in the library (fftenkf_set_tile_rows) and can be
saved as JSON and applied again in a later process.

    python -m paper_1001_1588_amd.autotune --grids 64 128 256 512 1024 --members 16 --out tuning.json
"""

from __future__ import annotations

import argparse
import json
from typing import Iterable, Optional

import torch

from . import _lib

DTYPES = {"float32": torch.float32, "float64": torch.float64}


def key(ny: int, nx: int, dtype: torch.dtype) -> str:
    return f"{ny}x{nx}:{'float32' if dtype == torch.float32 else 'float64'}"


def pick(timings: dict) -> int:
    """The fastest choice; ties go to the smaller R (fewer registers per tile)."""
    return min(timings, key=lambda r: (timings[r], r))


def time_choice(ny: int, nx: int, N: int, dtype: torch.dtype, rows: int, reps: int, device) -> float:
    """Median milliseconds of one analysis with R = rows."""
    _lib.set_tile_rows(ny, nx, dtype, rows)
    g = torch.Generator(device=device).manual_seed(ny * 7919 + nx)
    ens = torch.randn((N, ny, nx), generator=g, device=device, dtype=dtype)
    data = torch.randn((ny, nx), generator=g, device=device, dtype=dtype)
    ws = torch.empty(_lib.workspace_bytes(N, ny, nx, dtype), dtype=torch.uint8, device=device)
    out = torch.empty_like(ens)
    for _ in range(2):
        _lib.analyze(ens, data, 0.01, 1, out=out, workspace=ws)
    ts = []
    for r in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        _lib.analyze(ens, data, 0.01, r, out=out, workspace=ws)
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def tune(grids: Iterable, N: int, dtype: torch.dtype = torch.float32, reps: int = 9, device="cuda:0") -> dict:
    """Time every compiled R for each (ny, nx) and set the fastest; returns
    {key: {"rows": R, "ms": {R: ms}}}."""
    result = {}
    for ny, nx in grids:
        options = _lib.tile_rows_options(ny, nx, dtype)
        timings = {r: time_choice(ny, nx, N, dtype, r, reps, device) for r in options}
        best = pick(timings)
        _lib.set_tile_rows(ny, nx, dtype, best)
        result[key(ny, nx, dtype)] = {"rows": best, "ms": {str(r): t for r, t in timings.items()}, "members": N}
    return result


def apply(table: dict) -> None:
    """Set the tile rows recorded in a table from tune() (or its JSON)."""
    for k, rec in table.items():
        grid, dt = k.split(":")
        ny, nx = (int(v) for v in grid.split("x"))
        _lib.set_tile_rows(ny, nx, DTYPES[dt], int(rec["rows"]))


def load(path: str) -> dict:
    with open(path) as f:
        table = json.load(f)
    apply(table)
    return table


def main(argv: Optional[list] = None) -> None:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--grids", type=int, nargs="+", default=[64, 128, 256, 512, 1024], help="square sides")
    ap.add_argument("--members", type=int, default=16)
    ap.add_argument("--dtype", choices=sorted(DTYPES), default="float32")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    table = tune([(g, g) for g in args.grids], args.members, DTYPES[args.dtype])
    print(json.dumps(table, indent=1))
    if args.out:
        with open(args.out, "w") as f:
            json.dump(table, f, indent=1)


if __name__ == "__main__":
    main()
