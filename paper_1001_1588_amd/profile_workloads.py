"""Per-workload rocprofv3 summaries (profiles/*.md) from profile_summary's JSON.

Each summary lists, for one benchmark leg, the kernels it launches with their
trace times, counter bytes (FETCH_SIZE and WRITE_SIZE scaled by the copy
reference), the algorithmic bytes of each launch (its inputs read once and its
outputs written once) and their ratio, plus the commands that produced the data.

    python -m paper_1001_1588_amd.profile_workloads profiles/kernels_traffic.json bench.json profiles
"""

from __future__ import annotations

import argparse
import json
import os


def write(s: dict, bj: dict, outdir: str) -> None:
    """s: profile_summary's record; bj: one bench.py JSON line of the same machine."""
    K = {(k['name'], k['grid']): k for k in s['kernels']}
    def get(name, grid):
        return K[(name, grid)]

    def first(*cands):
        # the tile schedule (rows per tile) decides which instantiation ran
        for c in cands:
            if c in K:
                return c
        raise KeyError(cands)
    def row(name, grid, alg):
        k = get(name, grid)
        fb, wb = k.get('fetch_bytes'), k.get('write_bytes')
        t = (fb + wb) if fb is not None and wb is not None else None
        ratio = f"{t/alg:.3f}" if (alg and t) else "-"
        algs = f"{alg/1e6:.1f}" if alg else "-"
        gbs = f"{alg/(k['avg_ns']*1e-9)/1e9:.0f}" if alg else "-"
        fk = f"{k['fetch_kib']:.0f}" if k.get('fetch_kib') is not None else "-"
        wk = f"{k['write_kib']:.0f}" if k.get('write_kib') is not None else "-"
        ts = f"{t/1e6:.1f}" if t else "-"
        return f"| `{name}` | {grid} | {k['calls']} | {k['avg_ns']/1e3:.1f} | {k['min_ns']/1e3:.1f} | {k['max_ns']/1e3:.1f} | {fk} | {wk} | {ts} | {algs} | {ratio} | {gbs} |"
    hdr = "| Kernel | Grid (threads) | Calls | Avg (us) | Min (us) | Max (us) | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | Scaled traffic (MB) | Algorithmic (MB) | Ratio | Algorithmic GB/s |\n|---|---|---|---|---|---|---|---|---|---|---|---|"
    cp = get('__amd_rocclr_copyBuffer', 131072)
    copy_live = bj['copy_ceiling']['GBps'] / 1e3
    cmds = f'''## Commands (run from /tmp with TMPDIR=/tmp; R = repository root, O = output folder)

```
rocprofv3 --kernel-trace --stats -d O/trace -o run --output-format csv -- python3 R/bench.py --steps 20 --warmup 3 --cpu-members 0 --learned-steps 10 --rmse-seeds 1 --multi-steps 10 --batch-steps 5 --dst-steps 10
rocprofv3 --pmc FETCH_SIZE -d O/fetch -o run --output-format csv -- python3 R/bench.py --steps 2 --warmup 1 --cpu-members 0 --learned-steps 2 --rmse-seeds 1 --multi-steps 2 --batch-steps 2 --dst-steps 2
rocprofv3 --pmc WRITE_SIZE -d O/write -o run --output-format csv -- python3 R/bench.py --steps 2 --warmup 1 --cpu-members 0 --learned-steps 2 --rmse-seeds 1 --multi-steps 2 --batch-steps 2 --dst-steps 2
python -m paper_1001_1588_amd.profile_summary O --copy-mib 1024 --json R/profiles/kernels_traffic.json
python3 R/bench.py > O/bench.json
python -m paper_1001_1588_amd.profile_workloads R/profiles/kernels_traffic.json O/bench.json R/profiles
```

Counters are KiB per dispatch.  On bench.py's plain 1 GiB device copy (the largest `__amd_rocclr_copyBuffer` dispatch) FETCH_SIZE and WRITE_SIZE read {(1<<30)/s['copy_scale']['fetch']:.0f} and {(1<<30)/s['copy_scale']['write']:.0f} for 1 GiB read and 1 GiB written, so fetches are scaled by {s['copy_scale']['fetch']:.1f} bytes per counter unit and writes by {s['copy_scale']['write']:.0f}.  Algorithmic bytes are each launch's inputs read once plus its outputs written once.  Rows are keyed by kernel and total threads (one kernel serves several workloads).
'''
    n = 2048*2048; h = 2048*1025*8; r4 = 2048*1025*4
    K1, K2, K3 = ('fftenkf::k1_forward<float, 2048, 16, 4, false>', 688128), ('fftenkf::k2_spectral<float, 128, 20, 0>', 524288), ('fftenkf::k3_inverse<float, 2048, 16, 4, false>', 655360)
    tr = [get(*k) for k in (K1, K2, K3)]
    tb = sum(k['fetch_bytes'] + k['write_bytes'] for k in tr); tt = sum(k['avg_ns'] for k in tr)
    out = {}
    out['plain2048_n20_sweeps.md'] = f'''# rocprofv3 summary: the three sweeps on the 2048x2048, N=20, float32 workload

Workload: periodic 2048x2048 grid, N = 20 members, float32, spectrum |k|^-3, R = 0.05 I passed as an R_spec array (bench.py's main leg).  One MI355X (gfx950).

{cmds}
## Kernels (3 warm-up + 20 timed calls)

{hdr}
{row(*K1, 21*n*4 + 21*h)}
{row(*K2, 21*h + r4 + 20*h)}
{row(*K3, 20*h + 20*n*4)}

Three-sweep HBM rate on measured bytes: {' + '.join(f"{(k['fetch_bytes']+k['write_bytes'])/1e6:.1f}" for k in tr)} MB over {' + '.join(f"{k['avg_ns']/1e3:.1f}" for k in tr)} us = {tb/(tt*1e-9)/1e12:.2f} TB/s, {tb/(tt*1e-9)/8e12*100:.0f}% of 8 TB/s.  bench.py's 1 GiB device copy runs at {copy_live:.2f} TB/s on the same machine without the profiler.  The spectral sweep is the dominant kernel ({tr[1]['avg_ns']/tt*100:.0f}% of the time).
'''
    h5 = 2048*1025*8
    mlp = get('fftenkf::k7_spectral_mlp', 131072)
    out['learned2048_n5_perceptron.md'] = f'''# rocprofv3 summary: the learned-covariance analysis on 2048x2048, N=5, float32

Workload: periodic 2048x2048 grid, N = 5, float32, spectrum |k|^-3, R = 0.05 I (R_spec array), the shipped perceptron weights (bench.py's learned leg; its RMSE study adds plain and exact-covariance analyses of the same size, which share these kernels and grids).  One MI355X (gfx950).

{cmds}
## Kernels

{hdr}
{row('fftenkf::k1_forward<float, 2048, 16, 4, false>', 196608, 6*n*4 + 6*h5)}
{row('fftenkf::k2_spectral<float, 128, 8, 3>', 524288, 5*h5 + r4)}
{row('fftenkf::k7_spectral_mlp', 131072, 2048*1025*4*2)}
{row('fftenkf::k2_spectral<float, 128, 8, 1>', 524288, 6*h5 + r4 + 5*h5)}
{row('fftenkf::k3_inverse<float, 2048, 16, 4, false>', 163840, 5*h5 + 5*n*4)}

`k2_spectral<float, 128, 8, 3>` is the statistics-only pass (reads the 5 member spectra, writes c_hat; d is not read).  `k2_spectral<float, 128, 8, 1>` is the update pass with the perceptron's spectrum (the variant with a given spectrum; the RMSE study's exact-covariance analyses run it too, and its plain analyses `k2_spectral<float, 128, 8, 0>`).  The perceptron is bound by its arithmetic, not by HBM: 41.6 GFLOP per launch, {mlp['avg_ns']/1e3:.1f} us average here, {41.648e9/(mlp['avg_ns']*1e-9)/1e12:.0f} TFLOP/s of bf16 matrix work ({41.648e9/(mlp['avg_ns']*1e-9)/1e12/2500*100:.0f}% of 2.5 PFLOP/s).
'''
    n1 = 1024*1024; h1 = 1024*513*8
    out['multiblock4x1024_n10_sweeps.md'] = f'''# rocprofv3 summary: the multi-block analysis on 4 fields of 1024x1024, N=10, float32

Workload: 4 blocks of 1024x1024, N = 10, float32, spectra (1+|k|^2/L_b^2)^-2 with L_b in {{8, 16, 32, 64}}, coherence 0.6, block 0 observed with R = 0.02 I (R_spec array) (bench.py's multi-block leg).  One MI355X (gfx950).

{cmds}
## Kernels (3 warm-up + 10 timed calls)

{hdr}
{row(*first(('fftenkf::k1_forward<float, 1024, 8, 4, false>', 671744), ('fftenkf::k1_forward<float, 1024, 16, 8, false>', 335872)), 41*n1*4 + 41*h1)}
{row(*first(('fftenkf::k10_observed<float, 128, 10, 1>', 131072), ('fftenkf::k10_observed<float, 64, 10, 1>', 131072)), 41*h1 + 1024*513*4 + 40*h1)}
{row(*first(('fftenkf::k3_inverse<float, 1024, 8, 4, false>', 655360), ('fftenkf::k3_inverse<float, 1024, 16, 8, false>', 327680)), 40*h1 + 40*n1*4)}
'''
    out['sine2048_n20_sweeps.md'] = f'''# rocprofv3 summary: the analysis in the real sine basis on 2048x2048, N=20, float32

Workload: the main leg's ensemble (2048x2048, N = 20, float32, |k|^-3), R = 0.05 I, orthonormal DST-II basis (bench.py's sine-basis leg).  One MI355X (gfx950).

{cmds}
## Kernels (3 warm-up + 10 timed calls)

{hdr}
{row('fftenkf::k1_forward<float, 2048, 16, 4, true>', 688128, 21*n*4 + 21*h)}
{row('fftenkf::k11_dst_fused<float, 128, 20>', 589824, 21*h + 20*h)}
{row('fftenkf::k3_inverse<float, 2048, 16, 4, true>', 655360, 20*h + 20*n*4)}

Sweeps 1 and 3 read and write the fields through the sine reordering (`true` in their names).  `k11_dst_fused` is the whole spectral part of the sine-basis analysis (length-L transforms, eq. (2)-(3) on the sine coefficients, inverse transforms): 21 spectra in, 20 out.  Its grid is (R/2 + 1) row pairs x (nx/2)/4 column chunks of 256 threads, 12.5% more blocks than a single-block sweep because rows 0 and R/2 pair with themselves.
'''
    for name, text in out.items():
        open(os.path.join(outdir, name), 'w').write(text)
    rows = [k for k in s['kernels'] if '_batch<' in k['name']]
    graph_ms = float(bj.get('batch', {}).get('graph_ms_per_batch', float('nan')))
    lines = []; tot_us = 0; tot_b = 0
    for k in sorted(rows, key=lambda k: (k['name'], k['grid'])):
        fb, wb = k.get('fetch_bytes'), k.get('write_bytes')
        t = f"{(fb+wb)/1e6:.1f}" if fb is not None and wb is not None else "-"
        fk = f"{k['fetch_kib']:.0f}" if k.get('fetch_kib') is not None else "-"
        wk = f"{k['write_kib']:.0f}" if k.get('write_kib') is not None else "-"
        lines.append(f"| `{k['name']}` | {k['grid']} | {k['calls']} | {k['avg_ns']/1e3:.1f} | {k['min_ns']/1e3:.1f} | {k['max_ns']/1e3:.1f} | {fk} | {wk} | {t} |")
        tot_us += k['avg_ns']/1e3
        if fb is not None and wb is not None: tot_b += fb + wb
    text = f'''# rocprofv3 summary: 256 independent filters of uneven size in one captured graph

Workload: 256 filters, square sides drawn uniformly from {{64, 128, 256, 512, 1024}} (seeded: 55, 46, 49, 51 and 55 filters), N = 16, float32, spectrum (1+|k|^2)^-2, R = 0.01 I, tile rows chosen by the autotuner in each run, all launches of a batch captured in one HIP graph (bench.py's batch leg).  Up to 40 filters of one size share a launch (grid dimension y), so each size takes one or two launches per sweep.  One MI355X (gfx950).

{cmds}
## Kernels (the eager run, the capture and the timed replays of bench.py's batch leg; the autotuner's single-filter analyses are listed in kernels_traffic.json)

| Kernel | Grid (threads) | Calls | Avg (us) | Min (us) | Max (us) | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | Scaled traffic (MB) |
|---|---|---|---|---|---|---|---|---|
''' + "\n".join(lines) + f'''

Each launch chain (one grid size, up to 40 filters: sweeps 1, 2 and 3) runs on one of up to three streams forked from the caller's, so the chains overlap on the GPU and each launch's duration includes the time it shares the GPU with the others: one call of each row sums to {tot_us/1e3:.2f} ms of kernel time, against {graph_ms:.2f} ms of wall time per replayed batch (bench.py's graph_ms_per_batch in the same run).  Rows without counters (`-`) are launches whose grid differed between the counter runs and the trace run (the autotuner's choice of tile rows can differ between runs); their time is included.
'''
    open(os.path.join(outdir, 'batch256_uneven_n16.md'), 'w').write(text)


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("summary", help="profile_summary.py's JSON")
    ap.add_argument("bench", help="a bench.py JSON line from the same machine (for the copy ceiling)")
    ap.add_argument("outdir")
    args = ap.parse_args(argv)
    with open(args.summary) as f:
        s = json.load(f)
    with open(args.bench) as f:
        bj = json.loads(f.read().strip().splitlines()[-1])
    write(s, bj, args.outdir)


if __name__ == "__main__":
    main()
