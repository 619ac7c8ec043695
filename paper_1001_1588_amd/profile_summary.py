"""Summarise rocprofv3 runs of bench.py into per-kernel times and HBM traffic.

Input: one directory holding three rocprofv3 outputs of bench.py,
  trace/  (--kernel-trace --stats, csv)   per-dispatch durations
  fetch/  (--pmc FETCH_SIZE, csv)         KiB fetched from HBM per dispatch
  write/  (--pmc WRITE_SIZE, csv)         KiB written to HBM per dispatch
Kernels are keyed by name and grid size (one kernel serves several workloads);
only the library's kernels and the copy reference are kept.
Each byte counter is scaled by what it reads for bench.py's plain device copy
of known size (the `__amd_rocclr_copyBuffer` dispatch, 2 x copy-mib MiB moved):
the scale turns counter units into bytes.  Writes a JSON record (bench.py reads
it for the `traffic` field, and ignores entries whose kernel sources changed)
and prints a Markdown table.

    python -m paper_1001_1588_amd.profile_summary DIR --copy-mib 1024 --json profiles/kernels_traffic.json
"""

from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = "paper_1001_1588_amd/csrc/"
COMMON = [CSRC + "fft_core.hpp", CSRC + "kernels.hpp"]
SOURCES = {
    "k1_forward": COMMON + [CSRC + "k1_forward.hpp"],
    "k2_spectral": COMMON + [CSRC + "philox.hpp", CSRC + "spectral_unit.hpp", CSRC + "wave_fft.hpp",
                             CSRC + "k2_spectral.hpp"],
    "k3_inverse": COMMON + [CSRC + "k1_forward.hpp", CSRC + "k3_inverse.hpp"],
    "k10_observed": COMMON + [CSRC + "philox.hpp", CSRC + "spectral_unit.hpp", CSRC + "wave_fft.hpp",
                              CSRC + "k2_spectral.hpp", CSRC + "k10_observed.hpp"],
    "k7_spectral_mlp": [CSRC + "kernels.hpp", CSRC + "k7_spectral_mlp.hip"],
    "dst_": [CSRC + "fft_core.hpp", CSRC + "kernels.hpp", CSRC + "philox.hpp", CSRC + "k9_dst.hip"],
    "k11_dst_fused": COMMON + [CSRC + "philox.hpp", CSRC + "spectral_unit.hpp", CSRC + "wave_fft.hpp",
                               CSRC + "k2_spectral.hpp", CSRC + "k11_dst_fused.hpp"],
}
COPY = "__amd_rocclr_copyBuffer"


def family(name: str):
    for f in SOURCES:
        if f in name:
            return f
    return None


def sources_hash(files) -> str:
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def short(name: str) -> str:
    return name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "").strip()


def read_csv(pattern: str):
    rows = []
    for f in sorted(glob.glob(pattern)):
        rows.extend(csv.DictReader(open(f)))
    return rows


def summarise(base: str, copy_mib: int) -> dict:
    durs = collections.defaultdict(list)
    for r in read_csv(os.path.join(base, "trace", "*kernel_trace.csv")):
        # total threads, as the counter records give it
        grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"]) if "Grid_Size_X" in r \
            else int(r["Grid_Size"])
        durs[(short(r["Kernel_Name"]), grid)].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    counters = {}
    copy_max = {}
    for kind, counter in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE")):
        vals = collections.defaultdict(list)
        for r in read_csv(os.path.join(base, kind, "*counter_collection.csv")):
            if r["Counter_Name"] != counter:
                continue
            vals[(short(r["Kernel_Name"]), int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
        counters[kind] = {k: sum(v) / len(v) for k, v in vals.items()}
        # the largest copy dispatch is bench.py's reference copy: it reads copy_mib
        # MiB and writes copy_mib MiB (other copies of the same kernel are small)
        copy_max[kind] = max((max(v) for (n, _), v in vals.items() if n == COPY), default=None)
    copy_bytes = 2 * (copy_mib << 20)
    scale = {kind: ((copy_bytes / 2) / copy_max[kind] if copy_max[kind] else None) for kind in ("fetch", "write")}
    kernels = []
    for (name, grid), d in sorted(durs.items(), key=lambda kv: -sum(kv[1])):
        if not (name.startswith("fftenkf::") or name == COPY):
            continue  # the benchmark's own torch and rocFFT kernels (input generation)
        fam = family(name)
        rec = {"name": name, "grid": grid, "calls": len(d), "avg_ns": sum(d) / len(d),
               "min_ns": min(d), "max_ns": max(d)}
        for kind in ("fetch", "write"):
            v = counters[kind].get((name, grid))
            rec[kind + "_kib"] = v
            rec[kind + "_bytes"] = v * scale[kind] if (v is not None and scale[kind]) else None
        if fam is not None:
            rec["sources"] = SOURCES[fam]
            rec["sources_sha256_16"] = sources_hash(SOURCES[fam])
        kernels.append(rec)
    return {"copy_mib": copy_mib, "copy_scale": scale, "kernels": kernels}


def markdown(summary: dict) -> str:
    lines = ["| Kernel | Grid | Calls | Avg (us) | Min (us) | Max (us) | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | "
             "Traffic (MB) |", "|---|---|---|---|---|---|---|---|---|"]
    for k in summary["kernels"]:
        fb, wb = k.get("fetch_bytes"), k.get("write_bytes")
        traffic = f"{(fb + wb) / 1e6:.1f}" if fb is not None and wb is not None else "-"
        fk = f"{k['fetch_kib']:.0f}" if k.get("fetch_kib") is not None else "-"
        wk = f"{k['write_kib']:.0f}" if k.get("write_kib") is not None else "-"
        lines.append(f"| `{k['name']}` | {k['grid']} | {k['calls']} | {k['avg_ns'] / 1e3:.1f} | "
                     f"{k['min_ns'] / 1e3:.1f} | {k['max_ns'] / 1e3:.1f} | {fk} | {wk} | {traffic} |")
    return "\n".join(lines)


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("base")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--json", default=None)
    args = ap.parse_args(argv)
    s = summarise(args.base, args.copy_mib)
    if args.json:
        with open(args.json, "w") as f:
            json.dump(s, f, indent=1)
    print(f"counter scale (bytes per counter unit): fetch {s['copy_scale']['fetch']}, write {s['copy_scale']['write']}")
    print(markdown(s))


if __name__ == "__main__":
    main()
