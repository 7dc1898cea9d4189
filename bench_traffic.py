#!/usr/bin/env python3
"""HBM traffic of the step kernel from two rocprofv3 counter runs of bench.py.

Reads the `run_counter_collection.csv` files of a `--pmc FETCH_SIZE` run and
a `--pmc WRITE_SIZE` run (both of `bench.py ... --copy-mb M`), takes the mean
KiB per dispatch of `step_kernel`, and scales each counter by what it reads
for the plain device copy of M MiB that bench.py runs after its timed region
(expected: M MiB fetched and M MiB written).  Writes a short markdown summary
whose `- key: value` lines bench.py reads back; bench.py reports the figure
only while the kernel sources hash to the value recorded here.

    python3 bench_traffic.py --fetch DIR --write DIR --copy-mb 1024 \\
        --envs 4096 --bodies 15 --substeps 120 --command "..." --out FILE
"""
from __future__ import annotations

import argparse
import csv
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from bench import hbm_bytes_per_call, kernel_source_hash  # noqa: E402


def per_dispatch(path: str, counter: str) -> dict:
    """{kernel name: [KiB per dispatch, ...]} for one counter."""
    out: dict = {}
    with open(os.path.join(path, "run_counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def pick(d: dict, needle: str) -> list:
    vals = [v for k, vs in d.items() if needle in k for v in vs]
    if not vals:
        raise SystemExit(f"no dispatch of a kernel named like {needle!r}")
    return vals


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-mb", type=int, required=True)
    ap.add_argument("--envs", type=int, required=True)
    ap.add_argument("--bodies", type=int, required=True)
    ap.add_argument("--substeps", type=int, required=True)
    ap.add_argument("--command", required=True, help="the rocprofv3 commands that made the two runs")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()

    fetch = per_dispatch(a.fetch, "FETCH_SIZE")
    write = per_dispatch(a.write, "WRITE_SIZE")
    step_f = pick(fetch, "step_kernel")
    step_w = pick(write, "step_kernel")
    copy_kib = a.copy_mb * 1024.0
    # the copy of M MiB is the largest copy dispatch of the run
    copy_f = max(pick(fetch, "copyBuffer"))
    copy_w = max(pick(write, "copyBuffer"))
    sf, sw = copy_kib / copy_f, copy_kib / copy_w
    mf, mw = sum(step_f) / len(step_f), sum(step_w) / len(step_w)
    traffic = (mf * sf + mw * sw) * 1024.0
    algo = hbm_bytes_per_call(a.envs * a.bodies, a.envs)

    lines = [
        f"# step_kernel HBM traffic, {a.envs} envs x {a.bodies} cuboids, {a.substeps} substeps",
        "",
        "Commands (from the repository root, on one MI355X):",
        "",
        "```",
        a.command,
        "```",
        "",
        "| counter | step_kernel KiB/dispatch (mean of %d) | copy of %d MiB reads | scale | scaled KiB |" % (len(step_f), a.copy_mb),
        "|---|---|---|---|---|",
        f"| FETCH_SIZE | {mf:.1f} | {copy_f:.1f} | {sf:.4f} | {mf * sf:.1f} |",
        f"| WRITE_SIZE | {mw:.1f} | {copy_w:.1f} | {sw:.4f} | {mw * sw:.1f} |",
        "",
        f"Algorithmic bytes per launch: {algo:.0f} (136 B per body + 28 B per env).",
        f"Measured bytes per launch: {traffic:.0f} ({traffic / algo:.2f} x algorithmic).",
        "",
        f"- kernel_source_sha256: {kernel_source_hash()}",
        f"- envs: {a.envs}",
        f"- bodies_per_env: {a.bodies}",
        f"- substeps: {a.substeps}",
        f"- bytes_per_launch: {traffic:.0f}",
        "",
    ]
    with open(a.out, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))
    return 0


if __name__ == "__main__":
    sys.exit(main())
