"""Hardware-counter helpers for the roofline's HBM traffic figure.

``python -m paper_1711_02384_amd.pmc copy [--mib N] [--reps R]``
    A plain device-to-device copy of N MiB, R times: the calibration kernel.
    Run it under ``rocprofv3 --pmc FETCH_SIZE`` (then ``WRITE_SIZE``); the
    counter per dispatch divided by the N MiB actually read (written) is the
    counter's scale factor on this GPU.

``python -m paper_1711_02384_amd.pmc smear --kind prop|noise [--L 32] [--iters 50]``
    The smearing kernel alone on a random 32^3 propagator slice (48 colour
    vectors per site) or 50 random noise vectors (200 per site), ``iters``
    launches timed with HIP events; prints microseconds per launch and the
    algorithmic bytes (field read and written once, 216 B of links per site).

``python -m paper_1711_02384_amd.pmc summary DIR [--kernel SUBSTR] [--bytes B]``
    Summarise every ``*counter_collection.csv`` and ``*kernel_stats.csv`` under
    DIR (rocprofv3 output): per kernel, the mean of each counter per dispatch
    and the mean duration; with --bytes, the ratio of a counter (KiB) to B
    bytes per dispatch.
"""
from __future__ import annotations

import argparse
import csv
import glob
import os
import sys
from collections import defaultdict


def copy_main(mib: float, reps: int) -> None:
    import torch
    n = int(mib * (1 << 20))
    src = torch.empty(n, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {n} bytes x {reps}", flush=True)


def smear_main(kind: str, L: int, iters: int) -> None:
    import torch
    import paper_1711_02384_amd as c3pt
    V3 = L ** 3
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(5)
    U = torch.randn((4, 3, 3, V3), dtype=torch.complex64, device=dev, generator=g)
    geom = c3pt.Geom((L, L, L), 2 * L)
    if kind == "prop":
        f = torch.randn((12, 12, V3), dtype=torch.complex64, device=dev, generator=g)
        run = lambda: c3pt.smear_propagator(f, U, geom, 0.25, iters, out=f)
        alg = 144 * V3 * 8 * 2 + 216 * V3
    else:
        f = torch.randn((50, 12, V3), dtype=torch.complex64, device=dev, generator=g)
        run = lambda: c3pt.smear_vectors(f, U, geom, 0.25, iters, out=f)
        alg = 600 * V3 * 8 * 2 + 216 * V3
    run()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    run()
    b.record()
    torch.cuda.synchronize()
    us = a.elapsed_time(b) * 1e3 / iters
    print(f"smear {kind} {L}^3: {us:.1f} us per launch, algorithmic {alg / 1e6:.1f} MB, "
          f"{alg / us / 1e3:.0f} GB/s", flush=True)


def _rows(path):
    with open(path, newline="") as f:
        yield from csv.DictReader(f)


def summary(d: str, kernel: str | None = None):
    """{kernel: {"dispatches": n, counter: mean per dispatch, "avg_ns": mean duration}}."""
    per = defaultdict(lambda: defaultdict(float))         # (kernel, dispatch) -> counter -> value
    for p in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in _rows(p):
            name = r.get("Kernel_Name", "")
            if kernel and kernel not in name:
                continue
            per[(name, r.get("Dispatch_Id") or r.get("Correlation_Id"))][r["Counter_Name"]] += float(r["Counter_Value"])
    out = defaultdict(lambda: defaultdict(float))
    count = defaultdict(int)
    for (name, _), ctrs in per.items():
        count[name] += 1
        for c, v in ctrs.items():
            out[name][c] += v
    res = {}
    for name, ctrs in out.items():
        res[name] = {"dispatches": count[name]}
        for c, v in ctrs.items():
            res[name][c] = v / count[name]
    for p in glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True):
        for r in _rows(p):
            name = r.get("Name", "")
            if kernel and kernel not in name:
                continue
            res.setdefault(name, {})
            res[name]["avg_ns"] = float(r.get("AverageNs", "nan"))
            res[name]["calls"] = int(float(r.get("Calls", "0")))
    return res


def main(argv=None) -> None:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=float, default=1024.0)
    c.add_argument("--reps", type=int, default=5)
    m = sub.add_parser("smear")
    m.add_argument("--kind", choices=["prop", "noise"], default="prop")
    m.add_argument("--L", type=int, default=32)
    m.add_argument("--iters", type=int, default=50)
    s = sub.add_parser("summary")
    s.add_argument("dir")
    s.add_argument("--kernel", default=None)
    s.add_argument("--bytes", type=float, default=None, help="reference bytes per dispatch")
    a = ap.parse_args(argv)
    if a.cmd == "copy":
        copy_main(a.mib, a.reps)
        return
    if a.cmd == "smear":
        smear_main(a.kind, a.L, a.iters)
        return
    res = summary(a.dir, a.kernel)
    for name, d in sorted(res.items(), key=lambda kv: -kv[1].get("avg_ns", 0.0)):
        short = name if len(name) < 110 else name[:107] + "..."
        parts = [f"{k}={v:.6g}" for k, v in sorted(d.items())]
        if a.bytes:
            for k in ("FETCH_SIZE", "WRITE_SIZE"):
                if k in d:
                    parts.append(f"{k}_KiB/ref={d[k] * 1024.0 / a.bytes:.4f}")
        print(f"{short}\n    " + "  ".join(parts))
    sys.stdout.flush()


if __name__ == "__main__":
    main()
