"""Autotuner for the tile shapes of the fused contraction + projection kernels.

For every (kind, mode, momentum-tile class) that a workload uses, each
compiled variant is timed on the caller's own inputs (HIP events on the
current stream, after one warm-up call) and the fastest is selected in the
library.  Results can be saved as a JSON table and applied later with
``paper_1711_02384_amd.apply_tuning`` (the package applies
``tuning_mi355x.json`` at import when it exists, or the file named by the
environment variable C3PT_TUNING).
"""
from __future__ import annotations

import json
import time
from typing import Callable, Dict, List

import torch

from . import KIND, MODE, get_variant, set_variant, variant_count


def time_call(fn: Callable[[], object], reps: int = 3) -> float:
    """Median milliseconds of fn() on the current stream (after one warm-up)."""
    fn()
    st = torch.cuda.current_stream()
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        fn()
        b.record(st)
        b.synchronize()
        times.append(a.elapsed_time(b))
    times.sort()
    return times[len(times) // 2]


def tune(cases: List[dict], reps: int = 3, log=print) -> dict:
    """cases: [{"kind": name or id, "mode": name or id, "mt_class": c, "call": fn}, ...].

    Returns a table {"entries": [...], "device": ..., "when": ...} and leaves the
    fastest variant selected for each key."""
    entries = []
    for c in cases:
        kind = KIND.get(c["kind"], c["kind"])
        mode = MODE.get(c["mode"], c["mode"])
        cls = int(c["mt_class"])
        n = variant_count(kind, mode, cls)
        if n == 0:
            continue
        before = get_variant(kind, mode, cls)
        ms = []
        for v in range(n):
            set_variant(kind, mode, cls, v)
            ms.append(time_call(c["call"], reps))
        best = min(range(n), key=lambda v: ms[v])
        set_variant(kind, mode, cls, best)
        entries.append({"kind": kind, "mode": mode, "mt_class": cls, "variant": best,
                        "ms": [round(x, 4) for x in ms], "previous": before})
        if log:
            log(f"[autotune] kind={kind} mode={mode} class={cls}: ms={['%.3f' % x for x in ms]} -> variant {best}")
    return {"device": torch.cuda.get_device_name(0), "when": time.strftime("%Y-%m-%d %H:%M:%S"),
            "entries": entries}


def save(table: dict, path: str) -> None:
    with open(path, "w") as f:
        json.dump(table, f, indent=1)


def tune_recorded(kinds: List, mode, cls: int, record: Callable[[], object], run: Callable[[], object],
                  reps: int = 3, log=print) -> dict:
    """Tune variants that are fixed when work is recorded (batches: read by
    c3pt_batch_create).  For each kind in turn (the others at their current
    choice), every variant is selected, the work is recorded again with
    record() and its replay run() timed; the fastest stays selected and the
    work is left recorded with it."""
    mode = MODE.get(mode, mode)
    entries = []
    for kn in kinds:
        kind = KIND.get(kn, kn)
        n = variant_count(kind, mode, cls)
        if n == 0:
            continue
        before = get_variant(kind, mode, cls)
        ms = []
        for v in range(n):
            set_variant(kind, mode, cls, v)
            record()
            ms.append(time_call(run, reps))
        best = min(range(n), key=lambda v: ms[v])
        set_variant(kind, mode, cls, best)
        entries.append({"kind": kind, "mode": mode, "mt_class": cls, "variant": best,
                        "ms": [round(x, 4) for x in ms], "previous": before})
        if log:
            log(f"[autotune] recorded kind={kind} mode={mode} class={cls}: ms={['%.3f' % x for x in ms]} "
                f"-> variant {best}")
    record()
    return {"device": torch.cuda.get_device_name(0), "when": time.strftime("%Y-%m-%d %H:%M:%S"),
            "entries": entries}
