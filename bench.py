#!/usr/bin/env python3
"""Throughput of the spin-open three-point hot path on one MI355X.

One step = one pass of every hot-path stage over one batch of synthetic input
shaped like the 32^3 x 64 meson workload:

* meson spectator at t_f = 16 (Eq. (9)) and a nucleon-type epsilon-tensor
  spectator at the same timeslice,
* insertion (Eq. (10)) at tau = 0..16 with the local operator (all 16 Gamma
  open) and the four one-derivative operators D_nu,
* momentum projection of every part onto the 81 momenta with |k|^2 <= 6,
* the noise-weighted combine: local operator on all 81 x 81 momentum pairs,
  derivative operators and the nucleon on the 161 pairs with p' = q or p' = 0.

Inputs: 4 Z2xZ2 noise vectors, Gaussian propagators and stochastic solutions,
Haar SU(3) links, complex64 in HBM (FP32 contractions and FP32 MFMA
projection, FP64 split-site accumulation and FP64 combine).  Prints one JSON
line.  `--gpus` above 1 is refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)

PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-baryon", action="store_true", help="meson only (drop the nucleon spectator)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-slices", type=int, default=6, help="insertion timeslices in the CPU sample")
    ap.add_argument("--proj", choices=["f32", "bf16x2", "f16x2"], default="f32",
                    help="projection arithmetic: FP32 MFMA, or hi+lo BF16 / FP16 MFMA with FP32 accumulation")
    ap.add_argument("--tune", action="store_true", help="autotune kernel variants on this workload first")
    ap.add_argument("--tune-out", default=None, help="write the tuning table (JSON) here")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def pairs_diag_or_zero(n_mom):
    """(p', q) pairs with p' = q or p' = 0 (index 0 is k = 0)."""
    pr = [(p, p) for p in range(n_mom)] + [(0, q) for q in range(1, n_mom)]
    return np.array(pr, dtype=np.int32)


class Workload:
    name = "meson+nucleon 3pt, 32^3x64, t_f=16, tau=0..16, N=4, |k|^2<=6 (81 momenta), local+4 D_nu"
    L = (32, 32, 32)
    T = 64
    t_f = 16
    N = 4
    taus = list(range(0, 17))
    n2 = 6
    n_ops = 5
    cfg = 2


def cpu_baseline(W, k, n_slices):
    """Time the FP64 oracle on a bounded sample of the same workload on the host."""
    import c3pt_synth as syn
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    L, T = W.L, W.T
    G1 = syn.round_to_c64(syn.propagator_slice(L, W.cfg, syn.FIELD_G1, W.t_f))
    eta = syn.round_to_c64(syn.z2z2_noise(L, W.N, W.cfg, W.t_f))
    taus = W.taus[len(W.taus) // 2: len(W.taus) // 2 + n_slices]
    need = sorted({t for tau in taus for t in (tau - 1, tau, tau + 1)})
    G3 = {t % T: syn.round_to_c64(syn.propagator_slice(L, W.cfg, syn.FIELD_G3, t % T)) for t in need}
    s = {t: syn.round_to_c64(syn.solution_slice(L, W.N, W.cfg, t)) for t in taus}
    U = {t % T: syn.round_to_c64(syn.link_slice(L, W.cfg, t % T)) for t in sorted({t - 1 for t in taus} | set(taus))}
    t0 = time.perf_counter()
    oracle.spectator_meson(G1, eta, L, k)
    oracle.insertion(G3, s, taus, L, T, k, U_t=U, n_ops=W.n_ops)
    dt = time.perf_counter() - t0
    V3 = int(np.prod(L))
    units = W.N * V3 * len(k) * (1 + len(taus))
    return {"value": units / dt, "unit": "site*momenta/s", "cores": int(threads), "kind": "oracle",
            "sample": f"FP64 numpy oracle: meson spectator + insertion (5 ops) on {len(taus)} of 17 "
                      f"timeslices, full 32^3 slices, N=4, 81 momenta; {units:.3g} units in {dt:.1f} s; "
                      f"nucleon spectator and combine not in the sample",
            "seconds": dt}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import c3pt_synth as syn
    import paper_1711_02384_amd as c3pt

    W = Workload()
    baryon = not args.no_baryon
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    L, T = W.L, W.T
    V3 = int(np.prod(L))
    k = c3pt.momentum_list(W.n2)
    n_mom = len(k)

    def up(a):
        return torch.from_numpy(np.ascontiguousarray(a.astype(np.complex64))).to(dev)

    log(f"[bench] generating inputs for {W.name}")
    t0 = time.perf_counter()
    G1 = up(syn.propagator_slice(L, W.cfg, syn.FIELD_G1, W.t_f))
    eta = up(syn.z2z2_noise(L, W.N, W.cfg, W.t_f))
    g_slices = sorted({t % T for tau in W.taus for t in (tau - 1, tau, tau + 1)})
    u_slices = sorted({t % T for tau in W.taus for t in (tau - 1, tau)})
    G3 = {t: up(syn.propagator_slice(L, W.cfg, syn.FIELD_G3, t)) for t in g_slices}
    s = {t: up(syn.solution_slice(L, W.N, W.cfg, t)) for t in W.taus}
    U = {t: up(syn.link_slice(L, W.cfg, t)) for t in u_slices}
    torch.cuda.synchronize()
    log(f"[bench] inputs resident in HBM ({time.perf_counter() - t0:.1f} s)")

    proj_flag = {"f32": c3pt.PROJ_NATIVE, "bf16x2": c3pt.PROJ_SPLIT_BF16, "f16x2": c3pt.PROJ_SPLIT_F16}[args.proj]
    mode = {"f32": 1, "bf16x2": 2, "f16x2": 3}[args.proj]
    geom = c3pt.Geom(L, T, proj=proj_flag)
    n_tau = len(W.taus)
    S = torch.empty((W.N, n_mom, 192), dtype=torch.complex128, device=dev)
    SB = torch.empty((W.N, n_mom, 3072), dtype=torch.complex128, device=dev)
    I = torch.empty((W.N, n_tau, W.n_ops, n_mom, 192), dtype=torch.complex128, device=dev)
    pairs = pairs_diag_or_zero(n_mom)
    C_loc = torch.empty((n_mom * n_mom, n_tau, 1, 64, 64), dtype=torch.complex128, device=dev)
    C_der = torch.empty((len(pairs), n_tau, W.n_ops - 1, 64, 64), dtype=torch.complex128, device=dev)
    C_bar = torch.empty((len(pairs), n_tau, 1, 1024, 64), dtype=torch.complex128, device=dev) if baryon else None

    def step():
        c3pt.spectator_meson(G1, eta, k, geom, out=S)
        if baryon:
            c3pt.spectator_baryon(G1, G1, eta, k, geom, out=SB)
        c3pt.insertion(G3, s, W.taus, k, geom, U_t=U, n_ops=W.n_ops, out=I)
        c3pt.combine(S, I, op_begin=0, op_end=1, out=C_loc)
        c3pt.combine(S, I, pairs=pairs, op_begin=1, op_end=W.n_ops, out=C_der)
        if baryon:
            c3pt.combine(SB, I, pairs=pairs, op_begin=0, op_end=1, out=C_bar)

    tuning = None
    if args.tune:
        from paper_1711_02384_amd import autotune
        cls = c3pt.mt_class(n_mom)
        cases = [{"kind": "insertion", "mode": mode, "mt_class": cls,
                  "call": lambda: c3pt.insertion(G3, s, W.taus, k, geom, U_t=U, n_ops=W.n_ops, out=I)},
                 {"kind": "spectator_meson", "mode": mode, "mt_class": cls,
                  "call": lambda: c3pt.spectator_meson(G1, eta, k, geom, out=S)}]
        if baryon:
            cases.append({"kind": "spectator_baryon", "mode": mode, "mt_class": cls,
                          "call": lambda: c3pt.spectator_baryon(G1, G1, eta, k, geom, out=SB)})
        tuning = autotune.tune(cases, reps=3, log=log)
        if args.tune_out:
            autotune.save(tuning, args.tune_out)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    c3pt.profile_read(reset=True)
    c3pt.profile_enable(True)
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        step()
        b.record(stream)
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    c3pt.profile_enable(False)
    prof = c3pt.profile_read(reset=True)
    lat = sorted(a.elapsed_time(b) for a, b in evs)
    ms_per_step = (t_end - t_start) * 1e3 / args.steps

    units_spec = W.N * V3 * n_mom * (2 if baryon else 1)
    units_ins = W.N * n_tau * V3 * n_mom
    units = units_spec + units_ins
    value = units / (ms_per_step * 1e-3)

    # Dominant kernel: the fused insertion contraction + projection.
    peak = PEAK_FP32_MFMA_TFLOPS if args.proj == "f32" else PEAK_BF16_MFMA_TFLOPS
    ins_cols = W.N * n_tau * W.n_ops * 192
    flops_ins = 8.0 * n_mom * V3 * ins_cols                  # complex GEMM flops, useful rows only
    pi = prof.get("proj_insertion", {})
    ins_ms = pi.get("avg_ms", float("nan"))
    achieved = flops_ins / (ins_ms * 1e-3) / 1e12
    roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
                "kernel": f"proj_insertion (fused FP32 contraction + {args.proj} MFMA projection)",
                "flops_per_launch": flops_ins, "avg_ms": round(ins_ms, 4)}
    if args.proj != "f32":
        roofline["note"] = ("flops counted once per complex MAC (8 real flops); the hi+lo split issues "
                            "3 MFMA products per term, so MFMA issue is 3x the counted flops")

    res = {
        "metric": "contracted site*momenta/s (spectator+insertion)",
        "value": value,
        "unit": "site*momenta/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.proj == "f32" else f"f32 contraction, {args.proj} projection",
        "data": "synthetic",
        "config": {"workload": W.name + (", nucleon spectator" if baryon else ""), "L": list(L), "T": T,
                   "t_f": W.t_f, "n_noise": W.N, "n_tau": n_tau, "n_mom": n_mom, "n_ops": W.n_ops,
                   "units_per_step": units, "combine_pairs": {"local": n_mom * n_mom, "derivative": len(pairs),
                                                              "nucleon": len(pairs) if baryon else 0}},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "component_rate": {"projected_complex_values_per_s": (W.N * V3 * n_mom * (192 + (3072 if baryon else 0))
                                                              + W.N * n_tau * V3 * n_mom * 192 * W.n_ops)
                           / (ms_per_step * 1e-3)},
        "kernels_ms": {kname: round(v["avg_ms"], 4) for kname, v in prof.items()},
        "kernel_launches": {kname: v["count"] for kname, v in prof.items()},
        "roofline": roofline,
        "variants": {kn: c3pt.get_variant(c3pt.KIND[kn], mode, c3pt.mt_class(n_mom))
                     for kn in ("spectator_meson", "spectator_baryon", "insertion")},
    }
    if tuning is not None:
        res["tuning"] = tuning["entries"]
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on a host sample")
        res["cpu_baseline"] = cpu_baseline(W, k, args.cpu_slices)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
