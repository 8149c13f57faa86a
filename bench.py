#!/usr/bin/env python3
"""Throughput of the spin-open three-point hot path on one MI355X.

One step = one pass of every hot-path stage over one batch of synthetic input.
Default workload (``meson32``), shaped like the 32^3 x 64 meson measurement:

* meson spectator at t_f = 16 (Eq. (9)) and a nucleon-type epsilon-tensor
  spectator at the same timeslice,
* insertion (Eq. (10)) at tau = 0..16 with the local operator (all 16 Gamma
  open) and the four one-derivative operators D_nu,
* momentum projection of every part onto the 81 momenta with |k|^2 <= 6,
* the noise-weighted combine: local operator on all 81 x 81 momentum pairs,
  derivative operators and the nucleon on the 161 pairs with p' = q or p' = 0.

Inputs: 4 Z2xZ2 noise vectors, Gaussian propagators and stochastic solutions,
Haar SU(3) links, complex64 in HBM.  Arithmetic: FP32 contractions; the
projection factored over the three directions (``--proj fac``, the default:
x1 stage on FP32 MFMA) or as one dense (momenta x sites) GEMM (``--proj f32``
FP32 MFMA, ``bf16x2`` / ``f16x2`` hi+lo 16-bit MFMA with FP32 accumulation);
FP64 split-site accumulation and FP64 combine.

Other workloads (``--workload``): ``meson8`` (8^3 x 16, complex128, 27
momenta, local insertion at tau = 0..8, all-pairs combine), ``nucleon48``
(48^3 x 64, two nucleon spectators (u,u) and (u,d), isovector insertion with
u and d propagators at tau = 0..14, N = 8, 93 or 123 momenta, combine on the
185 pairs with p' = q or p' = 0), ``twosink32`` (forward and backward
diagrams with time-partitioned noise, 32^3 x 96, r_4 = 30, sinks at 20 and
40, N = 50, 93 momenta, local + 4 D_nu), ``batch64`` (64 sources in one recorded
graph) and ``serve`` (Poisson arrivals to the continuous-batching engine).

Prints one JSON line.  ``--gpus`` above 1 is refused: this build runs on one GPU.
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

PEAK = {"f64": 78.6, "f32": 157.3, "bf16x2": 2500.0, "f16x2": 2500.0, "fac": 157.3, "fs16": 2500.0,
        "fsbf16": 2500.0}   # dense MFMA TFLOP/s
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: 20; batch64: 3)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps (default: 3; batch64: 1)")
    ap.add_argument("--workload", choices=["meson32", "meson8", "nucleon48", "twosink32", "batch64", "serve"],
                    default="nucleon48")
    ap.add_argument("--n2", type=int, default=None, help="momentum cutoff |k|^2 (nucleon48: 8 or 9)")
    ap.add_argument("--no-baryon", action="store_true", help="meson32: drop the nucleon spectator")
    ap.add_argument("--analysis", action="store_true",
                    help="nucleon48: add the proton channels of both combines (c3pt_gamma_nucleon) to the step")
    ap.add_argument("--smear", type=int, default=0,
                    help="twosink32: steps of gauge-covariant smearing (kappa 0.25) of the sink propagators "
                         "and noise vectors, in the timed step")
    ap.add_argument("--ops", type=int, choices=[5, 9, 21, 37], default=None,
                    help="meson32 / twosink32 insertion operators: 5 = local + 4 D_nu (default), "
                         "9 = also the 4 symmetrized <->D_nu, 21 (meson32) = also the 16 D_nu D_rho, "
                         "37 (meson32) = also the 16 <->D_mu <->D_nu")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-slices", type=int, default=6, help="insertion timeslices in the CPU sample")
    ap.add_argument("--proj", choices=["f32", "bf16x2", "f16x2", "fac", "fs16", "fsbf16"], default=None,
                    help="projection: dense FP32 MFMA, dense hi+lo BF16 / FP16 MFMA with FP32 accumulation, "
                         "or factored (per-direction partial sums, FP32 MFMA)")
    ap.add_argument("--tune", action="store_true", help="autotune kernel variants on this workload first")
    ap.add_argument("--tune-out", default=None, help="write the tuning table (JSON) here")
    ap.add_argument("--sources", type=int, default=64, help="batch64: number of source positions")
    ap.add_argument("--partial-budget-gib", type=float, default=24.0,
                    help="batch64: device memory for FP32 split-site partial sums")
    ap.add_argument("--no-plain", action="store_true",
                    help="batch64: skip timing the same jobs as plain per-call FP32 launches")
    ap.add_argument("--requests", type=int, default=500, help="serve: requests per load level")
    ap.add_argument("--loads", default="0.5,0.8,0.95", help="serve: arrival rates as fractions of saturation")
    ap.add_argument("--lattices", default="16,32,48,64", help="serve: spatial extents of the resident lattices")
    ap.add_argument("--arena-gib", type=float, default=48.0, help="serve: output arena")
    ap.add_argument("--step-mib", type=float, default=1024.0, help="serve: partial-sum workspace per step")
    ap.add_argument("--max-active", type=int, default=32, help="serve: requests in flight")
    ap.add_argument("--streams", type=int, default=2, choices=[1, 2],
                    help="nucleon48: run the two isovector halves of the step on two streams (default) "
                         "or on one; kernel durations always come from one-stream profiled steps")
    ap.add_argument("--step-work", type=float, default=0.0,
                    help="serve: cap on a step's work in column blocks x sites while no request waits "
                         "for admission (0: none)")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# FP32 VALU peak without packed FP32 instructions (which this library does not
# use): 256 CU x 4 SIMD x 16 lanes x 2 flops (FMA) x 2.4 GHz.
PEAK_VALU_F32 = 78.6

# Contraction arithmetic per (site, column block of 192), 8 flops per complex
# multiply-add: meson spectator and local insertion 192 x 3; baryon 576 for the
# diquark products plus 192 x 3; derivative insertion 192 x 6 plus the
# transport of the stochastic vector 12 x 3 x 2; the left derivative of the
# symmetrized one 192 x 3 plus its transport 12 x 3 x 2.
CONTRACTION_FLOPS = {"spectator_meson": 8.0 * 576, "spectator_baryon": 8.0 * 1152,
                     "insertion_local": 8.0 * 576, "insertion_deriv": 8.0 * (1152 + 72),
                     "insertion_left": 8.0 * (576 + 72)}


# HBM bytes per launch of the dominant kernel, measured with rocprofv3
# FETCH_SIZE and WRITE_SIZE passes (KiB per dispatch, scaled by the plain-copy
# calibration: x2 for FETCH_SIZE, x1 for WRITE_SIZE) on the workload's default
# command; the summary with the full commands is in profiles/ under the kernel
# and workload names.  Each entry carries a hash of the kernel sources it was
# measured with and is reported only while they are unchanged.
TRAFFIC_SOURCES = ["c3pt_fac.h", "c3pt_fac_prod.h", "c3pt_producers.h", "c3pt_device.h", "c3pt_internal.h",
                   "c3pt_fac_meson.hip", "c3pt_fac_baryon.hip", "c3pt_fac_insertion.hip",
                   "c3pt_fs.h", "c3pt_fs_api.h", "c3pt_fs.hip"]
# host functions of c3pt_api.hip that plan and launch the factored and fused kernels
TRAFFIC_FUNCTIONS = ["momentum_groups", "build_factor_plan", "factor_plan_table", "plan_planes", "plan_chunks",
                     "run_projection", "c3pt_spectator_meson", "c3pt_spectator_baryon", "c3pt_insertion",
                     "fs_plans", "fs_setup", "fs_launch_noise_parts", "fs_scratch", "fs_spectator",
                     "fs_insertion"]
MEASURED_TRAFFIC = {
    # workload, projection, timed kernel name, insertion operators -> (bytes per call, source hash)
    # 48^3 step, split-precision fused form: one local insertion call, i.e. its
    # three-block launch (1457191 + 602640 KiB) and the two-block launch of the
    # last two noise vectors (1089615 + 200880 KiB)
    ("nucleon48", "fs16", "fs_insertion", 1): ((1457191 + 1089615) * 2048 + (602640 + 200880) * 1024,
                                               "44654bcb5941f5dc"),
    # 48^3 step, factored FP32 form: one nucleon spectator dispatch (413926 + 857088 KiB)
    ("nucleon48", "fac", "fac_spectator_baryon", 1): (413926 * 2048 + 857088 * 1024, "44654bcb5941f5dc"),
    # 32^3 meson step, factored FP32: one insertion call with local + 4 D_nu, i.e.
    # its local (484210 + 264310 KiB) and derivative (1794856 + 1114112 KiB)
    # dispatches; taken on sources 287b4b579a2a535b, whose factored kernels and
    # planning are those of this hash (only the fused kernel's tile loop differs)
    ("meson32", "fac", "fac_insertion", 5): ((484210 + 1794856) * 2048 + (264310 + 1114112) * 1024,
                                             "44654bcb5941f5dc"),
}


def _function_text(src: str, name: str) -> str:
    """Text of a top-level function definition: from the line that starts it
    (return type and name at column 0, or its template line) to the first
    closing brace at column 0."""
    lines = src.splitlines()
    for i, ln in enumerate(lines):
        if ln[:1].isalpha() and f" {name}(" in ln:
            j = i
            while lines[j] != "}":
                j += 1
            start = i - 1 if i > 0 and lines[i - 1].startswith("template") else i
            return "\n".join(lines[start:j + 1])
    raise KeyError(name)


def _code_only(src: str) -> str:
    """C++ source without its comments and blank lines, each line stripped, so
    that a change of comments alone leaves the hash of the kernels unchanged
    (the sources hold no string literal with comment markers)."""
    import re
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return "\n".join(ln.strip() for ln in src.splitlines() if ln.strip())


def sources_hash(read=None):
    """Hash of the code (comments excluded) of the factored and fused kernels
    and of the host functions that plan and launch them; `read(name)` returns
    the text of a file of csrc/ (default: the working tree)."""
    import hashlib
    if read is None:
        base = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1711_02384_amd", "csrc")

        def read(name):
            with open(os.path.join(base, name)) as f:
                return f.read()
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        h.update(_code_only(read(name)).encode())
    api = read("c3pt_api.hip")
    for name in TRAFFIC_FUNCTIONS:
        h.update(_code_only(_function_text(api, name)).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload, proj, kname, n_ops):
    e = MEASURED_TRAFFIC.get((workload, proj, kname, n_ops))
    if e is None or e[1] != sources_hash():
        return None
    return e[0]


def roofline_entry(kname, flops, kms, proj, traffic=None):
    """Roofline object: dense projections are MFMA-bound (projection flops
    against the MFMA peak of their type); factored ones are bound by the
    contraction's FP32 arithmetic (against the VALU peak)."""
    achieved = flops / (kms * 1e-3) / 1e12
    if proj == "fac":
        peak, bound = PEAK_VALU_F32, "alu"
        what = "fused contraction + factored projection; flops = contraction arithmetic"
    elif proj in ("fs16", "fsbf16"):
        peak, bound = PEAK_VALU_F32, "alu"
        what = ("contraction folded into the x1 stage of the factored projection on hi+lo 16-bit MFMA; "
                "flops = the contraction arithmetic (the plain form's count); the kernel is bound by "
                "VALU issue (A operands, hi+lo splits, stage 2)")
    else:
        peak, bound = PEAK[proj], "mfma"
        what = f"fused contraction + {proj} MFMA projection; flops = 8 per (site, momentum, column)"
    r = {"bound": bound, "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
         "frac": round(achieved / peak, 4), "traffic": traffic, "kernel": f"{kname} ({what})",
         "flops_per_launch": flops, "avg_ms": round(kms, 4)}
    if proj in ("bf16x2", "f16x2"):
        r["note"] = ("flops counted once per complex MAC (8 real flops); the hi+lo split issues "
                     "3 MFMA products per term, so MFMA issue is 3x the counted flops")
    return r


PEAK_HBM_GBS = 8000.0
PEAK_MFMA_F16 = 2500.0   # dense FP16 / BF16 MFMA, TFLOP/s


def fused_mfma_flops(L, N, n_slots, n_share, n_groups=1, cb=2):
    """MFMA flops the fused split-precision kernel issues in one call: every
    wave (four per column block, CB blocks per workgroup, ceil(N / CB)
    workgroups per slot and share; with CB = 3 the last N mod 3 blocks run two
    to a workgroup) runs, per tile of KT sites of one (x2, x3)
    row, 3 summed colours x KT / 16 K steps x 3 column tiles x 3 products
    (lo.hi, hi.lo, hi.hi) of a 16x16x32 MFMA (16384 flops)."""
    kt = 32 if L[0] % 32 == 0 else 16
    tiles = L[1] * L[2] * ((L[0] + kt - 1) // kt)
    if cb == 3:
        # full groups of three, then the last N mod 3 noise vectors as a two-block launch
        blocks = 3 * (N // 3) + 2 * ((N % 3 + 1) // 2)
    else:
        blocks = cb * ((N + cb - 1) // cb)
    waves = 4 * blocks * n_slots * n_share * n_groups
    return float(waves) * tiles * 27 * (kt // 16) * 16384


def pairs_diag_or_zero(n_mom):
    """(p', q) pairs with p' = q or p' = 0 (index 0 is k = 0)."""
    pr = [(p, p) for p in range(n_mom)] + [(0, q) for q in range(1, n_mom)]
    return np.array(pr, dtype=np.int32)


def _up(a, dev, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a.astype(dtype))).to(dev)


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------
class Meson32:
    L = (32, 32, 32)
    T = 64
    t_f = 16
    N = 4
    taus = list(range(0, 17))
    n2 = 6
    n_ops = 5
    cfg = 2
    dtype = "c64"
    default_proj = "fac"
    default_steps = 20
    default_warmup = 3

    def __init__(self, args):
        self.baryon = not args.no_baryon
        self.n_ops = args.ops or 5
        self.name = ("meson+nucleon 3pt, 32^3x64, t_f=16, tau=0..16, N=4, |k|^2<=6 (81 momenta), "
                     "local+4 D_nu" + {5: "", 9: " + 4 symmetrized <->D_nu", 21: " + 16 D_nu D_rho",
                                       37: " + 16 D_nu D_rho + 16 <->D_mu <->D_nu"}[self.n_ops]
                     + (", nucleon spectator" if self.baryon else ""))

    def setup(self, c3pt, syn, dev, geom, k):
        import torch
        L, T = self.L, self.T
        up = lambda a: _up(a, dev, np.complex64)
        self.G1 = up(syn.propagator_slice(L, self.cfg, syn.FIELD_G1, self.t_f))
        self.eta = up(syn.z2z2_noise(L, self.N, self.cfg, self.t_f))
        wide = self.n_ops >= 21          # D_rho G on tau +- 1 needs G on tau +- 2
        gsl = sorted({t % T for tau in self.taus for t in range(tau - 1 - wide, tau + 2 + wide)})
        usl = sorted({t % T for tau in self.taus for t in range(tau - 1 - wide, tau + 1 + wide)})
        self.G3 = {t: up(syn.propagator_slice(L, self.cfg, syn.FIELD_G3, t)) for t in gsl}
        ssl = gsl if self.n_ops in (9, 37) else self.taus
        self.s = {t: up(syn.solution_slice(L, self.N, self.cfg, t)) for t in ssl}
        self.U = {t: up(syn.link_slice(L, self.cfg, t)) for t in usl}
        n_mom, n_tau = len(k), len(self.taus)
        mk = lambda *sh: torch.empty(sh, dtype=torch.complex128, device=dev)
        self.S = mk(self.N, n_mom, 192)
        self.SB = mk(self.N, n_mom, 3072) if self.baryon else None
        self.I = mk(self.N, n_tau, self.n_ops, n_mom, 192)
        self.pairs = pairs_diag_or_zero(n_mom)
        self.C_loc = mk(n_mom * n_mom, n_tau, 1, 64, 64)
        self.C_der = mk(len(self.pairs), n_tau, self.n_ops - 1, 64, 64)
        self.C_bar = mk(len(self.pairs), n_tau, 1, 1024, 64) if self.baryon else None
        self.c3pt, self.geom, self.k = c3pt, geom, k

    def calls(self):
        c, g, k = self.c3pt, self.geom, self.k
        out = [("insertion", lambda: c.insertion(self.G3, self.s, self.taus, k, g, U_t=self.U, n_ops=self.n_ops,
                                                 out=self.I)),
               ("spectator_meson", lambda: c.spectator_meson(self.G1, self.eta, k, g, out=self.S))]
        if self.baryon:
            out.append(("spectator_baryon",
                        lambda: c.spectator_baryon(self.G1, self.G1, self.eta, k, g, out=self.SB)))
        return out

    def step(self):
        c, g, k = self.c3pt, self.geom, self.k
        c.spectator_meson(self.G1, self.eta, k, g, out=self.S)
        if self.baryon:
            c.spectator_baryon(self.G1, self.G1, self.eta, k, g, out=self.SB)
        c.insertion(self.G3, self.s, self.taus, k, g, U_t=self.U, n_ops=self.n_ops, out=self.I)
        c.combine(self.S, self.I, op_begin=0, op_end=1, out=self.C_loc)
        c.combine(self.S, self.I, pairs=self.pairs, op_begin=1, op_end=self.n_ops, out=self.C_der)
        if self.baryon:
            c.combine(self.SB, self.I, pairs=self.pairs, op_begin=0, op_end=1, out=self.C_bar)

    def units(self, n_mom):
        V3 = int(np.prod(self.L))
        spec = self.N * V3 * n_mom * (2 if self.baryon else 1)
        ins = self.N * len(self.taus) * V3 * n_mom
        return spec + ins

    def components(self, n_mom):
        V3 = int(np.prod(self.L))
        return (self.N * V3 * n_mom * (192 + (3072 if self.baryon else 0))
                + self.N * len(self.taus) * V3 * n_mom * 192 * self.n_ops)

    def dominant(self, n_mom, proj):
        V3 = int(np.prod(self.L))
        if proj == "fac":
            # column blocks per (noise, timeslice) of each producer
            n_local = {1: 1, 5: 1, 9: 1, 21: 1, 37: 17}[self.n_ops]
            n_deriv = {1: 0, 5: 4, 9: 4, 21: 20, 37: 36}[self.n_ops]
            n_left = 4 if self.n_ops == 9 else 0
            per = (n_local * CONTRACTION_FLOPS["insertion_local"] + n_deriv * CONTRACTION_FLOPS["insertion_deriv"]
                   + n_left * CONTRACTION_FLOPS["insertion_left"])
            return "fac_insertion", self.N * len(self.taus) * V3 * per
        cols = self.N * len(self.taus) * self.n_ops * 192
        return "proj_insertion", 8.0 * n_mom * V3 * cols

    def config(self, n_mom):
        return {"workload": self.name, "L": list(self.L), "T": self.T, "t_f": self.t_f, "n_noise": self.N,
                "n_tau": len(self.taus), "n_mom": n_mom, "n_ops": self.n_ops,
                "units_per_step": self.units(n_mom)}

    def cpu_sample(self, k, n_slices):
        import c3pt_synth as syn
        import oracle
        L, T = self.L, self.T
        G1 = syn.round_to_c64(syn.propagator_slice(L, self.cfg, syn.FIELD_G1, self.t_f))
        eta = syn.round_to_c64(syn.z2z2_noise(L, self.N, self.cfg, self.t_f))
        if self.n_ops >= 21:
            n_slices = max(1, n_slices // (4 if self.n_ops == 21 else 8))   # the oracle's cost grows with the operators
        taus = self.taus[len(self.taus) // 2: len(self.taus) // 2 + n_slices]
        wide = self.n_ops >= 21
        need = sorted({t % T for tau in taus for t in range(tau - 1 - wide, tau + 2 + wide)})
        G3 = {t: syn.round_to_c64(syn.propagator_slice(L, self.cfg, syn.FIELD_G3, t)) for t in need}
        s_sl = need if self.n_ops in (9, 37) else taus
        s = {t: syn.round_to_c64(syn.solution_slice(L, self.N, self.cfg, t)) for t in s_sl}
        U = {t % T: syn.round_to_c64(syn.link_slice(L, self.cfg, t % T))
             for t in sorted({t + d for t in taus for d in range(-1 - wide, 1 + wide)})}
        t0 = time.perf_counter()
        oracle.spectator_meson(G1, eta, L, k)
        oracle.insertion(G3, s, taus, L, T, k, U_t=U, n_ops=self.n_ops)
        dt = time.perf_counter() - t0
        units = self.N * int(np.prod(L)) * len(k) * (1 + len(taus))
        return units, dt, (f"FP64 numpy oracle: meson spectator + insertion ({self.n_ops} ops) on {len(taus)} of "
                           f"{len(self.taus)} timeslices, full 32^3 slices, N=4, {len(k)} momenta; nucleon "
                           f"spectator and combine not in the sample")


class Meson8(Meson32):
    L = (8, 8, 8)
    T = 16
    t_f = 8
    N = 1
    taus = list(range(0, 9))
    n2 = 3
    n_ops = 1
    cfg = 1
    dtype = "c128"
    default_proj = "f64"

    def __init__(self, args):
        self.baryon = False
        self.name = "meson 3pt, 8^3x16, complex128, t_f=8, tau=0..8, N=1, |k|^2<=3 (27 momenta), local"

    def setup(self, c3pt, syn, dev, geom, k):
        import torch
        L = self.L
        up = lambda a: _up(a, dev, np.complex128)
        self.G1 = up(syn.propagator_slice(L, self.cfg, syn.FIELD_G1, self.t_f))
        self.eta = up(syn.z2z2_noise(L, self.N, self.cfg, self.t_f))
        self.G3 = {t: up(syn.propagator_slice(L, self.cfg, syn.FIELD_G3, t)) for t in self.taus}
        self.s = {t: up(syn.solution_slice(L, self.N, self.cfg, t)) for t in self.taus}
        n_mom = len(k)
        mk = lambda *sh: torch.empty(sh, dtype=torch.complex128, device=dev)
        self.S = mk(self.N, n_mom, 192)
        self.I = mk(self.N, len(self.taus), 1, n_mom, 192)
        self.C = mk(n_mom * n_mom, len(self.taus), 1, 64, 64)
        self.c3pt, self.geom, self.k = c3pt, geom, k

    def calls(self):
        c, g, k = self.c3pt, self.geom, self.k
        return [("insertion", lambda: c.insertion(self.G3, self.s, self.taus, k, g, out=self.I)),
                ("spectator_meson", lambda: c.spectator_meson(self.G1, self.eta, k, g, out=self.S))]

    def step(self):
        c, g, k = self.c3pt, self.geom, self.k
        c.spectator_meson(self.G1, self.eta, k, g, out=self.S)
        c.insertion(self.G3, self.s, self.taus, k, g, out=self.I)
        c.combine(self.S, self.I, out=self.C)

    def dominant(self, n_mom, proj):
        V3 = int(np.prod(self.L))
        if proj == "fac":
            return "fac_insertion", self.N * len(self.taus) * V3 * CONTRACTION_FLOPS["insertion_local"]
        cols = self.N * len(self.taus) * 192
        return "proj_insertion", 8.0 * n_mom * V3 * cols

    def cpu_sample(self, k, n_slices):
        import c3pt_synth as syn
        import oracle
        L, T = self.L, self.T
        G1 = syn.propagator_slice(L, self.cfg, syn.FIELD_G1, self.t_f)
        eta = syn.z2z2_noise(L, self.N, self.cfg, self.t_f)
        G3 = {t: syn.propagator_slice(L, self.cfg, syn.FIELD_G3, t) for t in self.taus}
        s = {t: syn.solution_slice(L, self.N, self.cfg, t) for t in self.taus}
        t0 = time.perf_counter()
        reps = 0
        while time.perf_counter() - t0 < 10.0:
            S = oracle.spectator_meson(G1, eta, L, k)
            I = oracle.insertion(G3, s, self.taus, L, T, k)
            oracle.combine(S, I)
            reps += 1
        dt = time.perf_counter() - t0
        return self.units(len(k)) * reps, dt, f"FP64 numpy oracle: the whole step, repeated {reps} times"


class Nucleon48(Meson32):
    L = (48, 48, 48)
    T = 64
    t_f = 14
    N = 8
    taus = list(range(0, 15))
    n2 = 8
    n_ops = 1
    cfg = 3
    dtype = "c64"
    default_proj = "fs16"
    default_warmup = 6     # the first steps of a fresh process run slower (measured 17.3, 15.7, 15.0, then 14.8 ms)
    plain_proj = "fac"
    # outputs the CPU-baseline sample recomputes with the oracle (2 of 8 noise
    # vectors of the (u,u) spectator, the u insertion on 2 of 15 timeslices)
    sample_noise = 2
    sample_taus = [7, 8]

    def __init__(self, args):
        self.baryon = True
        self.n2 = args.n2 if args.n2 is not None else 8
        self.analysis = args.analysis
        self.streams = args.streams
        self.one_stream = False   # set while profiling: kernel durations without sharing
        self.name = (f"nucleon 3pt, 48^3x64, t_f=14, tau=0..14, N=8, |k|^2<={self.n2}, spectators (u,u) and "
                     f"(u,d), isovector insertion (u and d), local"
                     + (", proton channels (C gamma5, parity projectors, 16 Gamma_ins)" if self.analysis else "")
                     + (", the two isovector halves on two streams" if self.streams == 2 else ""))

    def setup(self, c3pt, syn, dev, geom, k):
        import torch
        L = self.L
        up = lambda a: _up(a, dev, np.complex64)
        self.Gu = {t: up(syn.propagator_slice(L, self.cfg, syn.FIELD_G3, t)) for t in self.taus}
        self.Gd = {t: up(syn.propagator_slice(L, self.cfg, syn.FIELD_G1, t)) for t in self.taus}
        self.eta = up(syn.z2z2_noise(L, self.N, self.cfg, self.t_f))
        self.s = {t: up(syn.solution_slice(L, self.N, self.cfg, t)) for t in self.taus}
        n_mom, n_tau = len(k), len(self.taus)
        mk = lambda *sh: torch.empty(sh, dtype=torch.complex128, device=dev)
        self.Suu = mk(self.N, n_mom, 3072)
        self.Sud = mk(self.N, n_mom, 3072)
        self.Iu = mk(self.N, n_tau, 1, n_mom, 192)
        self.Id = mk(self.N, n_tau, 1, n_mom, 192)
        self.pairs = pairs_diag_or_zero(n_mom)
        self.Cd = mk(len(self.pairs), n_tau, 1, 1024, 64)
        self.Cu = mk(len(self.pairs), n_tau, 1, 1024, 64)
        self.c3pt, self.geom, self.k = c3pt, geom, k
        self.side = torch.cuda.Stream(device=dev) if self.streams == 2 else None   # default priority
        j0, j1 = self.taus.index(self.sample_taus[0]), self.taus.index(self.sample_taus[-1]) + 1
        self.sample_outputs = {"spectator_baryon": lambda: self.Suu[:self.sample_noise],
                               "insertion": lambda: self.Iu[:, j0:j1]}

    def calls(self):
        c, g, k = self.c3pt, self.geom, self.k
        tf = self.t_f
        return [("insertion", lambda: c.insertion(self.Gu, self.s, self.taus, k, g, out=self.Iu)),
                ("spectator_baryon", lambda: c.spectator_baryon(self.Gu[tf], self.Gu[tf], self.eta, k, g,
                                                                out=self.Suu))]

    def step(self):
        """With --streams 2 the two isovector halves of the step run on two
        streams: (u,u) spectator, d insertion and their combine on the current
        stream, (u,d) spectator, u insertion and their combine on a second one
        (default priority), joined at the end, so that the memory-bound passes
        of one half (diquark, reduction, combine) run beside the
        arithmetic-bound kernels of the other and the launch tails overlap.
        Kernel durations then include that sharing."""
        import torch
        c, g, k = self.c3pt, self.geom, self.k
        tf = self.t_f
        main = torch.cuda.current_stream()
        side = self.side if self.side is not None and not self.one_stream else main
        fork = torch.cuda.Event()
        fork.record(main)
        side.wait_event(fork)
        gs = c.Geom(g.L, g.T, r=g.r, proj=g.proj, stream=side.cuda_stream)
        # proton isovector: spectators (u,u) with the d insertion, (u,d) with the u
        # insertion; the second stream starts with its insertion while the first
        # forms its diquark, so that the memory-bound passes do not coincide
        c.spectator_baryon(self.Gu[tf], self.Gu[tf], self.eta, k, g, out=self.Suu)
        c.insertion(self.Gu, self.s, self.taus, k, gs, out=self.Iu)
        c.insertion(self.Gd, self.s, self.taus, k, g, out=self.Id)
        c.spectator_baryon(self.Gu[tf], self.Gd[tf], self.eta, k, gs, out=self.Sud)
        c.combine(self.Suu, self.Id, pairs=self.pairs, out=self.Cd)
        c.combine(self.Sud, self.Iu, pairs=self.pairs, out=self.Cu, stream=side.cuda_stream)
        join = torch.cuda.Event()
        join.record(side)
        main.wait_event(join)
        if self.analysis:
            # proton channels of both currents: tr[P_pm G] for the 16 Gamma_ins
            self.ch_d = c.gamma_nucleon(self.Cd, c.PROTON_D)
            self.ch_u = c.gamma_nucleon(self.Cu, c.PROTON_U)

    def units(self, n_mom):
        V3 = int(np.prod(self.L))
        return 2 * self.N * V3 * n_mom + 2 * self.N * len(self.taus) * V3 * n_mom

    def components(self, n_mom):
        V3 = int(np.prod(self.L))
        return 2 * self.N * V3 * n_mom * 3072 + 2 * self.N * len(self.taus) * V3 * n_mom * 192

    def dominant(self, n_mom, proj):
        """Candidate kernels and their contraction flops per launch; the one with
        the most time per step is reported."""
        V3 = int(np.prod(self.L))
        spec = 16 * self.N * V3 * CONTRACTION_FLOPS["spectator_baryon"]
        ins = self.N * len(self.taus) * V3 * CONTRACTION_FLOPS["insertion_local"]
        if proj == "fac":
            return {"fac_spectator_baryon": spec, "fac_insertion": ins}
        if proj in ("fs16", "fsbf16"):
            return {"fs_spectator_baryon": spec, "fs_insertion": ins}
        cols = self.N * 3072
        return "proj_spectator_baryon", 8.0 * n_mom * V3 * cols

    def mfma_flops(self, kname, proj):
        """MFMA flops issued per launch of the fused kernels (one momentum group)."""
        if proj not in ("fs16", "fsbf16") or len(self.k) > 128:
            return None
        c = self.c3pt
        kind = 1 if kname == "fs_spectator_baryon" else 2
        v = c.get_variant(kind, c.MODE[proj], c.mt_class(len(self.k)))
        cb = 3 if v == 4 and self.L[0] % 32 != 0 else (1 if v in (2, 3) else 2)
        if kname == "fs_insertion":
            return fused_mfma_flops(self.L, self.N, 1, len(self.taus), cb=cb)
        if kname == "fs_spectator_baryon":
            return fused_mfma_flops(self.L, self.N, 16, 1, cb=cb)
        return None

    def cpu_sample(self, k, n_slices):
        """One noise vector of the (u,u) nucleon spectator, the u insertion on
        one timeslice with all 8 noise vectors, and the combine of that noise
        vector's spectator with its insertion on the step's pairs."""
        import c3pt_synth as syn
        import oracle
        L = self.L
        tau = self.taus[len(self.taus) // 2]
        Gf = syn.round_to_c64(syn.propagator_slice(L, self.cfg, syn.FIELD_G3, self.t_f))
        ns, ts = self.sample_noise, self.sample_taus
        nt = len(ts)
        eta = syn.round_to_c64(syn.z2z2_noise(L, ns, self.cfg, self.t_f))
        Gu = {t: syn.round_to_c64(syn.propagator_slice(L, self.cfg, syn.FIELD_G3, t)) for t in ts}
        s = {t: syn.round_to_c64(syn.solution_slice(L, self.N, self.cfg, t)) for t in ts}
        pairs = pairs_diag_or_zero(len(k))
        t0 = time.perf_counter()
        S = oracle.spectator_baryon(Gf, Gf, eta, L, k)
        I = oracle.insertion(Gu, s, ts, L, self.T, k)
        oracle.combine(S, I[:ns], pairs=pairs)
        dt = time.perf_counter() - t0
        # the same outputs as the step's (u,u) spectator noise 0..ns-1 and u insertion at ts
        self.oracle_ref = {"spectator_baryon": S, "insertion": I}
        V3 = int(np.prod(L))
        units = ns * V3 * len(k) + self.N * nt * V3 * len(k)
        return units, dt, (f"FP64 numpy oracle: (u,u) nucleon spectator with {ns} of 8 noise vectors, u "
                           f"insertion on {nt} of 15 timeslices with N=8, and the combine of those {ns} noise "
                           f"vectors on {len(pairs)} pairs; full 48^3 slices, {len(k)} momenta")

class TwoSink32(Meson32):
    """Forward and backward meson diagrams with time-partitioned noise in the
    shape of the paper's measurement (Sec. 3): 32^3 x 96, source r_4 = 30,
    sinks x'_4 = 20 and x''_4 = 40, N = 50 noise vectors with support on both
    sink timeslices, momenta |k|^2 <= 8 (93).  One step = spectators at both
    sinks, the insertion (local and the four D_nu) on the 21 timeslices
    20..40, and the forward / backward combines on the 185 pairs with p' = q or
    p' = 0, all in one c3pt_two_sink_meson call; then the 16 x 16 x 16 Gamma
    channels of both diagrams (c3pt_gamma_meson)."""
    L = (32, 32, 32)
    T = 96
    t_src, t_fwd, t_bwd = 30, 20, 40
    N = 50
    n2 = 8
    n_ops = 5
    cfg = 5
    dtype = "c64"
    default_proj = "fac"
    default_steps = 10
    default_warmup = 2

    def __init__(self, args):
        self.baryon = False
        self.n_ops = args.ops or 5
        if self.n_ops >= 21:
            raise SystemExit("twosink32 takes --ops 5 or 9")
        self.taus = [(self.t_fwd + j) % self.T for j in range((self.t_bwd - self.t_fwd) % self.T + 1)]
        self.smear_iter, self.kappa = args.smear, 0.25
        self.name = ("meson 3pt forward + backward with time-partitioned noise, 32^3x96, r_4=30, x'_4=20, "
                     "x''_4=40, N=50, |k|^2<=8 (93 momenta), local+4 D_nu"
                     + (" + 4 symmetrized <->D_nu" if self.n_ops == 9 else "") + ", 185 pairs, 16^3 Gamma channels"
                     + (f", sink smearing {self.smear_iter} x kappa {self.kappa}" if self.smear_iter else ""))

    def setup(self, c3pt, syn, dev, geom, k):
        L, T = self.L, self.T
        up = lambda a: _up(a, dev, np.complex64)
        self.Gf = up(syn.propagator_slice(L, self.cfg, syn.FIELD_G1, self.t_fwd))
        self.Gb = up(syn.propagator_slice(L, self.cfg, syn.FIELD_G1, self.t_bwd))
        self.eta_f = up(syn.z2z2_noise(L, self.N, self.cfg, self.t_fwd))
        self.eta_b = up(syn.z2z2_noise(L, self.N, self.cfg, self.t_bwd))
        wide = self.n_ops >= 21          # D_rho G on tau +- 1 needs G on tau +- 2
        gsl = sorted({t % T for tau in self.taus for t in range(tau - 1 - wide, tau + 2 + wide)})
        usl = sorted({t % T for tau in self.taus for t in range(tau - 1 - wide, tau + 1 + wide)})
        self.G3 = {t: up(syn.propagator_slice(L, self.cfg, syn.FIELD_G3, t)) for t in gsl}
        ssl = gsl if self.n_ops in (9, 37) else self.taus
        self.s = {t: up(syn.solution_slice(L, self.N, self.cfg, t)) for t in ssl}
        self.U = {t: up(syn.link_slice(L, self.cfg, t)) for t in usl}
        self.pairs = pairs_diag_or_zero(len(k))
        import torch
        self.sm = [torch.empty_like(x) for x in (self.Gf, self.Gb, self.eta_f, self.eta_b)]
        self.c3pt, self.geom, self.k = c3pt, geom, k

    def _run(self):
        Gf, Gb, ef, eb = self.Gf, self.Gb, self.eta_f, self.eta_b
        if self.smear_iter:
            # sink smearing of the spectator's propagator and of the noise at both sinks
            c, g, n, kap = self.c3pt, self.geom, self.smear_iter, self.kappa
            Gf = c.smear_propagator(self.Gf, self.U[self.t_fwd], g, kap, n, out=self.sm[0])
            Gb = c.smear_propagator(self.Gb, self.U[self.t_bwd], g, kap, n, out=self.sm[1])
            ef = c.smear_vectors(self.eta_f, self.U[self.t_fwd], g, kap, n, out=self.sm[2])
            eb = c.smear_vectors(self.eta_b, self.U[self.t_bwd], g, kap, n, out=self.sm[3])
        return self.c3pt.two_sink_meson(Gf, ef, self.t_fwd, Gb, eb, self.t_bwd,
                                        self.t_src, self.G3, self.s, self.k, self.geom, U_t=self.U,
                                        n_ops=self.n_ops, pairs=self.pairs)

    def calls(self):
        c, g, k = self.c3pt, self.geom, self.k
        return [("insertion", lambda: c.insertion(self.G3, self.s, self.taus, k, g, U_t=self.U, n_ops=self.n_ops)),
                ("spectator_meson", lambda: c.spectator_meson(self.Gf, self.eta_f, k, g))]

    def step(self):
        self.out = self._run()
        # analysis stage: every Gamma_snk x Gamma_ins x Gamma_src channel of both diagrams
        self.ch_fwd = self.c3pt.gamma_meson(self.out["fwd"])
        self.ch_bwd = self.c3pt.gamma_meson(self.out["bwd"])

    def units(self, n_mom):
        return self.N * int(np.prod(self.L)) * n_mom * (2 + len(self.taus))

    def components(self, n_mom):
        return self.N * int(np.prod(self.L)) * n_mom * 192 * (2 + len(self.taus) * self.n_ops)

    def config(self, n_mom):
        return {"workload": self.name, "L": list(self.L), "T": self.T, "t_src": self.t_src, "t_fwd": self.t_fwd,
                "t_bwd": self.t_bwd, "n_noise": self.N, "n_tau": len(self.taus), "n_mom": n_mom,
                "n_ops": self.n_ops, "n_pairs": len(self.pairs), "smear_steps": self.smear_iter,
                "units_per_step": self.units(n_mom)}

    def cpu_sample(self, k, n_slices):
        import c3pt_synth as syn
        import oracle
        L, T, n = self.L, self.T, 12
        c64 = syn.round_to_c64
        Gf = c64(syn.propagator_slice(L, self.cfg, syn.FIELD_G1, self.t_fwd))
        Gb = c64(syn.propagator_slice(L, self.cfg, syn.FIELD_G1, self.t_bwd))
        eta_f = c64(syn.z2z2_noise(L, self.N, self.cfg, self.t_fwd))[:n]
        eta_b = c64(syn.z2z2_noise(L, self.N, self.cfg, self.t_bwd))[:n]
        ns = max(1, n_slices // 2)
        taus = [(self.t_src + j) % T for j in range(ns)]
        need = sorted({t % T for tau in taus for t in (tau - 1, tau, tau + 1)})
        G3 = {t: c64(syn.propagator_slice(L, self.cfg, syn.FIELD_G3, t)) for t in need}
        s_sl = need if self.n_ops == 9 else taus
        s = {t: c64(syn.solution_slice(L, self.N, self.cfg, t))[:n] for t in s_sl}
        U = {t % T: c64(syn.link_slice(L, self.cfg, t % T)) for t in sorted({t - 1 for t in taus} | set(taus))}
        t0 = time.perf_counter()
        oracle.spectator_meson(Gf, eta_f, L, k)
        oracle.spectator_meson(Gb, eta_b, L, k)
        oracle.insertion(G3, s, taus, L, T, k, U_t=U, n_ops=self.n_ops)
        dt = time.perf_counter() - t0
        units = n * int(np.prod(L)) * len(k) * (2 + len(taus))
        return units, dt, (f"FP64 numpy oracle: meson spectators at both sinks + insertion (5 ops) on {len(taus)} "
                           f"of {len(self.taus)} timeslices, full 32^3 slices, {n} of {self.N} noise vectors, "
                           f"{len(k)} momenta; combines not in the sample")


class Batch64:
    """Many source positions over uneven lattices in one recorded graph.

    Source j sits on lattice j mod 3 of (24^3 x 48, 32^3 x 64, 48^3 x 96), at a
    seeded random (r, t_src) with t_f - t_src drawn uniformly from 8..16; even
    j are mesons (one propagator: spectator at t_f, insertion at every tau of
    t_src..t_f), odd j nucleons (two spectators (u,u), (u,d) and two insertions
    with the u and d propagators).  N = 8 noise vectors per source, 93 momenta,
    local insertion.  Combines: mesons on the 185 pairs with p' = q or p' = 0,
    nucleons on the 7 pairs with p' = 0, |q|^2 <= 1.

    The inputs (about 100 GB for 64 sources) are drawn on the GPU from seeded
    torch generators, with the distributions of the seeded host generators
    (unit complex Gaussians, Z2 x Z2 noise); drawing them on the host would
    take minutes.  Every source has buffers of its own."""
    lattices = (((24, 24, 24), 48), ((32, 32, 32), 64), ((48, 48, 48), 96))
    N = 8
    n2 = 8
    n_ops = 1
    cfg = 4
    dtype = "c64"
    default_proj = "fac"
    default_steps = 3
    default_warmup = 1
    sample_slices = 4

    def __init__(self, args):
        self.n_src = int(args.sources)
        self.budget = int(args.partial_budget_gib * (1 << 30))
        self.plain = not args.no_plain
        self.name = (f"batched 3pt: {self.n_src} sources x N=8 over 24^3x48, 32^3x64, 48^3x96 (source j on lattice "
                     f"j mod 3), t_f-t_src ~ U{{8..16}}, meson (even j) : nucleon (odd j) = 1:1, |k|^2<=8 "
                     f"(93 momenta), local insertion, one graph replay per step")
        self.L = [list(L) for L, _ in self.lattices]
        self.T = [T for _, T in self.lattices]
        self.t_f = "t_src + U{8..16}"

    def sources(self):
        import c3pt_synth as syn
        out = []
        for j in range(self.n_src):
            L, T = self.lattices[j % 3]
            g = syn.rng(self.cfg, 99, j)
            r = [int(g.integers(0, L[d])) for d in range(3)]
            t_src = int(g.integers(0, T))
            dt = int(g.integers(8, 17))
            out.append({"j": j, "L": L, "T": T, "r": r, "t_src": t_src, "dt": dt,
                        "taus": [(t_src + i) % T for i in range(dt + 1)], "t_f": (t_src + dt) % T,
                        "nucleon": j % 2 == 1})
        return out

    def setup(self, c3pt, syn, dev, geom, k):
        import torch
        gen = torch.Generator(device=dev)
        N = self.N
        inv = 1.0 / np.sqrt(2.0)

        def draw(shape, seed):
            gen.manual_seed(seed)
            return torch.randn(shape, dtype=torch.complex64, device=dev, generator=gen)

        def noise(V3, seed):
            gen.manual_seed(seed)
            b = torch.randint(0, 2, (N, 12, V3, 2), device=dev, generator=gen, dtype=torch.int8)
            return torch.view_as_complex(((1 - 2 * b).float() * inv).contiguous())

        n_mom = len(k)
        mk = lambda *sh: torch.empty(sh, dtype=torch.complex128, device=dev)
        pairs_m = pairs_diag_or_zero(n_mom)
        pairs_n = np.array([(0, q) for q in range(7)], dtype=np.int32)
        self.src = self.sources()
        self.proj = geom.proj
        jobs, combs, self.plain_calls = [], [], []
        self.flops = {"spectator_meson": 0.0, "spectator_baryon": 0.0, "insertion": 0.0}
        self.units_total = 0
        for s in self.src:
            L, T, V3 = s["L"], s["T"], int(np.prod(s["L"]))
            seed = lambda field, t: ((self.cfg * 1024 + s["j"]) * 16 + field) * 4096 + t
            eta = noise(V3, seed(syn.FIELD_ETA, s["t_f"]))
            sl = {t: draw((N, 12, V3), seed(syn.FIELD_S, t)) for t in s["taus"]}
            flav = {"u": {t: draw((12, 12, V3), seed(syn.FIELD_G3, t)) for t in s["taus"]}}
            if s["nucleon"]:
                flav["d"] = {t: draw((12, 12, V3), seed(syn.FIELD_G1, t)) for t in s["taus"]}
            base = dict(L=L, T=T, r=s["r"])
            n_tau, tf = len(s["taus"]), s["t_f"]
            dense = self.proj != 3
            ins_flops = (8.0 * n_mom * 192 if dense else CONTRACTION_FLOPS["insertion_local"]) * V3 * N * n_tau
            mes_flops = (8.0 * n_mom * 192 if dense else CONTRACTION_FLOPS["spectator_meson"]) * V3 * N
            bar_flops = (8.0 * n_mom * 3072 if dense else 16 * CONTRACTION_FLOPS["spectator_baryon"]) * V3 * N
            if not s["nucleon"]:
                G = flav["u"]
                jobs.append(dict(kind="spectator_meson", G=G[tf], eta=eta, **base))
                jobs.append(dict(kind="insertion", G_t=G, s_t=sl, taus=s["taus"], n_ops=1, **base))
                combs.append({"spec": len(jobs) - 2, "ins": len(jobs) - 1, "pairs": pairs_m})
                self.flops["spectator_meson"] += mes_flops
                self.flops["insertion"] += ins_flops
                self.units_total += N * V3 * n_mom * (1 + n_tau)
            else:
                Gu, Gd = flav["u"], flav["d"]
                jobs.append(dict(kind="spectator_baryon", G1=Gu[tf], G2=Gu[tf], eta=eta, **base))
                jobs.append(dict(kind="spectator_baryon", G1=Gu[tf], G2=Gd[tf], eta=eta, **base))
                jobs.append(dict(kind="insertion", G_t=Gu, s_t=sl, taus=s["taus"], n_ops=1, **base))
                jobs.append(dict(kind="insertion", G_t=Gd, s_t=sl, taus=s["taus"], n_ops=1, **base))
                n = len(jobs)
                # proton isovector: (u,u) spectator with the d insertion, (u,d) with the u insertion
                combs.append({"spec": n - 4, "ins": n - 1, "pairs": pairs_n})
                combs.append({"spec": n - 3, "ins": n - 2, "pairs": pairs_n})
                self.flops["spectator_baryon"] += 2 * bar_flops
                self.flops["insertion"] += 2 * ins_flops
                self.units_total += 2 * N * V3 * n_mom * (1 + n_tau)
        torch.cuda.synchronize()
        log(f"[bench] {len(jobs)} jobs, {len(combs)} combines; "
            f"{torch.cuda.memory_allocated() / 2**30:.1f} GiB of inputs resident")
        self.jobs, self.combs = jobs, combs
        self.c3pt, self.k, self.proj = c3pt, k, geom.proj
        self.record()
        # outputs the CPU-baseline sample recomputes with the oracle: source 0's
        # spectator and its first insertion timeslices
        nt = min(self.sample_slices, len(self.src[0]["taus"]))
        self.sample_outputs = {"spectator_meson": lambda: self.batch.outputs[0],
                               "insertion": lambda: self.batch.outputs[1][:, :nt]}

    def record(self):
        """(Re)record the batch graph; kernel variants are fixed at recording."""
        old = getattr(self, "batch", None)
        outs = (old.outputs, old.combine_outputs) if old is not None else None
        if old is not None:
            old.close()
        jobs = self.jobs
        if outs is not None:
            jobs = [dict(j, out=o) for j, o in zip(self.jobs, outs[0])]
        self.batch = self.c3pt.Batch(jobs, self.k, proj=self.proj, combines=self.combs,
                                     partial_budget=self.budget)
        log(f"[bench] batch recorded: {self.batch.info()}")

    def _single(self, j, g, out):
        c, k = self.c3pt, self.k
        if j["kind"] == "spectator_meson":
            return c.spectator_meson(j["G"], j["eta"], k, g, out=out)
        if j["kind"] == "spectator_baryon":
            return c.spectator_baryon(j["G1"], j["G2"], j["eta"], k, g, out=out)
        return c.insertion(j["G_t"], j["s_t"], j["taus"], k, g, n_ops=1, out=out)

    def calls(self):
        """Single calls of one 48^3 nucleon source (for the tuner)."""
        c = self.c3pt
        nuc = [i for i, s in enumerate(self.src) if s["nucleon"]]
        big = [i for i in nuc if self.src[i]["L"][0] == 48]
        idx = (big or nuc or [0])[0]
        jn = sum(4 if s["nucleon"] else 2 for s in self.src[:idx])
        out = []
        for kn, off in (("spectator_baryon", 0), ("insertion", 2)):
            j = self.jobs[jn + off]
            g = c.Geom(j["L"], j["T"], r=j["r"], proj=self.proj_flag)
            o = self.batch.outputs[jn + off]
            out.append((kn, (lambda j=j, g=g, o=o: self._single(j, g, o))))
        return out

    def step(self):
        self.batch.run()

    def plain_step(self, proj_flag):
        """The same jobs as plain per-call launches with projection proj_flag (no graph, no batching)."""
        c = self.c3pt
        for j, o in zip(self.jobs, self.batch.outputs):
            self._single(j, c.Geom(j["L"], j["T"], r=j["r"], proj=proj_flag), o)
        for cm, o in zip(self.combs, self.batch.combine_outputs):
            c.combine(self.batch.outputs[cm["spec"]], self.batch.outputs[cm["ins"]], pairs=cm["pairs"], out=o)

    def units(self, n_mom):
        return self.units_total

    def components(self, n_mom):
        tot = 0
        for s in self.src:
            V3, nt = int(np.prod(s["L"])), len(s["taus"])
            if s["nucleon"]:
                tot += 2 * self.N * V3 * n_mom * (3072 + nt * 192)
            else:
                tot += self.N * V3 * n_mom * (192 + nt * 192)
        return tot

    def kernel_flops(self):
        prefix = "batch_fac_" if self.proj == 3 else "batch_proj_"
        return {prefix + kn: f for kn, f in self.flops.items()}

    def config(self, n_mom):
        return {"workload": self.name, "lattices": ["24^3x48", "32^3x64", "48^3x96"], "n_sources": self.n_src,
                "n_noise": self.N, "n_mom": n_mom, "n_ops": 1, "jobs": len(self.jobs),
                "combines": len(self.combs), "units_per_step": self.units_total, "batch": self.batch.info()}

    def cpu_sample(self, k, n_slices):
        """Source 0 (a 24^3 meson) from the batch's own resident inputs: its
        spectator and its first sample_slices insertion timeslices; the outputs
        are kept as the reference for the accuracy of every form."""
        import oracle
        L, T = self.lattices[0]
        src = self.src[0]
        js, ji = self.jobs[0], self.jobs[1]
        G = js["G"].cpu().numpy()
        eta = js["eta"].cpu().numpy()
        taus = src["taus"][:self.sample_slices]
        Gt = {t: ji["G_t"][t].cpu().numpy() for t in taus}
        st = {t: ji["s_t"][t].cpu().numpy() for t in taus}
        t0 = time.perf_counter()
        S = oracle.spectator_meson(G, eta, L, k, r=src["r"])
        I = oracle.insertion(Gt, st, taus, L, T, k, r=src["r"])
        dt = time.perf_counter() - t0
        self.oracle_ref = {"spectator_meson": S, "insertion": I}
        units = self.N * int(np.prod(L)) * len(k) * (1 + len(taus))
        return units, dt, (f"FP64 numpy oracle: source 0 (24^3 meson) on the batch's own inputs, spectator + "
                           f"{len(taus)} insertion timeslices, N=8, {len(k)} momenta; nucleon sources and "
                           f"combines not in the sample")


WORKLOADS = {"meson32": Meson32, "meson8": Meson8, "nucleon48": Nucleon48, "twosink32": TwoSink32,
             "batch64": Batch64}


# ---------------------------------------------------------------------------
# Serving: Poisson arrivals of contraction requests (continuous batching)
# ---------------------------------------------------------------------------
SERVE_LATTICES = {16: 32, 32: 64, 48: 96, 64: 128}     # L -> T
SERVE_WEIGHTS = {16: 4, 32: 3, 48: 2, 64: 1}


class ServePool:
    """Resident inputs per lattice: one source's u and d propagators on every
    timeslice, stochastic solutions of 16 noise vectors on every timeslice,
    and 16 noise vectors on one sink slice (shared by every t_f).  Drawn on the
    GPU from seeded torch generators (unit complex Gaussians, Z2 x Z2 noise)."""
    N_MAX = 16

    def __init__(self, lattices, dev):
        import torch
        gen = torch.Generator(device=dev)
        self.lat = {}
        inv = 1.0 / np.sqrt(2.0)
        sd = float(np.sqrt(0.5))
        for li, Ls in enumerate(lattices):
            T = SERVE_LATTICES[Ls]
            V3 = Ls ** 3
            d = {"T": T, "V3": V3}
            for fi, name in enumerate(("u", "d")):
                buf = torch.empty((T, 12, 12, V3), dtype=torch.complex64, device=dev)
                gen.manual_seed((5 * 1024 + li) * 8 + fi)
                buf.view(torch.float32).normal_(0.0, sd, generator=gen)
                d[name] = buf
            sbuf = torch.empty((T, self.N_MAX, 12, V3), dtype=torch.complex64, device=dev)
            gen.manual_seed((6 * 1024 + li) * 8)
            sbuf.view(torch.float32).normal_(0.0, sd, generator=gen)
            d["s"] = sbuf
            gen.manual_seed(7 * 1024 + li)
            b = torch.randint(0, 2, (self.N_MAX, 12, V3, 2), device=dev, generator=gen, dtype=torch.int8)
            d["eta"] = torch.view_as_complex(((1 - 2 * b).float() * inv).contiguous())
            self.lat[Ls] = d
            torch.cuda.synchronize()
            log(f"[serve] lattice {Ls}^3x{T} resident ({torch.cuda.memory_allocated() / 2**30:.1f} GiB in HBM)")
        self._k = {}

    def request(self, c3pt, spec):
        """Request dict for the server from a drawn spec (views into the pool)."""
        d = self.lat[spec["L"]]
        T, N = d["T"], spec["N"]
        G = {t: d["u"][t] for t in range(T)}
        G2 = {t: d["d"][t] for t in range(T)} if spec["kind"] == "nucleon" else None
        s_t = {t: d["s"][t, :N] for t in range(T)}
        if spec["n2"] not in self._k:
            k = c3pt.momentum_list(spec["n2"])
            self._k[spec["n2"]] = (k, pairs_diag_or_zero(len(k)))
        k, pairs = self._k[spec["n2"]]
        return {"kind": spec["kind"], "L": (spec["L"],) * 3, "T": T, "r": spec["r"], "t_src": spec["t_src"],
                "t_f": spec["t_f"], "eta": d["eta"][:N], "G_t": G, "G2_t": G2, "s_t": s_t, "n_ops": 1,
                "k": k, "pairs": pairs}


def serve_draw(n, lattices, seed):
    """Seeded request specs: lattice 4:3:2:1, |k|^2 in 3..9, meson or nucleon,
    N in 1..16, t_f - t_src in 8..16, uniform source position and t_src."""
    import c3pt_synth as syn
    g = syn.rng(5, 98, seed)
    w = np.array([SERVE_WEIGHTS[L] for L in lattices], dtype=float)
    w /= w.sum()
    out = []
    for _ in range(n):
        L = int(lattices[g.choice(len(lattices), p=w)])
        T = SERVE_LATTICES[L]
        t_src = int(g.integers(0, T))
        dt = int(g.integers(8, 17))
        out.append({"L": L, "n2": int(g.integers(3, 10)), "kind": "nucleon" if g.integers(0, 2) else "meson",
                    "N": int(g.integers(1, 17)), "t_src": t_src, "t_f": (t_src + dt) % T, "n_tau": dt + 1,
                    "r": [int(g.integers(0, L)) for _ in range(3)]})
    return out


def serve_units(spec, momenta):
    n_mom = momenta[spec["n2"]]
    f = 2 if spec["kind"] == "nucleon" else 1
    return f * spec["N"] * spec["L"] ** 3 * n_mom * (1 + spec["n_tau"])


def serve_flops(spec, momenta, proj):
    """Algorithmic flops per producer kind: projection flops (8 per site,
    momentum and column) for the dense forms, contraction flops for the
    factored form."""
    n_mom, V3, N, nt = momenta[spec["n2"]], spec["L"] ** 3, spec["N"], spec["n_tau"]
    if proj == "fac":
        p, cm, cb, ci = ("serve_fac_", CONTRACTION_FLOPS["spectator_meson"],
                         16 * CONTRACTION_FLOPS["spectator_baryon"], CONTRACTION_FLOPS["insertion_local"])
    else:
        p, cm, cb, ci = "serve_proj_", 8.0 * n_mom * 192, 8.0 * n_mom * 3072, 8.0 * n_mom * 192
    if spec["kind"] == "nucleon":
        return {p + "spectator_baryon": 2 * cb * V3 * N, p + "insertion": 2 * ci * V3 * N * nt}
    return {p + "spectator_meson": cm * V3 * N, p + "insertion": ci * V3 * N * nt}


def serve_main(args):
    import torch
    import paper_1711_02384_amd as c3pt
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    proj = args.proj or "fac"
    proj_flag = {"f32": c3pt.PROJ_NATIVE, "bf16x2": c3pt.PROJ_SPLIT_BF16, "f16x2": c3pt.PROJ_SPLIT_F16,
                 "fac": c3pt.PROJ_FACTORED}[proj]
    lattices = [int(x) for x in args.lattices.split(",")]
    loads = [float(x) for x in args.loads.split(",")]
    momenta = {n2: len(c3pt.momentum_list(n2)) for n2 in range(3, 10)}
    t0 = time.perf_counter()
    pool = ServePool(lattices, dev)
    log(f"[serve] inputs resident ({time.perf_counter() - t0:.1f} s)")
    sv = c3pt.Server(proj=proj_flag, arena_bytes=int(args.arena_gib * 2**30),
                     step_bytes=int(args.step_mib * 2**20), max_active=args.max_active, step_work=args.step_work)
    clock = time.perf_counter

    def drive(specs, arrivals):
        """Submit each request at its arrival time (seconds from start), step the
        engine, and record completion times; returns (latencies, wall seconds)."""
        order = np.argsort(arrivals, kind="stable")
        lat = np.zeros(len(specs))
        pending = {}
        nxt = 0
        start = clock()
        while nxt < len(order) or pending:
            now = clock() - start
            while nxt < len(order) and arrivals[order[nxt]] <= now:
                i = int(order[nxt])
                rid = sv.submit(pool.request(c3pt, specs[i]))
                pending[rid] = i
                nxt += 1
            na, nq = sv.step() if pending else (0, 0)
            for rid in list(pending):
                if sv.poll(rid):
                    i = pending.pop(rid)
                    lat[i] = (clock() - start) - arrivals[i]
                    sv.release(rid)
            if not pending and nxt < len(order):
                wait = arrivals[order[nxt]] - (clock() - start)
                if wait > 0:
                    time.sleep(min(wait, 0.01))
            elif pending and na == 0:
                time.sleep(0.0005)
        return lat, clock() - start

    # warm-up: one request per (lattice, cutoff, kind) builds every phase table
    warm = []
    for L in lattices:
        for n2 in range(3, 10):
            for kind in ("meson", "nucleon"):
                T = SERVE_LATTICES[L]
                warm.append({"L": L, "n2": n2, "kind": kind, "N": 1, "t_src": 0, "t_f": 8, "n_tau": 9,
                             "r": [0, 0, 0]})
    log(f"[serve] warm-up: {len(warm)} requests")
    drive(warm, np.zeros(len(warm)))
    torch.cuda.synchronize()

    # saturation: a closed batch of requests all present at t = 0
    n_sat = max(40, args.requests // 2)
    sat = serve_draw(n_sat, lattices, seed=1)
    log(f"[serve] saturation run: {n_sat} requests at once")
    lat_sat, wall = drive(sat, np.zeros(n_sat))
    units_sat = sum(serve_units(sp, momenta) for sp in sat)
    rate = n_sat / wall
    value = units_sat / wall
    log(f"[serve] saturated: {rate:.1f} requests/s, {value:.3g} units/s")

    # per-kernel timing on a profiled closed batch
    prof_specs = serve_draw(max(12, n_sat // 4), lattices, seed=2)
    c3pt.profile_read(reset=True)
    c3pt.profile_enable(True)
    drive(prof_specs, np.zeros(len(prof_specs)))
    torch.cuda.synchronize()
    c3pt.profile_enable(False)
    prof = c3pt.profile_read(reset=True)
    kflops = {}
    for sp in prof_specs:
        for kn, f in serve_flops(sp, momenta, proj).items():
            kflops[kn] = kflops.get(kn, 0.0) + f
    kname = max((kn for kn in kflops if kn in prof), key=lambda kn: prof[kn]["total_ms"])
    launches = prof[kname]["count"]
    roof = roofline_entry(kname, kflops[kname] / launches, prof[kname]["avg_ms"], proj)
    roof["kernel"] += ", over a profiled closed batch"

    levels = []
    for li, rho in enumerate(loads):
        specs = serve_draw(args.requests, lattices, seed=10 + li)
        g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([1711, 2384, 5, 97, li])))
        arrivals = np.cumsum(g.exponential(1.0 / (rho * rate), size=len(specs)))
        log(f"[serve] load {rho}: {len(specs)} Poisson arrivals at {rho * rate:.1f} requests/s")
        lat, wall_l = drive(specs, arrivals)
        units = sum(serve_units(sp, momenta) for sp in specs)
        per_L = {}
        for L in lattices:
            sel = np.array([sp["L"] == L for sp in specs])
            if sel.any():
                per_L[f"{L}^3"] = {"requests": int(sel.sum()), "p50_ms": float(np.percentile(lat[sel], 50) * 1e3),
                                   "p99_ms": float(np.percentile(lat[sel], 99) * 1e3)}
        # slowdown: latency over the request's own share of the saturated rate
        # (its units / the saturated units per second)
        slow = lat / np.array([serve_units(sp, momenta) / value for sp in specs])
        levels.append({"rho": rho, "arrival_rate_per_s": rho * rate, "requests": len(specs),
                       "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                       "mean_ms": float(lat.mean() * 1e3), "throughput_requests_per_s": len(specs) / wall_l,
                       "throughput_units_per_s": units / wall_l, "per_lattice": per_L,
                       "slowdown_p50": float(np.percentile(slow, 50)), "slowdown_p99": float(np.percentile(slow, 99))})
        log(f"[serve]   p50 {levels[-1]['p50_ms']:.1f} ms  p99 {levels[-1]['p99_ms']:.1f} ms")
    sv.close()
    res = {
        "metric": "contracted site*momenta/s (spectator+insertion)",
        "value": value,
        "unit": "site*momenta/s",
        "n_gpus": 1,
        "steps": n_sat,
        "warmup": len(warm),
        "ms_per_step": wall * 1e3 / n_sat,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "bf16x2": "f32 contraction, bf16 hi+lo projection",
                  "f16x2": "f32 contraction, f16 hi+lo projection", "fac": "f32"}[proj],
        "data": "synthetic",
        "config": {"workload": "serving: Poisson arrivals; lattices 16^3x32:32^3x64:48^3x96:64^3x128 = 4:3:2:1, "
                               "|k|^2 ~ U{3..9}, meson:nucleon 1:1, N ~ U{1..16}, t_f-t_src ~ U{8..16}, local "
                               "insertion, combine on pairs p'=q or p'=0; one step = one request of the saturated "
                               "closed batch",
                   "lattices": lattices, "arena_gib": args.arena_gib, "step_mib": args.step_mib,
                   "max_active": args.max_active, "step_work": args.step_work, "saturation_requests": n_sat},
        "latency_ms": {"p50": levels[-1]["p50_ms"] if levels else None,
                       "p99": levels[-1]["p99_ms"] if levels else None,
                       "at_rho": loads[-1] if loads else None},
        "saturation": {"requests_per_s": rate, "units_per_s": value,
                       "latency_p50_ms": float(np.percentile(lat_sat, 50) * 1e3),
                       "latency_p99_ms": float(np.percentile(lat_sat, 99) * 1e3)},
        "load_levels": levels,
        "kernels_ms": {kn: round(v["avg_ms"], 4) for kn, v in prof.items()},
        "kernel_launches": {kn: v["count"] for kn, v in prof.items()},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on served requests")
        res["cpu_baseline"] = serve_cpu_baseline(min(lattices), momenta)
    print(json.dumps(res), flush=True)


def serve_cpu_baseline(L, momenta, budget_s=12.0):
    """The FP64 oracle on whole requests of the seeded serving draw on the
    smallest resident lattice, one after the other until about budget_s of
    host time: spectator(s) at t_f, insertion(s) on every timeslice from t_src
    to t_f, and the combines, as the server computes them.  Inputs are drawn
    on the host with the pool's distributions and shapes."""
    import c3pt_synth as syn
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    T = SERVE_LATTICES[L]
    Ls = (L, L, L)
    specs = [sp for sp in serve_draw(400, [L], seed=3)]
    Gu = {t: syn.round_to_c64(syn.propagator_slice(Ls, 5, syn.FIELD_G3, t)) for t in range(T)}
    Gd = {t: syn.round_to_c64(syn.propagator_slice(Ls, 5, syn.FIELD_G1, t)) for t in range(T)}
    s_all = {t: syn.round_to_c64(syn.solution_slice(Ls, ServePool.N_MAX, 5, t)) for t in range(T)}
    eta_all = syn.round_to_c64(syn.z2z2_noise(Ls, ServePool.N_MAX, 5, 0))
    done, units, dt = 0, 0, 0.0
    for sp in specs:
        k = oracle.momenta(sp["n2"])
        N, r = sp["N"], sp["r"]
        taus = [(sp["t_src"] + j) % T for j in range(sp["n_tau"])]
        s = {t: s_all[t][:N] for t in taus}
        eta = eta_all[:N]
        pairs = pairs_diag_or_zero(len(k))
        t0 = time.perf_counter()
        if sp["kind"] == "nucleon":
            for G2, Gi in ((Gu, Gd), (Gd, Gu)):
                S = oracle.spectator_baryon(Gu[sp["t_f"]], G2[sp["t_f"]], eta, Ls, k, r=r)
                oracle.combine(S, oracle.insertion(Gi, s, taus, Ls, T, k, r=r), pairs=pairs)
        else:
            S = oracle.spectator_meson(Gu[sp["t_f"]], eta, Ls, k, r=r)
            oracle.combine(S, oracle.insertion(Gu, s, taus, Ls, T, k, r=r), pairs=pairs)
        dt += time.perf_counter() - t0
        units += serve_units(sp, momenta)
        done += 1
        if dt > budget_s:
            break
    return {"value": units / dt, "unit": "site*momenta/s", "cores": int(threads), "kind": "oracle",
            "sample": (f"FP64 numpy oracle on {done} whole requests of the seeded serving draw on {L}^3x{T} "
                       f"(spectators, insertions on every timeslice t_src..t_f, combines); {units:.3g} units "
                       f"in {dt:.1f} s"), "seconds": dt}



def cpu_baseline(W, k, n_slices):
    """Time the FP64 oracle on a bounded sample of the same workload on the host."""
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    units, dt, what = W.cpu_sample(k, n_slices)
    return {"value": units / dt, "unit": "site*momenta/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{what}; {units:.3g} units in {dt:.1f} s", "seconds": dt}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "serve":
        return serve_main(args)
    import torch
    import c3pt_synth as syn
    import paper_1711_02384_amd as c3pt

    W = WORKLOADS[args.workload](args)
    if args.steps is None:
        args.steps = W.default_steps
    if args.warmup is None:
        args.warmup = W.default_warmup
    proj = args.proj or W.default_proj
    if W.dtype == "c128":
        proj = "f64"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    k = c3pt.momentum_list(W.n2)
    n_mom = len(k)
    proj_flag = {"f64": c3pt.PROJ_NATIVE, "f32": c3pt.PROJ_NATIVE, "bf16x2": c3pt.PROJ_SPLIT_BF16,
                 "f16x2": c3pt.PROJ_SPLIT_F16, "fac": c3pt.PROJ_FACTORED, "fs16": c3pt.PROJ_FACTORED_F16,
                 "fsbf16": c3pt.PROJ_FACTORED_BF16}[proj]
    mode = c3pt.MODE.get(proj, c3pt.MODE["fac"])
    batched = isinstance(W, Batch64)
    geom = c3pt.Geom((1, 1, 1) if batched else W.L, 1 if batched else W.T, proj=proj_flag)
    W.proj_flag = proj_flag
    log(f"[bench] generating inputs for {W.name}")
    t0 = time.perf_counter()
    W.setup(c3pt, syn, dev, geom, k)
    torch.cuda.synchronize()
    log(f"[bench] inputs resident in HBM ({time.perf_counter() - t0:.1f} s)")
    cls = c3pt.mt_class(n_mom, proj == "f64")

    tuning = None
    if args.tune:
        from paper_1711_02384_amd import autotune
        cases = [{"kind": kn, "mode": mode, "mt_class": cls, "call": fn} for kn, fn in W.calls()]
        tuning = autotune.tune(cases, reps=3, log=log)
        if batched and proj == "fac":
            # the batch's own kernels: 32-site tiles and chunk size per producer kind
            tb = autotune.tune_recorded(["spectator_meson", "spectator_baryon", "insertion"], "batchfac", cls,
                                        W.record, W.step, reps=3, log=log)
            tuning["entries"] += tb["entries"]
        elif batched:
            W.record()
        if args.tune_out:
            autotune.save(tuning, args.tune_out)
    for _ in range(args.warmup):
        W.step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    log(f"[bench] timing {args.steps} steps")
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        W.step()
        b.record(stream)
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    lat = [a.elapsed_time(b) for a, b in evs]
    log("[bench] step times (ms): " + " ".join(f"{x:.2f}" for x in lat))
    lat = sorted(lat)
    ms_per_step = (t_end - t_start) * 1e3 / args.steps
    units = W.units(n_mom)
    value = units / (ms_per_step * 1e-3)

    # per-kernel durations: HIP events around every library launch on its
    # stream, over separate profiled steps (a batch then runs its recorded
    # launches one by one instead of the graph)
    prof_steps = max(1, min(args.steps, 3))
    log(f"[bench] profiling {prof_steps} steps")
    if hasattr(W, "one_stream"):
        W.one_stream = True    # per-kernel durations on one stream, without sharing
    c3pt.profile_read(reset=True)
    c3pt.profile_enable(True)
    for _ in range(prof_steps):
        W.step()
    torch.cuda.synchronize()
    c3pt.profile_enable(False)
    if hasattr(W, "one_stream"):
        W.one_stream = False
    prof = c3pt.profile_read(reset=True)

    if batched:
        # dominant = the projection kernel kind with the most time per step
        kf = {kn: f for kn, f in W.kernel_flops().items() if kn in prof and f > 0}
        kname = max(kf, key=lambda kn: prof[kn]["total_ms"])
        launches = prof[kname]["count"] / prof_steps
        flops = kf[kname] / launches
        kms = prof[kname]["total_ms"] / prof[kname]["count"]
    else:
        dom = W.dominant(n_mom, proj)
        if isinstance(dom, dict):
            cand = {kn: f for kn, f in dom.items() if kn in prof}
            kname = max(cand, key=lambda kn: prof[kn]["total_ms"]) if cand else next(iter(dom))
            flops = dom[kname]
        else:
            kname, flops = dom
        kms = prof.get(kname, {}).get("avg_ms", float("nan"))
    roofline = roofline_entry(kname, flops, kms, proj, measured_traffic(args.workload, proj, kname, getattr(W, "n_ops", 1)))
    if roofline["traffic"] is not None:
        roofline["traffic_note"] = ("HBM bytes per call of the timed kernel (all its launches) from rocprofv3 "
                                    "FETCH_SIZE x 2 + WRITE_SIZE x 1 (copy-calibrated), measured on these kernel "
                                    "sources")
        roofline["hbm_frac"] = round(roofline["traffic"] / (kms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)
    mf = getattr(W, "mfma_flops", lambda kn, pj: None)(kname, proj)
    if mf is not None:
        roofline["mfma_frac"] = round(mf / (kms * 1e-3) / 1e12 / PEAK_MFMA_F16, 4)
        roofline["mfma_note"] = ("MFMA flops the kernel issues (16x16x32 16-bit products, 3 per hi+lo term) "
                                 "per launch over its average duration, against the dense FP16/BF16 peak")

    plain = None
    plain_proj = getattr(W, "plain_proj", None)
    if not batched and plain_proj and plain_proj != proj:
        # the plain FP32 form of the same step, timed the same way
        pflag = {"fac": c3pt.PROJ_FACTORED, "f32": c3pt.PROJ_NATIVE}[plain_proj]
        head_geom = W.geom
        W.geom = c3pt.Geom(W.L, W.T, proj=pflag)
        n_plain = max(3, min(args.steps, 10))
        log(f"[bench] timing {n_plain} steps of the plain form ({plain_proj})")
        # timed like the headline: warm-up steps, then wall clock over the
        # steps, with per-step events for the median
        for _ in range(max(1, args.warmup)):
            W.step()
        torch.cuda.synchronize()
        pevs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_plain)]
        t0 = time.perf_counter()
        for a, b in pevs:
            a.record(stream)
            W.step()
            b.record(stream)
        torch.cuda.synchronize()
        pms = (time.perf_counter() - t0) * 1e3 / n_plain
        plat = sorted(a.elapsed_time(b) for a, b in pevs)
        plain = {"proj": plain_proj, "ms_per_step": pms, "p50_ms": plat[len(plat) // 2],
                 "value": units / (pms * 1e-3),
                 "form": "the same step with the FP32 factored projection (FP32 contraction on the VALU)",
                 "speedup_of_headline": plat[len(plat) // 2] / lat[len(lat) // 2],
                 "speedup_note": "ratio of the median step times (HIP events) of the two forms"}
        W.plain_outputs = {kn: fn().cpu().numpy() for kn, fn in getattr(W, "sample_outputs", {}).items()}
        W.geom = head_geom
        W.step()
        torch.cuda.synchronize()
    plain_dense = None
    if batched and W.plain:
        # the same jobs as plain per-call launches: first with the batch's own
        # projection (isolates batching), then with the dense FP32 projection
        forms = [(proj, proj_flag, f"one c3pt_* call per job and per combine, the batch's own ({proj}) "
                                   "projection, no graph")]
        if proj != "f32":
            forms.append(("f32", c3pt.PROJ_NATIVE, "one c3pt_* call per job and per combine, dense FP32 MFMA "
                                                   "projection, no graph"))
        W.plain_outputs = {}
        got = []
        for pj, pflag, what in forms:
            log(f"[bench] timing the same jobs as plain per-call launches ({pj})")
            W.plain_step(pflag)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            W.plain_step(pflag)
            b.record(stream)
            torch.cuda.synchronize()
            pms = a.elapsed_time(b)
            # per-kernel time of one profiled plain step, beside the batch's kernels_ms
            c3pt.profile_read(reset=True)
            c3pt.profile_enable(True)
            W.plain_step(pflag)
            torch.cuda.synchronize()
            c3pt.profile_enable(False)
            pprof = c3pt.profile_read(reset=True)
            got.append({"value": units / (pms * 1e-3), "ms_per_step": pms, "proj": pj, "form": what,
                        "batched_speedup": pms / ms_per_step,
                        "kernels_ms_per_step": {kn: round(v["total_ms"], 3) for kn, v in pprof.items()}})
            W.plain_outputs[f"{pj} per call"] = {kn: fn().cpu().numpy()
                                                 for kn, fn in getattr(W, "sample_outputs", {}).items()}
        plain = got[0]
        plain_dense = got[1] if len(got) > 1 else None
        # the batch's own outputs again, for its accuracy below
        W.step()
        torch.cuda.synchronize()
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
        "dtype": {"f64": "f64", "f32": "f32", "bf16x2": "f32 contraction, bf16 hi+lo projection",
                  "f16x2": "f32 contraction, f16 hi+lo projection", "fac": "f32",
                  "fs16": "f16 hi+lo MFMA (contraction folded into the projection), f32 accumulation",
                  "fsbf16": "bf16 hi+lo MFMA (contraction folded into the projection), f32 accumulation"}[proj],
        "data": "synthetic",
        "config": W.config(n_mom),
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "component_rate": {"projected_complex_values_per_s": W.components(n_mom) / (ms_per_step * 1e-3)},
        "kernels_ms": {kn: round(v["avg_ms"], 4) for kn, v in prof.items()},
        "kernels_ms_per_step": {kn: round(v["total_ms"] / prof_steps, 3) for kn, v in prof.items()},
        "kernel_launches": {kn: v["count"] for kn, v in prof.items()},
        "kernels_note": ("per-call durations (HIP events on the launch stream) over "
                         f"{prof_steps} separate profiled steps"
                         + (" run on one stream" if hasattr(W, "one_stream") else "")),
        "roofline": roofline,
        "variants": {kn: c3pt.get_variant(c3pt.KIND[kn], mode, cls)
                     for kn in ("spectator_meson", "spectator_baryon", "insertion")},
    }
    if plain is not None:
        res["plain_form"] = plain
    if plain_dense is not None:
        res["plain_form_dense"] = plain_dense
    if tuning is not None:
        res["tuning"] = tuning["entries"]
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on a host sample")
        res["cpu_baseline"] = cpu_baseline(W, k, args.cpu_slices)
        acc = sample_accuracy(W, proj, plain)
        if acc:
            res["accuracy"] = acc
    print(json.dumps(res), flush=True)


def rel_err(got, want) -> float:
    """The larger of ||got - want||_F / ||want||_F and max|got - want| / max|want|."""
    d = (np.asarray(got) - np.asarray(want)).ravel()
    w = np.asarray(want).ravel()
    return float(max(np.linalg.norm(d) / np.linalg.norm(w), np.abs(d).max() / np.abs(w).max()))


def sample_accuracy(W, proj, plain):
    """Error of the headline form (and of the plain form, when timed) against
    the FP64 oracle on the outputs the CPU-baseline sample computed; inputs
    are the same seeded values, rounded to complex64 for both."""
    ref = getattr(W, "oracle_ref", None)
    if not ref:
        return None
    out = {"metric": "max(||d||_F/||ref||_F, max|d|/max|ref|) per part", proj: {}}
    for kn, fn in W.sample_outputs.items():
        out[proj][kn] = rel_err(fn().cpu().numpy(), ref[kn])
    po = getattr(W, "plain_outputs", {})
    if po and all(isinstance(v, dict) for v in po.values()):
        # several plain forms, keyed by name (captured when each ran)
        for name, outs in po.items():
            out[name] = {kn: rel_err(v, ref[kn]) for kn, v in outs.items()}
    elif plain is not None:
        # the plain form's outputs were captured when it ran
        out[plain["proj"]] = {kn: rel_err(v, ref[kn]) for kn, v in po.items()}
    return out


if __name__ == "__main__":
    main()
