"""Shared test helpers: seeded workloads and error metrics (no method arithmetic)."""
from __future__ import annotations

import numpy as np

import c3pt_synth as syn


def rel_err(got, want) -> float:
    """The larger of ||got - want||_F / ||want||_F and max|got - want| / max|want|.

    The first is the tolerance metric per part and timeslice; the second
    catches an error confined to a few elements, which the Frobenius ratio
    averages away (it can be sqrt(size) times smaller)."""
    got = np.asarray(got)
    want = np.asarray(want)
    d = (got - want).ravel()
    den = np.linalg.norm(want.ravel())
    fro = np.linalg.norm(d) / (den if den > 0 else 1.0)
    amax = np.abs(want).max() if want.size else 0.0
    mx = (np.abs(d).max() if d.size else 0.0) / (amax if amax > 0 else 1.0)
    return float(max(fro, mx))


def per_slice_rel(got, want, axis_tau=1):
    """rel_err per insertion timeslice."""
    got = np.moveaxis(np.asarray(got), axis_tau, 0)
    want = np.moveaxis(np.asarray(want), axis_tau, 0)
    return [rel_err(g, w) for g, w in zip(got, want)]


class Workload:
    """Seeded inputs for one lattice: complex128 host arrays, plus the values a
    complex64 device buffer holds (promoted back) when reduced precision is used."""

    def __init__(self, L, T, n_noise, cfg=0, t_f=None, taus=(), links=False, reduced=False,
                 second_prop=False):
        self.L, self.T, self.N = tuple(L), int(T), int(n_noise)
        self.V3 = int(np.prod(L))
        self.t_f = (T // 2) if t_f is None else t_f
        self.taus = list(taus)
        need = set(self.taus)
        if links:
            for t in self.taus:
                need |= {(t + 1) % T, (t - 1) % T}
        cast = syn.round_to_c64 if reduced else (lambda a: a)
        self.G1 = cast(syn.propagator_slice(L, cfg, syn.FIELD_G1, self.t_f))
        self.G1b = cast(syn.propagator_slice(L, cfg, syn.FIELD_G3, 1000 + self.t_f)) if second_prop else None
        self.eta = cast(syn.z2z2_noise(L, n_noise, cfg, self.t_f))
        self.G3 = {t: cast(syn.propagator_slice(L, cfg, syn.FIELD_G3, t)) for t in sorted(need)}
        self.s = {t: cast(syn.solution_slice(L, n_noise, cfg, t)) for t in self.taus}
        self.U = None
        if links:
            ut = set(self.taus) | {(t - 1) % T for t in self.taus}
            self.U = {t: cast(syn.link_slice(L, cfg, t)) for t in sorted(ut)}
