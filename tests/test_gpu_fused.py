"""Parity of the split-precision fused projection (C3PT_PROJ_FACTORED_F16 and
_BF16: the colour contraction folded into the x1 stage of the factored
projection on hi+lo 16-bit MFMA, FP32 accumulation) with the FP64 oracle.

Cases: 32-site tiles (rows of 32, 64: one and two segments), rows of 48 (one
48-site tile under variant 5), 16-site tiles
(rows of 24 and 72: ragged last segment, five segments; rows of 6 shorter
than a tile), an extent of 1 in x2 (the derivative's neighbours are the site
itself), an odd noise count (the second block of the last pair is empty), a
source off the origin, the |k|^2 <= 9 list (a k1 with seven k2 over two
stage-1 slots; five noise vectors), timeslices wrapping around T.  Every part: meson spectator,
nucleon spectator, insertion with the local operator alone and with the four
D_nu (whose shifted parts are combined in the FP64 reduction).  Inputs are
complex64; the oracle gets the same values in FP64.  Tolerance 1e-5 (rel_err:
Frobenius and max-element ratios), the reduced-precision bar.
"""
import numpy as np
import pytest

import oracle
from helpers import Workload, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
TOL = 1e-5


def _say(msg):
    print(msg, flush=True)


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a.astype(np.complex64))).cuda()


CASES = [
    # L, T, taus, N, n2, r
    ((32, 4, 3), 6, [0, 2], 2, 3, (5, 1, 2)),
    ((24, 3, 2), 6, [1, 5], 3, 6, (0, 2, 1)),
    ((6, 5, 4), 6, [0, 3], 1, 3, (1, 0, 3)),
    ((12, 8, 6), 4, [0, 3], 5, 9, (3, 1, 2)),
    ((72, 3, 2), 4, [1], 1, 3, (0, 1, 1)),
    ((6, 1, 5), 4, [2], 2, 3, (2, 0, 4)),
    ((64, 2, 2), 4, [0, 3], 2, 8, (1, 1, 1)),
    ((48, 3, 2), 4, [0, 3], 4, 8, (7, 2, 1)),
]


def _set_fused_variant(c3pt, v):
    for kind in (0, 1, 2):
        for cls in range(4):
            c3pt.set_variant(kind, c3pt.MODE["fs16"], cls, v)


@pytest.mark.parametrize("prec,variant", [("f16", 0), ("f16", 1), ("f16", 2), ("f16", 3), ("f16", 4), ("f16", 5),
                                          ("bf16", 0), ("bf16", 3), ("bf16", 4), ("bf16", 5)])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_fused_parts(case, prec, variant):
    """variant 0 splits the propagator tiles in the kernel, 1 in a pass first, 2 with one
    column block per workgroup, 3 in the kernel with one column block per workgroup, 4 in
    the kernel with three column blocks per workgroup (16-site tiles; N = 4 and 5 run the
    last one or two noise vectors as a two-block launch, N = 1 and 2 as that launch
    alone; 32-site tiles and the derivative slots run as 0),
    5 as 0 with 48-site tiles for the local insertion when L1 = 48 (elsewhere as 0)."""
    import paper_1711_02384_amd as c3pt
    L, T, taus, N, n2, r = CASES[case]
    k = c3pt.momentum_list(n2)
    w = Workload(L, T, N, cfg=60 + case, taus=taus, links=True, reduced=True, second_prop=True)
    proj = c3pt.PROJ_FACTORED_F16 if prec == "f16" else c3pt.PROJ_FACTORED_BF16
    geom = c3pt.Geom(L, T, r=r, proj=proj)
    _say(f"fused {prec} variant {variant} case {case} L={L} N={N} n2={n2}: GPU")
    _set_fused_variant(c3pt, variant)
    try:
        S = c3pt.spectator_meson(_t(w.G1), _t(w.eta), k, geom).cpu().numpy()
        SB = c3pt.spectator_baryon(_t(w.G1), _t(w.G1b), _t(w.eta), k, geom).cpu().numpy()
        G = {t: _t(v) for t, v in w.G3.items()}
        s = {t: _t(v) for t, v in w.s.items()}
        U = {t: _t(v) for t, v in w.U.items()}
        I1 = c3pt.insertion(G, s, taus, k, geom, n_ops=1).cpu().numpy()
        I5 = c3pt.insertion(G, s, taus, k, geom, U_t=U, n_ops=5).cpu().numpy()
        torch.cuda.synchronize()
    finally:
        _set_fused_variant(c3pt, 0)
    S_o = oracle.spectator_meson(w.G1, w.eta, L, k, r=r)
    SB_o = oracle.spectator_baryon(w.G1, w.G1b, w.eta, L, k, r=r)
    I_o = oracle.insertion(w.G3, w.s, taus, L, T, k, r=r, U_t=w.U, n_ops=5)
    es, eb = rel_err(S, S_o), rel_err(SB, SB_o)
    e1 = max(rel_err(I1[:, j, 0], I_o[:, j, 0]) for j in range(len(taus)))
    e5 = [rel_err(I5[:, j, op], I_o[:, j, op]) for j in range(len(taus)) for op in range(5)]
    _say(f"fused {prec} variant {variant} case {case}: meson {es:.2e} nucleon {eb:.2e} local {e1:.2e} with D_nu max {max(e5):.2e}")
    assert es < TOL and eb < TOL and e1 < TOL and max(e5) < TOL


def test_fused_is_deterministic_and_matches_fp32_factored():
    """Repeated calls are bit-identical; the FP32 factored form agrees within the bar."""
    import paper_1711_02384_amd as c3pt
    L, T = (32, 6, 5), 4
    k = c3pt.momentum_list(6)
    w = Workload(L, T, 2, cfg=70, taus=[0, 1], links=True, reduced=True)
    G = {t: _t(v) for t, v in w.G3.items()}
    s = {t: _t(v) for t, v in w.s.items()}
    U = {t: _t(v) for t, v in w.U.items()}
    geom = c3pt.Geom(L, T, proj=c3pt.PROJ_FACTORED_F16)
    a = c3pt.insertion(G, s, [0, 1], k, geom, U_t=U, n_ops=5)
    b = c3pt.insertion(G, s, [0, 1], k, geom, U_t=U, n_ops=5)
    f = c3pt.insertion(G, s, [0, 1], k, c3pt.Geom(L, T, proj=c3pt.PROJ_FACTORED), U_t=U, n_ops=5)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert rel_err(a.cpu().numpy(), f.cpu().numpy()) < TOL


def test_fused_two_momentum_groups():
    """A momentum list of more than 128 momenta (|k|^2 <= 10: 147) runs as two
    groups, each with its own factor plan; every part against the oracle."""
    import paper_1711_02384_amd as c3pt
    L, T, taus, N, r = (12, 8, 6), 4, [0, 3], 2, (3, 1, 2)
    k = c3pt.momentum_list(10)
    assert len(k) > 128
    w = Workload(L, T, N, cfg=71, taus=taus, links=True, reduced=True, second_prop=True)
    geom = c3pt.Geom(L, T, r=r, proj=c3pt.PROJ_FACTORED_F16)
    _say(f"fused f16 two groups: {len(k)} momenta")
    S = c3pt.spectator_meson(_t(w.G1), _t(w.eta), k, geom).cpu().numpy()
    SB = c3pt.spectator_baryon(_t(w.G1), _t(w.G1b), _t(w.eta), k, geom).cpu().numpy()
    G = {t: _t(v) for t, v in w.G3.items()}
    s = {t: _t(v) for t, v in w.s.items()}
    U = {t: _t(v) for t, v in w.U.items()}
    I5 = c3pt.insertion(G, s, taus, k, geom, U_t=U, n_ops=5).cpu().numpy()
    torch.cuda.synchronize()
    S_o = oracle.spectator_meson(w.G1, w.eta, L, k, r=r)
    SB_o = oracle.spectator_baryon(w.G1, w.G1b, w.eta, L, k, r=r)
    I_o = oracle.insertion(w.G3, w.s, taus, L, T, k, r=r, U_t=w.U, n_ops=5)
    es, eb = rel_err(S, S_o), rel_err(SB, SB_o)
    e5 = max(rel_err(I5[:, j, op], I_o[:, j, op]) for j in range(len(taus)) for op in range(5))
    _say(f"fused f16 two groups: meson {es:.2e} nucleon {eb:.2e} insertion max {e5:.2e}")
    assert es < TOL and eb < TOL and e5 < TOL


def test_fused_three_blocks_remainder_of_one_and_two_groups():
    """Variant 4 (three blocks per workgroup) with N = 7 (groups of three, then
    one vector in a two-block launch with its second block empty) and a
    147-momentum list (two momentum groups, each planned with at most five
    pairs per k1 slot); every part against the oracle."""
    import paper_1711_02384_amd as c3pt
    L, T, taus, N, r = (12, 8, 6), 4, [1, 2], 7, (2, 3, 1)
    k = c3pt.momentum_list(10)
    w = Workload(L, T, N, cfg=72, taus=taus, links=True, reduced=True, second_prop=True)
    geom = c3pt.Geom(L, T, r=r, proj=c3pt.PROJ_FACTORED_F16)
    _say(f"fused f16 variant 4, N = {N}, {len(k)} momenta")
    _set_fused_variant(c3pt, 4)
    try:
        S = c3pt.spectator_meson(_t(w.G1), _t(w.eta), k, geom).cpu().numpy()
        SB = c3pt.spectator_baryon(_t(w.G1), _t(w.G1b), _t(w.eta), k, geom).cpu().numpy()
        G = {t: _t(v) for t, v in w.G3.items()}
        s = {t: _t(v) for t, v in w.s.items()}
        I1 = c3pt.insertion(G, s, taus, k, geom, n_ops=1).cpu().numpy()
        torch.cuda.synchronize()
    finally:
        _set_fused_variant(c3pt, 0)
    S_o = oracle.spectator_meson(w.G1, w.eta, L, k, r=r)
    SB_o = oracle.spectator_baryon(w.G1, w.G1b, w.eta, L, k, r=r)
    I_o = oracle.insertion(w.G3, w.s, taus, L, T, k, r=r, n_ops=1)
    es, eb = rel_err(S, S_o), rel_err(SB, SB_o)
    e1 = max(rel_err(I1[:, j, 0], I_o[:, j, 0]) for j in range(len(taus)))
    _say(f"fused f16 variant 4, N = {N}: meson {es:.2e} nucleon {eb:.2e} insertion {e1:.2e}")
    assert es < TOL and eb < TOL and e1 < TOL
