"""Parity of the factored projection (C3PT_PROJ_FACTORED) with the FP64 oracle.

Cases cover both kernel forms (variant 0: every x3 plane its own chunk;
variant 1: chunks of planes summed in registers), 32-site tiles (x1 rows of
32) and 16-site tiles (rows of 24, and rows shorter than a tile), complex128
(FP64 MFMA, 1e-12) and complex64 (FP32 MFMA, 1e-5), several FP64 momentum
groups, a source off the origin, and a momentum list with more distinct k1
than the kernel holds (that group runs on the dense kernel).  The |k|^2 <= 9
list has a k1 with seven distinct k2, more than one stage-1 slot keeps: it is
split over two slots.  Rows of five 16-site segments (more than the stage-1
operands kept in LDS) and an extent of 1 are covered too.
"""
import numpy as np
import pytest

import oracle
from helpers import Workload, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _t(a, reduced):
    return torch.from_numpy(np.ascontiguousarray(a.astype(np.complex64 if reduced else np.complex128))).cuda()


CASES = [
    # L, T, taus, N, n2, reduced, r
    ((32, 4, 3), 6, [0, 2], 2, 3, True, (5, 1, 2)),      # 32-site tiles
    ((24, 3, 2), 6, [1, 5], 2, 6, True, (0, 2, 1)),      # 16-site tiles, second segment ragged
    ((6, 5, 4), 6, [0, 3], 1, 3, True, (1, 0, 3)),       # rows shorter than a tile
    ((8, 8, 8), 6, [2], 1, 3, False, (3, 5, 1)),         # complex128, one FP64 group
    ((6, 5, 4), 6, [0, 4], 2, 5, False, (0, 1, 2)),      # complex128, two FP64 groups (57 momenta)
    ((12, 8, 6), 4, [0, 2], 1, 9, True, (3, 1, 2)),      # |k|^2 <= 9: k1 = 0 has seven k2, two stage-1 slots
    ((72, 3, 2), 4, [1], 1, 3, True, (0, 1, 1)),         # five row segments: stage-1 operands refilled per tile
    ((80, 2, 3), 4, [0, 3], 1, 2, False, (7, 1, 0)),     # complex128, five segments, last one ragged
    ((6, 1, 5), 4, [2], 2, 3, True, (2, 0, 4)),          # extent 1 in x2: neighbours are the site itself
]


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_factored_parts(case, variant):
    import paper_1711_02384_amd as c3pt
    L, T, taus, N, n2, reduced, r = CASES[case]
    tol = 1e-5 if reduced else 1e-12
    k = c3pt.momentum_list(n2)
    w = Workload(L, T, N, cfg=40 + case, taus=taus, links=True, reduced=reduced, second_prop=True)
    geom = c3pt.Geom(L, T, r=r, proj=c3pt.PROJ_FACTORED)
    mode = c3pt.MODE["fac"]
    for kind in (0, 1, 2):
        for cls in range(4):
            c3pt.set_variant(kind, mode, cls, variant)
    try:
        S = c3pt.spectator_meson(_t(w.G1, reduced), _t(w.eta, reduced), k, geom).cpu().numpy()
        SB = c3pt.spectator_baryon(_t(w.G1, reduced), _t(w.G1b, reduced), _t(w.eta, reduced), k, geom).cpu().numpy()
        G = {t: _t(v, reduced) for t, v in w.G3.items()}
        s = {t: _t(v, reduced) for t, v in w.s.items()}
        U = {t: _t(v, reduced) for t, v in w.U.items()}
        I = c3pt.insertion(G, s, taus, k, geom, U_t=U, n_ops=5).cpu().numpy()
        torch.cuda.synchronize()
    finally:
        for kind in (0, 1, 2):
            for cls in range(4):
                c3pt.set_variant(kind, mode, cls, 0)
    S_o = oracle.spectator_meson(w.G1, w.eta, L, k, r=r)
    SB_o = oracle.spectator_baryon(w.G1, w.G1b, w.eta, L, k, r=r)
    I_o = oracle.insertion(w.G3, w.s, taus, L, T, k, r=r, U_t=w.U, n_ops=5)
    es, eb = rel_err(S, S_o), rel_err(SB, SB_o)
    ei = [rel_err(I[:, j, op], I_o[:, j, op]) for j in range(len(taus)) for op in range(5)]
    _say(f"factored case {case} variant {variant} L={L}: meson {es:.2e} baryon {eb:.2e} insertion max {max(ei):.2e}")
    assert es < tol and eb < tol and max(ei) < tol


def test_factored_falls_back_for_wide_momentum_lists():
    """Nine distinct k1 values exceed one stage-1 row tile: the group runs on the dense kernel."""
    import paper_1711_02384_amd as c3pt
    L, T = (20, 4, 3), 4
    k = np.array([[k1, 0, 0] for k1 in range(-4, 5)] + [[0, 1, 1], [1, 1, 0]], dtype=np.int32)
    w = Workload(L, T, 1, cfg=49, taus=[1], reduced=True)
    geom = c3pt.Geom(L, T, r=(2, 1, 0), proj=c3pt.PROJ_FACTORED)
    S = c3pt.spectator_meson(_t(w.G1, True), _t(w.eta, True), k, geom).cpu().numpy()
    I = c3pt.insertion({1: _t(w.G3[1], True)}, {1: _t(w.s[1], True)}, [1], k, geom).cpu().numpy()
    assert rel_err(S, oracle.spectator_meson(w.G1, w.eta, L, k, r=(2, 1, 0))) < 1e-5
    assert rel_err(I, oracle.insertion(w.G3, w.s, [1], L, T, k, r=(2, 1, 0))) < 1e-5


def test_factored_is_deterministic():
    import paper_1711_02384_amd as c3pt
    L, T = (32, 6, 5), 4
    k = c3pt.momentum_list(6)
    w = Workload(L, T, 2, cfg=50, taus=[0, 1], reduced=True)
    geom = c3pt.Geom(L, T, proj=c3pt.PROJ_FACTORED)
    G = {t: _t(v, True) for t, v in w.G3.items()}
    s = {t: _t(v, True) for t, v in w.s.items()}
    a = c3pt.insertion(G, s, [0, 1], k, geom)
    b = c3pt.insertion(G, s, [0, 1], k, geom)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
