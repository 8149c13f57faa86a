"""The largest extent the ABI takes (C3PT_MAX_L = 256) in each direction, on
small volumes: every projection form (dense FP64 and FP32, factored FP32,
fused FP16 hi+lo) for the meson and nucleon spectators and the insertion with
the four derivatives, the combine, and smearing, against the FP64 oracle.
The phase and root tables, the factored kernels' row segments (sixteen
16-site or eight 32-site tiles per row) and the fused kernel's lattice-sized
LDS tables are at their largest here."""
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


LATTICES = [(256, 2, 2), (2, 256, 2), (3, 2, 256)]
FORMS = [("dense f64", 0, False), ("dense f32", 0, True), ("factored f32", 3, True), ("fused f16", 4, True)]


@pytest.mark.parametrize("form", range(len(FORMS)))
@pytest.mark.parametrize("lat", range(len(LATTICES)))
def test_max_extent(lat, form):
    import paper_1711_02384_amd as c3pt
    L = LATTICES[lat]
    name, proj, reduced = FORMS[form]
    tol = 1e-5 if reduced else 1e-12
    T, taus, N, r = 4, [0, 2], 2, (L[0] - 1, 1, L[2] // 2)
    k = c3pt.momentum_list(3)
    w = Workload(L, T, N, cfg=90 + lat, taus=taus, links=True, reduced=reduced, second_prop=True)
    geom = c3pt.Geom(L, T, r=r, proj=proj)
    _say(f"max extent L={L} {name}")
    S = c3pt.spectator_meson(_t(w.G1, reduced), _t(w.eta, reduced), k, geom)
    SB = c3pt.spectator_baryon(_t(w.G1, reduced), _t(w.G1b, reduced), _t(w.eta, reduced), k, geom)
    G = {t: _t(v, reduced) for t, v in w.G3.items()}
    s = {t: _t(v, reduced) for t, v in w.s.items()}
    U = {t: _t(v, reduced) for t, v in w.U.items()}
    I = c3pt.insertion(G, s, taus, k, geom, U_t=U, n_ops=5)
    C = c3pt.combine(S, I, pairs=[(0, 0), (5, 11)])
    torch.cuda.synchronize()
    S_o = oracle.spectator_meson(w.G1, w.eta, L, k, r=r)
    SB_o = oracle.spectator_baryon(w.G1, w.G1b, w.eta, L, k, r=r)
    I_o = oracle.insertion(w.G3, w.s, taus, L, T, k, r=r, U_t=w.U, n_ops=5)
    C_o = oracle.combine(S_o, I_o, pairs=[(0, 0), (5, 11)])
    errs = {"meson": rel_err(S.cpu().numpy(), S_o), "nucleon": rel_err(SB.cpu().numpy(), SB_o),
            "insertion": max(rel_err(I.cpu().numpy()[:, j, op], I_o[:, j, op]) for j in range(len(taus))
                             for op in range(5)),
            "combine": rel_err(C.cpu().numpy(), C_o)}
    _say("   " + "  ".join(f"{kk} {v:.2e}" for kk, v in errs.items()))
    for kk, v in errs.items():
        assert v < tol, (L, name, kk, v)


@pytest.mark.parametrize("lat", range(len(LATTICES)))
def test_max_extent_smearing(lat):
    import paper_1711_02384_amd as c3pt
    import c3pt_synth as syn
    L = LATTICES[lat]
    for reduced in (False, True):
        cast = syn.round_to_c64 if reduced else (lambda a: a)
        U = cast(syn.link_slice(L, 95 + lat, 0))
        f = cast(syn.solution_slice(L, 2, 95 + lat, 0))
        got = c3pt.smear_vectors(_t(f, reduced), _t(U, reduced), c3pt.Geom(L, 1), 0.25, 3)
        torch.cuda.synchronize()
        err = rel_err(got.cpu().numpy(), oracle.smear(f, U, L, 0.25, 3, 8, 1))
        _say(f"max extent smearing L={L} reduced={reduced}: {err:.2e}")
        assert err < (1e-5 if reduced else 1e-12)
