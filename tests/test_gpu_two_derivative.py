"""Two-derivative insertion operators (n_ops = 21: ops 5 + 4 rho + nu = D_nu D_rho;
n_ops = 37: also ops 21 + 4 mu + nu = <->D_mu <->D_nu)
on the factored projection against the FP64 oracle (pinned by the doubly
applied matrix-form derivative traced as Eq. (1) and by the unit-link
identities).  complex128 at 1e-12, complex64 at 1e-5; timeslices at both ends
of the periodic time direction (G needed on tau +- 2), ragged rows, a source
off the origin; argument errors."""
import numpy as np
import pytest

import c3pt_synth as syn
import oracle
from helpers import rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _inputs(L, T, N, taus, cfg, reduced, wide_s=False):
    cast = syn.round_to_c64 if reduced else (lambda a: a)
    gsl = sorted({(t + d) % T for t in taus for d in (-2, -1, 0, 1, 2)})
    usl = sorted({(t + d) % T for t in taus for d in (-2, -1, 0, 1)})
    G = {t: cast(syn.propagator_slice(L, cfg, syn.FIELD_G3, t)) for t in gsl}
    s = {t: cast(syn.solution_slice(L, N, cfg, t)) for t in (gsl if wide_s else taus)}
    U = {t: cast(syn.link_slice(L, cfg, t)) for t in usl}
    return G, s, U


def _dev(d, reduced):
    dt = np.complex64 if reduced else np.complex128
    return {t: torch.from_numpy(np.ascontiguousarray(v.astype(dt))).cuda() for t, v in d.items()}


CASES = [
    # L, T, taus, N, n2, reduced, r
    ((32, 4, 3), 8, [0, 7], 2, 3, True, (5, 1, 2)),     # 32-site tiles for the local part, both time ends
    ((6, 5, 4), 7, [1, 4], 2, 3, True, (1, 0, 3)),      # rows shorter than a tile
    ((6, 5, 4), 6, [5, 2], 1, 5, False, (0, 1, 2)),     # complex128, two FP64 momentum groups
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_two_derivatives_match_oracle(case):
    import paper_1711_02384_amd as c3pt
    L, T, taus, N, n2, reduced, r = CASES[case]
    tol = 1e-5 if reduced else 1e-12
    _say(f"two-derivative case {case}: L={L} T={T} taus={taus} N={N} |k|^2<={n2} reduced={reduced}")
    k = c3pt.momentum_list(n2)
    G, s, U = _inputs(L, T, N, taus, 140 + case, reduced)
    geom = c3pt.Geom(L, T, r=r, proj=c3pt.PROJ_FACTORED)
    got = c3pt.insertion(_dev(G, reduced), _dev(s, reduced), taus, k, geom, U_t=_dev(U, reduced), n_ops=21)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    want = oracle.insertion(G, s, taus, L, T, k, r=r, U_t=U, n_ops=21)
    errs = [rel_err(got[:, :, op], want[:, :, op]) for op in range(21)]
    _say(f"   max error {max(errs):.1e} (op {int(np.argmax(errs))})")
    assert max(errs) < tol


CASES37 = [
    ((6, 5, 4), 7, [0, 3], 2, 3, True, (1, 0, 3)),      # complex64, a timeslice at the time boundary
    ((5, 4, 4), 6, [4], 1, 3, False, (0, 2, 1)),        # complex128
]


@pytest.mark.parametrize("case", range(len(CASES37)))
def test_symmetrized_two_derivatives_match_oracle(case):
    import paper_1711_02384_amd as c3pt
    L, T, taus, N, n2, reduced, r = CASES37[case]
    tol = 1e-5 if reduced else 1e-12
    _say(f"symmetrized two-derivative case {case}: L={L} T={T} taus={taus} N={N} reduced={reduced}")
    k = c3pt.momentum_list(n2)
    G, s, U = _inputs(L, T, N, taus, 160 + case, reduced, wide_s=True)
    geom = c3pt.Geom(L, T, r=r, proj=c3pt.PROJ_FACTORED)
    got = c3pt.insertion(_dev(G, reduced), _dev(s, reduced), taus, k, geom, U_t=_dev(U, reduced), n_ops=37)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    want = oracle.insertion(G, s, taus, L, T, k, r=r, U_t=U, n_ops=37)
    errs = [rel_err(got[:, :, op], want[:, :, op]) for op in range(37)]
    _say(f"   max error {max(errs):.1e} (op {int(np.argmax(errs))})")
    assert max(errs) < tol


def test_two_derivatives_reject_bad_arguments():
    import paper_1711_02384_amd as c3pt
    _say("two-derivative argument checks")
    L, T, N = (4, 4, 4), 8, 1
    G, s, U = _inputs(L, T, N, [3], 150, False)
    k = c3pt.momentum_list(1)
    fac = c3pt.Geom(L, T, proj=c3pt.PROJ_FACTORED)
    with pytest.raises(c3pt.C3ptError):          # dense projection
        c3pt.insertion(_dev(G, False), _dev(s, False), [3], k, c3pt.Geom(L, T), U_t=_dev(U, False), n_ops=21)
    G_missing = {t: v for t, v in G.items() if t != 5}
    with pytest.raises(c3pt.C3ptError):          # G(tau + 2) missing
        c3pt.insertion(_dev(G_missing, False), _dev(s, False), [3], k, fac, U_t=_dev(U, False), n_ops=21)
    U_missing = {t: v for t, v in U.items() if t != 1}
    with pytest.raises(c3pt.C3ptError):          # U(tau - 2) missing
        c3pt.insertion(_dev(G, False), _dev(s, False), [3], k, fac, U_t=_dev(U_missing, False), n_ops=21)
