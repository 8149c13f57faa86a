"""GPU parity: every entry point of libc3pt against the FP64 oracle.

Tolerances (relative Frobenius norm per part and timeslice):
* complex128 inputs (FP64 contraction and FP64 MFMA projection): 1e-12
* complex64 inputs (FP32 contraction, FP32 MFMA projection, FP64 chunk sums): 1e-5
The oracle is fed the values the device holds (complex64 inputs are rounded
on the host first), so the error measures the computation only.
"""
import numpy as np
import pytest

import c3pt_synth as syn
import oracle
from oracle import brute
from helpers import Workload, rel_err, per_slice_rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


def _lib():
    import paper_1711_02384_amd as c
    return c


def dev(a, reduced):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if reduced:
        t = t.to(torch.complex64)
    return t.cuda()


def _say(msg):
    print(msg, flush=True)


# ---------------------------------------------------------------------------
# Spectators
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("L,N,n2,reduced,r", [
    ((8, 8, 8), 1, 3, False, (0, 0, 0)),         # the 8^3 x 16 meson workload
    ((6, 5, 7), 3, 3, False, (2, 1, 5)),         # non-cubic, ragged site tail, source offset
    ((6, 5, 7), 2, 6, True, (1, 0, 3)),          # FP32, 81 momenta
    ((5, 5, 5), 2, 9, True, (0, 0, 0)),          # FP32, 123 momenta (two momentum groups)
    ((4, 4, 4), 1, 5, False, (3, 3, 3)),         # FP64, 57 momenta (two FP64 groups)
])
def test_spectator_meson(L, N, n2, reduced, r):
    c = _lib()
    _say(f"spectator_meson L={L} N={N} n2={n2} reduced={reduced}")
    w = Workload(L, 8, N, cfg=101, reduced=reduced)
    k = oracle.momenta(n2)
    got = c.spectator_meson(dev(w.G1, reduced), dev(w.eta, reduced), k, c.Geom(L, 8, r)).cpu().numpy()
    want = oracle.spectator_meson(w.G1, w.eta, L, k, r)
    err = rel_err(got, want)
    assert err < (TOL32 if reduced else TOL64), err


@pytest.mark.parametrize("L,N,n2,reduced", [
    ((4, 3, 5), 2, 3, False),
    ((6, 4, 4), 1, 6, True),
])
def test_spectator_baryon(L, N, n2, reduced):
    c = _lib()
    _say(f"spectator_baryon L={L} N={N} n2={n2} reduced={reduced}")
    w = Workload(L, 8, N, cfg=102, reduced=reduced, second_prop=True)
    k = oracle.momenta(n2)
    r = (1, 2, 0)
    got = c.spectator_baryon(dev(w.G1, reduced), dev(w.G1b, reduced), dev(w.eta, reduced), k,
                             c.Geom(L, 8, r)).cpu().numpy()
    want = oracle.spectator_baryon(w.G1, w.G1b, w.eta, L, k, r)
    err = rel_err(got, want)
    assert err < (TOL32 if reduced else TOL64), err


# ---------------------------------------------------------------------------
# Insertion
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("L,T,N,taus,n_ops,n2,reduced", [
    ((8, 8, 8), 16, 1, list(range(9)), 1, 3, False),      # the 8^3 x 16 meson workload
    ((4, 5, 6), 6, 2, [0, 2, 5], 5, 3, False),           # derivative ops, time wrap
    ((5, 4, 6), 6, 2, [5, 1], 5, 6, True),               # FP32 derivative ops
    ((3, 3, 4), 32, 1, list(range(1, 27)), 1, 2, True),  # > 24 timeslices: two launches
])
def test_insertion(L, T, N, taus, n_ops, n2, reduced):
    c = _lib()
    _say(f"insertion L={L} T={T} N={N} taus={taus} n_ops={n_ops} reduced={reduced}")
    w = Workload(L, T, N, cfg=103, taus=taus, links=(n_ops == 5), reduced=reduced)
    k = oracle.momenta(n2)
    r = (1, 0, 2)
    Gd = {t: dev(v, reduced) for t, v in w.G3.items()}
    sd = {t: dev(v, reduced) for t, v in w.s.items()}
    Ud = {t: dev(v, reduced) for t, v in w.U.items()} if w.U else None
    got = c.insertion(Gd, sd, taus, k, c.Geom(L, T, r), U_t=Ud, n_ops=n_ops).cpu().numpy()
    want = oracle.insertion(w.G3, w.s, taus, L, T, k, r, U_t=w.U, n_ops=n_ops)
    errs = per_slice_rel(got, want)
    assert max(errs) < (TOL32 if reduced else TOL64), errs
    for op in range(n_ops):
        assert rel_err(got[:, :, op], want[:, :, op]) < (TOL32 if reduced else TOL64)


# ---------------------------------------------------------------------------
# Combine
# ---------------------------------------------------------------------------
def test_combine_from_oracle_parts():
    c = _lib()
    _say("combine from oracle parts")
    rng = np.random.default_rng(7)
    N, n_p, n_q, n_tau, n_ops = 5, 4, 3, 2, 5
    S = syn.gaussian((N, n_p, 192), rng)
    SB = syn.gaussian((N, n_p, 3072), rng)
    I = syn.gaussian((N, n_tau, n_ops, n_q, 192), rng)
    w = rng.random(N)
    Sd, SBd, Id = (torch.from_numpy(x).cuda() for x in (S, SB, I))
    got = c.combine(Sd, Id, w=w).cpu().numpy()
    assert rel_err(got, oracle.combine(S, I, w=w)) < TOL64
    pairs = [(3, 2), (0, 0), (1, 2), (3, 2)]
    got = c.combine(SBd, Id, pairs=pairs, op_begin=1, op_end=4).cpu().numpy()
    assert rel_err(got, oracle.combine(SB, I, pairs=pairs, op_begin=1, op_end=4)) < TOL64
    got = c.combine(Sd, Id).cpu().numpy()   # default weights 1/N
    assert rel_err(got, oracle.combine(S, I)) < TOL64


def test_end_to_end_against_bruteforce_trace():
    """GPU spectator + insertion + combine against the direct evaluation of the
    three-point trace, Eq. (1), with the stochastic estimate of Eq. (5)."""
    c = _lib()
    _say("end to end vs brute force")
    L, T, N = (3, 2, 4), 4, 3
    w = Workload(L, T, N, cfg=104, t_f=3, taus=[0, 1, 2])
    kp = oracle.momenta(2)[:5]
    q = oracle.momenta(2)[3:9]
    r = (1, 1, 2)
    geom = c.Geom(L, T, r)
    S = c.spectator_meson(dev(w.G1, False), dev(w.eta, False), kp, geom)
    I = c.insertion({t: dev(v, False) for t, v in w.G3.items()}, {t: dev(v, False) for t, v in w.s.items()},
                    [0, 1, 2], q, geom)
    pairs = [(0, 0), (2, 3), (4, 5)]
    wts = np.array([0.2, 0.5, 0.3])
    C = c.combine(S, I, w=wts, pairs=pairs).cpu().numpy()
    for j, (p, qq) in enumerate(pairs):
        for it, tau in enumerate([0, 1, 2]):
            Ghat = brute.stochastic_all_to_all(w.s[tau], w.eta, wts)
            Cb = brute.meson_spin_open(w.G1, Ghat, w.G3[tau], L, kp[p], q[qq], r)
            assert rel_err(C[j, it, 0].reshape((4,) * 6), Cb) < TOL64


# ---------------------------------------------------------------------------
# Behaviour
# ---------------------------------------------------------------------------
def test_bitwise_deterministic():
    c = _lib()
    _say("determinism")
    L = (8, 6, 6)
    w = Workload(L, 8, 2, cfg=105, taus=[1, 2], links=True, reduced=True)
    k = oracle.momenta(6)
    geom = c.Geom(L, 8)
    Gd = {t: dev(v, True) for t, v in w.G3.items()}
    sd = {t: dev(v, True) for t, v in w.s.items()}
    Ud = {t: dev(v, True) for t, v in w.U.items()}
    a = c.insertion(Gd, sd, [1, 2], k, geom, U_t=Ud, n_ops=5)
    b = c.insertion(Gd, sd, [1, 2], k, geom, U_t=Ud, n_ops=5)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_invalid_call_leaves_output_untouched():
    c = _lib()
    _say("invalid call")
    L = (4, 4, 4)
    w = Workload(L, 8, 1, cfg=106, taus=[1])
    out = torch.full((1, 1, 5, 1, 192), 3.0 + 1.0j, dtype=torch.complex128, device="cuda")
    Gd = {1: dev(w.G3[1], False)}
    sd = {1: dev(w.s[1], False)}
    with pytest.raises(c.C3ptError):
        c.insertion(Gd, sd, [1], [[0, 0, 0]], c.Geom(L, 8), U_t=None, n_ops=5, out=out)
    torch.cuda.synchronize()
    assert torch.all(out == (3.0 + 1.0j))


def test_runs_on_a_side_stream():
    c = _lib()
    _say("side stream")
    L = (6, 6, 6)
    w = Workload(L, 8, 2, cfg=107)
    k = oracle.momenta(3)
    s = torch.cuda.Stream()
    G, e = dev(w.G1, True), dev(w.eta, True)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        got = c.spectator_meson(G, e, k, c.Geom(L, 8))
    s.synchronize()
    assert rel_err(got.cpu().numpy(), oracle.spectator_meson(w.G1, w.eta, L, k)) < TOL32


# ---------------------------------------------------------------------------
# Every compiled kernel variant and every projection arithmetic
# ---------------------------------------------------------------------------
MODES = {1: ("f32", 0), 2: ("bf16x2", 2), 3: ("f16x2", 1)}   # mode -> (name, proj flag)


@pytest.mark.parametrize("cls,n2", [(0, 3), (1, 5), (2, 8), (3, 9)])
def test_every_variant_and_precision(cls, n2):
    c = _lib()
    L, T, N = (6, 5, 7), 6, 2
    taus = [0, 4]
    k = oracle.momenta(n2)
    assert c.mt_class(len(k)) == cls
    r = (2, 1, 3)
    w = Workload(L, T, N, cfg=108, taus=taus, links=True, reduced=True, second_prop=True)
    want_s = oracle.spectator_meson(w.G1, w.eta, L, k, r)
    want_b = oracle.spectator_baryon(w.G1, w.G1b, w.eta, L, k, r)
    want_i = oracle.insertion(w.G3, w.s, taus, L, T, k, r, U_t=w.U, n_ops=5)
    G1, G1b, eta = dev(w.G1, True), dev(w.G1b, True), dev(w.eta, True)
    Gd = {t: dev(v, True) for t, v in w.G3.items()}
    sd = {t: dev(v, True) for t, v in w.s.items()}
    Ud = {t: dev(v, True) for t, v in w.U.items()}
    for mode, (mname, proj) in MODES.items():
        geom = c.Geom(L, T, r, proj=proj)
        for kind in range(3):
            prev = c.get_variant(kind, mode, cls)
            try:
                for v in range(c.variant_count(kind, mode, cls)):
                    c.set_variant(kind, mode, cls, v)
                    _say(f"variant kind={kind} mode={mname} class={cls} v={v}")
                    if kind == 0:
                        errs = [rel_err(c.spectator_meson(G1, eta, k, geom).cpu().numpy(), want_s)]
                    elif kind == 1:
                        errs = [rel_err(c.spectator_baryon(G1, G1b, eta, k, geom).cpu().numpy(), want_b)]
                    else:
                        got = c.insertion(Gd, sd, taus, k, geom, U_t=Ud, n_ops=5).cpu().numpy()
                        errs = per_slice_rel(got, want_i)
                    _say(f"    max rel err {max(errs):.2e}")
                    assert max(errs) < TOL32, (kind, mname, v, errs)
            finally:
                c.set_variant(kind, mode, cls, prev)
