"""Parity at the benchmark's full sizes, in the launch configuration bench.py times.

The GPU computes every part of the step; the FP64 oracle recomputes sampled
outputs (selected timeslices, noise vectors or momenta) one by one.

* 32^3 x 64 meson step (FP32, dense and factored projection): spectator (all outputs), insertion with the
  five operators at tau = 0, 8, 16 (the full 17-slice launch runs on the GPU),
  and the combine on sampled pairs built from the oracle's own parts.
* the same insertion with the symmetrized derivative (n_ops = 9), checked at
  the first and last timeslice;
* 48^3 x 64 nucleon step with the fused split-precision projection (FP16 hi+lo,
  the benchmark's form, and BF16), the dense split-precision projection and
  the factored FP32 one: the nucleon spectator for one noise vector and a
  momentum subset, and one insertion timeslice.  Tolerance 1e-5 relative
  (the larger of Frobenius and max-element), the same as FP32.
* the 48^3 x 64 nucleon step in the exact launch configuration of the
  benchmark (93 momenta, tuned fused variants with the two-block remainder
  launch, 15 timeslices in one insertion call, 185 combine pairs), sampled
  in both launches of each call.
"""
import numpy as np
import pytest

import c3pt_synth as syn
import oracle
from helpers import rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
TOL32 = 1e-5


def _say(msg):
    print(msg, flush=True)


def _up(a):
    return torch.from_numpy(np.ascontiguousarray(a.astype(np.complex64))).cuda()


@pytest.mark.parametrize("proj,name", [(0, "dense f32"), (3, "factored")])
def test_meson32_step_sampled(proj, name):
    import paper_1711_02384_amd as c3pt
    L, T, N, t_f, cfg = (32, 32, 32), 64, 4, 16, 2
    taus = list(range(17))
    k = c3pt.momentum_list(6)
    _say("meson32: generating inputs")
    G1 = syn.round_to_c64(syn.propagator_slice(L, cfg, syn.FIELD_G1, t_f))
    eta = syn.round_to_c64(syn.z2z2_noise(L, N, cfg, t_f))
    gsl = sorted({t % T for tau in taus for t in (tau - 1, tau, tau + 1)})
    usl = sorted({t % T for tau in taus for t in (tau - 1, tau)})
    G3 = {t: syn.round_to_c64(syn.propagator_slice(L, cfg, syn.FIELD_G3, t)) for t in gsl}
    s = {t: syn.round_to_c64(syn.solution_slice(L, N, cfg, t)) for t in taus}
    U = {t: syn.round_to_c64(syn.link_slice(L, cfg, t)) for t in usl}
    geom = c3pt.Geom(L, T, proj=proj)
    _say(f"meson32 {name}: GPU step")
    S = c3pt.spectator_meson(_up(G1), _up(eta), k, geom)
    I = c3pt.insertion({t: _up(v) for t, v in G3.items()}, {t: _up(v) for t, v in s.items()}, taus, k, geom,
                       U_t={t: _up(v) for t, v in U.items()}, n_ops=5)
    torch.cuda.synchronize()
    S_o = oracle.spectator_meson(G1, eta, L, k)
    err = rel_err(S.cpu().numpy(), S_o)
    _say(f"meson32 {name}: spectator rel err {err:.2e}")
    assert err < TOL32
    Ih = I.cpu().numpy()
    for tau in (0, 8, 16):
        I_o = oracle.insertion(G3, s, [tau], L, T, k, U_t=U, n_ops=5)
        for op in range(5):
            e = rel_err(Ih[:, tau, op], I_o[:, 0, op])
            _say(f"meson32 {name}: insertion tau={tau} op={op} rel err {e:.2e}")
            assert e < TOL32
    # combine on sampled pairs, from the oracle's parts (checks the full-size launch shape)
    pairs = [(0, 0), (40, 40), (80, 3), (0, 80)]
    I8 = oracle.insertion(G3, s, [8], L, T, k, U_t=U, n_ops=5)
    C = c3pt.combine(torch.from_numpy(S_o).cuda(), torch.from_numpy(I8).cuda(), pairs=pairs).cpu().numpy()
    assert rel_err(C, oracle.combine(S_o, I8, pairs=pairs)) < 1e-12


def test_meson32_symmetric_sampled():
    """The 32^3 insertion with the symmetrized derivative (n_ops = 9, factored
    FP32) over tau = 0..16 as bench.py --ops 9 launches it; the oracle checks
    the first and last timeslice (their s(tau -+ 1) lie outside the range)."""
    import paper_1711_02384_amd as c3pt
    L, T, N, cfg = (32, 32, 32), 64, 4, 2
    taus = list(range(17))
    k = c3pt.momentum_list(6)
    _say("meson32 symmetric: generating inputs")
    gsl = sorted({t % T for tau in taus for t in (tau - 1, tau, tau + 1)})
    usl = sorted({t % T for tau in taus for t in (tau - 1, tau)})
    G3 = {t: syn.round_to_c64(syn.propagator_slice(L, cfg, syn.FIELD_G3, t)) for t in gsl}
    s = {t: syn.round_to_c64(syn.solution_slice(L, N, cfg, t)) for t in gsl}
    U = {t: syn.round_to_c64(syn.link_slice(L, cfg, t)) for t in usl}
    geom = c3pt.Geom(L, T, proj=3)
    _say("meson32 symmetric: GPU insertion")
    I = c3pt.insertion({t: _up(v) for t, v in G3.items()}, {t: _up(v) for t, v in s.items()}, taus, k, geom,
                       U_t={t: _up(v) for t, v in U.items()}, n_ops=9).cpu().numpy()
    for tau in (0, 16):
        I_o = oracle.insertion(G3, s, [tau], L, T, k, U_t=U, n_ops=9)
        for op in range(9):
            e = rel_err(I[:, tau, op], I_o[:, 0, op])
            _say(f"meson32 symmetric: tau={tau} op={op} rel err {e:.2e}")
            assert e < TOL32


@pytest.mark.parametrize("proj,name", [(4, "fused f16 (the benchmark's form)"), (5, "fused bf16"), (2, "bf16x2"),
                                       (1, "f16x2"), (3, "factored")])
def test_nucleon48_split_sampled(proj, name):
    import paper_1711_02384_amd as c3pt
    L, T, N, t_f, cfg = (48, 48, 48), 64, 8, 14, 3
    k = c3pt.momentum_list(9)          # 123 momenta: one 128-row group
    _say(f"nucleon48 {name}: generating inputs")
    Gu = syn.round_to_c64(syn.propagator_slice(L, cfg, syn.FIELD_G3, t_f))
    Gd = syn.round_to_c64(syn.propagator_slice(L, cfg, syn.FIELD_G1, t_f))
    eta = syn.round_to_c64(syn.z2z2_noise(L, N, cfg, t_f))
    geom = c3pt.Geom(L, T, proj=proj)
    SB = c3pt.spectator_baryon(_up(Gu), _up(Gd), _up(eta), k, geom).cpu().numpy()
    sel_m = [0, 1, 30, 92, 122]
    want = oracle.spectator_baryon(Gu, Gd, eta[3:4], L, k[sel_m])
    err = rel_err(SB[3:4, sel_m], want)
    _say(f"nucleon48 {name}: baryon spectator (noise 3, 5 momenta) rel err {err:.2e}")
    assert err < TOL32
    tau = 7
    G7 = syn.round_to_c64(syn.propagator_slice(L, cfg, syn.FIELD_G3, tau))
    s7 = syn.round_to_c64(syn.solution_slice(L, N, cfg, tau))
    Id = c3pt.insertion({tau: _up(G7)}, {tau: _up(s7)}, [tau], k, geom)
    I = Id.cpu().numpy()
    I_o = oracle.insertion({tau: G7}, {tau: s7}, [tau], L, T, k)
    err = rel_err(I, I_o)
    _say(f"nucleon48 {name}: insertion tau={tau} rel err {err:.2e}")
    assert err < TOL32
    if proj == 4:
        # the full-size nucleon combine (1024 x 64 per pair) on these parts
        pairs = [(0, 0), (30, 30), (0, 92), (122, 7)]
        SBd = torch.from_numpy(SB).cuda()
        C = c3pt.combine(SBd, Id, pairs=pairs).cpu().numpy()
        e = rel_err(C, oracle.combine(SB, I, pairs=pairs))
        _say(f"nucleon48 {name}: combine on {len(pairs)} pairs rel err {e:.2e}")
        assert e < 1e-12


def test_nucleon48_benchmark_launches_sampled():
    """The 48^3 x 64 nucleon step exactly as bench.py launches it: 93 momenta
    (|k|^2 <= 8, one momentum group), N = 8, the fused FP16 projection with the
    tuned variants (three column blocks per workgroup over noise vectors 0-5 and
    a two-block launch over 6-7), the insertion over all 15 timeslices in one
    call and the combine on the 185 (p' = q or p' = 0) pairs.  Sampled: the
    (u,d) spectator for noise vectors 2 and 7 (one from each launch) at three
    momenta, the (u,u) spectator (one buffer for both propagators, as the step
    passes it) for noise vector 6 at two momenta, the insertion at tau = 0 and
    14 for every noise vector and momentum, and the combine of the GPU's parts
    on four pairs."""
    import paper_1711_02384_amd as c3pt
    c3pt.apply_tuning(c3pt.DEFAULT_TUNING)
    L, T, N, t_f, cfg = (48, 48, 48), 64, 8, 14, 3
    taus = list(range(15))
    k = c3pt.momentum_list(8)
    assert len(k) == 93
    cls = c3pt.mt_class(len(k))
    for kind in ("spectator_baryon", "insertion"):
        assert c3pt.get_variant(c3pt.KIND[kind], c3pt.MODE["fs16"], cls) == 4, kind
    geom = c3pt.Geom(L, T, proj=c3pt.PROJ_FACTORED_F16)
    _say("nucleon48 benchmark launches: generating inputs")
    Gu = syn.round_to_c64(syn.propagator_slice(L, cfg, syn.FIELD_G3, t_f))
    Gd = syn.round_to_c64(syn.propagator_slice(L, cfg, syn.FIELD_G1, t_f))
    eta = syn.round_to_c64(syn.z2z2_noise(L, N, cfg, t_f))
    Gu_dev, eta_dev = _up(Gu), _up(eta)
    SB = c3pt.spectator_baryon(Gu_dev, _up(Gd), eta_dev, k, geom)
    # (u,u) as the step calls it: one buffer for both propagators
    SBuu = c3pt.spectator_baryon(Gu_dev, Gu_dev, eta_dev, k, geom)
    # distinct slices at the checked timeslices and one other slice shared by
    # the rest (a launch reading the wrong slice shows at tau = 0 or 14)
    G = {t: syn.round_to_c64(syn.propagator_slice(L, cfg, syn.FIELD_G3, t)) for t in (0, 7, 14)}
    s = {t: syn.round_to_c64(syn.solution_slice(L, N, cfg, t)) for t in (0, 7, 14)}
    Gdev = {t: _up(a) for t, a in G.items()}
    sdev = {t: _up(a) for t, a in s.items()}
    Gt = {t: Gdev.get(t, Gdev[7]) for t in taus}
    st = {t: sdev.get(t, sdev[7]) for t in taus}
    Id = c3pt.insertion(Gt, st, taus, k, geom)
    pairs = np.array([(p, p) for p in range(93)] + [(0, q) for q in range(1, 93)], dtype=np.int32)
    C = c3pt.combine(SB, Id, pairs=pairs)
    torch.cuda.synchronize()
    sel_p = [0, 50, 93, 184]
    C_sel = C[sel_p].cpu().numpy()
    del C
    S = SB.cpu().numpy()
    I = Id.cpu().numpy()
    sel_n, sel_m = [2, 7], [0, 46, 92]
    want = oracle.spectator_baryon(Gu, Gd, eta[sel_n], L, k[sel_m])
    err = rel_err(S[sel_n][:, sel_m], want)
    _say(f"nucleon48 benchmark launches: spectator (noise 2 and 7, 3 momenta) rel err {err:.2e}")
    assert err < TOL32
    want = oracle.spectator_baryon(Gu, Gu, eta[6:7], L, k[[0, 92]])
    err = rel_err(SBuu[6:7, [0, 92]].cpu().numpy(), want)
    _say(f"nucleon48 benchmark launches: (u,u) spectator (noise 6, 2 momenta) rel err {err:.2e}")
    assert err < TOL32
    for tau in (0, 14):
        I_o = oracle.insertion({tau: G[tau]}, {tau: s[tau]}, [tau], L, T, k)
        err = rel_err(I[:, tau], I_o[:, 0])
        _say(f"nucleon48 benchmark launches: insertion tau={tau} (8 noise vectors, 93 momenta) rel err {err:.2e}")
        assert err < TOL32
    e = rel_err(C_sel, oracle.combine(S, I, pairs=pairs[sel_p]))
    _say(f"nucleon48 benchmark launches: combine on pairs {sel_p} rel err {e:.2e}")
    assert e < 1e-12
