"""Batches (c3pt_batch_*): uneven lattices in one recorded graph.

* every job output against the FP64 oracle (1e-5 relative, the FP32 and
  split-precision tolerance) and against the single calls;
* combines recorded in the graph equal c3pt_combine on the batch's outputs;
* replays: outputs cleared between replays, eager work in between, every
  replay bit-identical to the first; inputs refilled in place are picked up;
* a job gives bit-identical results alone and in a mix, and under a partial-sum
  budget that splits the batch into several groups.
"""
import numpy as np
import pytest

import c3pt_synth as syn
import oracle
from helpers import Workload, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
TOL = 1e-5
# batch vs single call: same products, different FP32 chunking of the site sums
SAME = 3e-6


def _say(msg):
    print(msg, flush=True)


def _up(a):
    return torch.from_numpy(np.ascontiguousarray(a.astype(np.complex64))).cuda()


class Lattice:
    """One lattice of the batch: a meson or baryon spectator and an insertion."""

    def __init__(self, L, T, r, N, taus, n_ops, baryon, cfg):
        self.L, self.T, self.r, self.N, self.taus, self.n_ops, self.baryon = L, T, r, N, taus, n_ops, baryon
        self.w = Workload(L, T, N, cfg=cfg, t_f=T - 2, taus=taus, links=n_ops == 5, reduced=True,
                          second_prop=baryon)
        self.dev = {}
        self.upload()

    def upload(self):
        w = self.w
        if not self.dev:
            self.dev = {"G1": _up(w.G1), "eta": _up(w.eta), "G3": {t: _up(v) for t, v in w.G3.items()},
                        "s": {t: _up(v) for t, v in w.s.items()},
                        "U": {t: _up(v) for t, v in w.U.items()} if w.U else None}
            if self.baryon:
                self.dev["G1b"] = _up(w.G1b)
        else:   # refill in place (the batch keeps the device addresses)
            self.dev["G1"].copy_(_up(w.G1))
            self.dev["eta"].copy_(_up(w.eta))
            for t, v in w.G3.items():
                self.dev["G3"][t].copy_(_up(v))
            for t, v in w.s.items():
                self.dev["s"][t].copy_(_up(v))
            if self.baryon:
                self.dev["G1b"].copy_(_up(w.G1b))
            if w.U:
                for t, v in w.U.items():
                    self.dev["U"][t].copy_(_up(v))

    def spec_job(self):
        d = self.dev
        if self.baryon:
            return {"kind": "spectator_baryon", "L": self.L, "T": self.T, "r": self.r, "G1": d["G1"],
                    "G2": d["G1b"], "eta": d["eta"]}
        return {"kind": "spectator_meson", "L": self.L, "T": self.T, "r": self.r, "G": d["G1"], "eta": d["eta"]}

    def ins_job(self):
        d = self.dev
        return {"kind": "insertion", "L": self.L, "T": self.T, "r": self.r, "G_t": d["G3"], "s_t": d["s"],
                "taus": self.taus, "U_t": d["U"], "n_ops": self.n_ops}

    def oracle_parts(self, k):
        w = self.w
        if self.baryon:
            S = oracle.spectator_baryon(w.G1, w.G1b, w.eta, self.L, k, r=self.r)
        else:
            S = oracle.spectator_meson(w.G1, w.eta, self.L, k, r=self.r)
        I = oracle.insertion(w.G3, w.s, self.taus, self.L, self.T, k, r=self.r, U_t=w.U, n_ops=self.n_ops)
        return S, I

    def single_calls(self, c3pt, k, proj):
        d = self.dev
        geom = c3pt.Geom(self.L, self.T, r=self.r, proj=proj)
        if self.baryon:
            S = c3pt.spectator_baryon(d["G1"], d["G1b"], d["eta"], k, geom)
        else:
            S = c3pt.spectator_meson(d["G1"], d["eta"], k, geom)
        I = c3pt.insertion(d["G3"], d["s"], self.taus, k, geom, U_t=d["U"], n_ops=self.n_ops)
        return S, I


def _lattices():
    # a multi-chunk lattice (2688 sites: two FP32 chunks, ragged last tile),
    # an odd small one, and a baryon one; source positions off the origin
    return [Lattice((14, 12, 16), 8, (3, 5, 7), 3, [0, 3, 7], 5, False, cfg=11),
            Lattice((5, 3, 4), 6, (4, 1, 2), 2, [1, 2], 1, False, cfg=12),
            Lattice((4, 4, 6), 6, (0, 1, 2), 2, [0, 5], 1, True, cfg=13)]


def _batch(c3pt, lats, k, proj, budget=0, combine_pairs=((0, 0), (3, 5), (26, 1))):
    jobs, combs = [], []
    for lat in lats:
        jobs += [lat.spec_job(), lat.ins_job()]
        combs.append({"spec": len(jobs) - 2, "ins": len(jobs) - 1, "pairs": list(combine_pairs)})
    return c3pt.Batch(jobs, k, proj=proj, combines=combs, partial_budget=budget)


@pytest.mark.parametrize("proj,name", [(0, "f32"), (2, "bf16x2"), (1, "f16x2"), (3, "factored")])
def test_batch_matches_oracle_and_single_calls(proj, name):
    import paper_1711_02384_amd as c3pt
    k = c3pt.momentum_list(3)          # 27 momenta
    lats = _lattices()
    _say(f"batch {name}: create")
    b = _batch(c3pt, lats, k, proj)
    _say(f"batch {name}: {b.info()}")
    b.run()
    torch.cuda.synchronize()
    for li, lat in enumerate(lats):
        S_o, I_o = lat.oracle_parts(k)
        S, I = b.outputs[2 * li].cpu().numpy(), b.outputs[2 * li + 1].cpu().numpy()
        es, ei = rel_err(S, S_o), rel_err(I, I_o)
        _say(f"batch {name}: lattice {lat.L} spectator {es:.2e} insertion {ei:.2e}")
        assert es < TOL and ei < TOL
        for tl in range(len(lat.taus)):
            for op in range(lat.n_ops):
                assert rel_err(I[:, tl, op], I_o[:, tl, op]) < TOL
        Ss, Is = lat.single_calls(c3pt, k, proj)
        torch.cuda.synchronize()
        assert rel_err(S, Ss.cpu().numpy()) < SAME
        assert rel_err(I, Is.cpu().numpy()) < SAME
        C_ref = c3pt.combine(b.outputs[2 * li], b.outputs[2 * li + 1], pairs=[(0, 0), (3, 5), (26, 1)])
        torch.cuda.synchronize()
        assert torch.equal(b.combine_outputs[li], C_ref)
    b.close()


def test_batch_graph_replays_and_refill():
    import paper_1711_02384_amd as c3pt
    k = c3pt.momentum_list(3)
    lats = _lattices()
    b = _batch(c3pt, lats, k, 0)
    b.run()
    torch.cuda.synchronize()
    first = [o.clone() for o in b.outputs + b.combine_outputs]
    x = torch.randn(512, 512, device="cuda")
    for rep in range(3):
        for o in b.outputs + b.combine_outputs:
            o.zero_()
        y = x @ x                       # eager work between replays
        torch.cuda.synchronize()
        b.run()
        torch.cuda.synchronize()
        for o, f in zip(b.outputs + b.combine_outputs, first):
            assert torch.equal(o, f), f"replay {rep} differs"
        _say(f"replay {rep}: identical ({float(y[0, 0]):.3f})")
    # refill the inputs in place with another configuration: the graph reads them
    for lat, cfg in zip(lats, (21, 22, 23)):
        lat.w = Workload(lat.L, lat.T, lat.N, cfg=cfg, t_f=lat.T - 2, taus=lat.taus, links=lat.n_ops == 5,
                         reduced=True, second_prop=lat.baryon)
        lat.upload()
    torch.cuda.synchronize()
    b.run()
    torch.cuda.synchronize()
    for li, lat in enumerate(lats):
        Ss, Is = lat.single_calls(c3pt, k, 0)
        torch.cuda.synchronize()
        assert rel_err(b.outputs[2 * li].cpu().numpy(), Ss.cpu().numpy()) < SAME
        assert rel_err(b.outputs[2 * li + 1].cpu().numpy(), Is.cpu().numpy()) < SAME
        assert not torch.equal(b.outputs[2 * li], first[2 * li])
    b.close()


@pytest.mark.parametrize("proj", [2, 3])
def test_batch_alone_vs_mix_and_budget_groups(proj):
    import paper_1711_02384_amd as c3pt
    k = c3pt.momentum_list(3)
    lats = _lattices()
    mix = _batch(c3pt, lats, k, proj)
    mix.run()
    # each lattice alone
    alone = [_batch(c3pt, [lat], k, proj) for lat in lats]
    for a in alone:
        a.run()
    # the mix again under a budget that forces several groups
    n_mom = len(k)
    biggest = 0
    for lat in lats:
        for kind_cols in ((16 if lat.baryon else 1) * lat.N, lat.N * len(lat.taus) * lat.n_ops):
            V3 = int(np.prod(lat.L))
            if proj == 3:   # factored: chunks of x3 planes of about 2048 sites
                planes = max(1, min(lat.L[2], 2048 // (lat.L[0] * lat.L[1])))
                n_chunks = -(-lat.L[2] // planes)
            else:
                n_chunks = -(-V3 // 2048)
            biggest = max(biggest, n_chunks * kind_cols * n_mom * 192 * 8)
    split = _batch(c3pt, lats, k, proj, budget=biggest)
    split.run()
    torch.cuda.synchronize()
    info = split.info()
    _say(f"mix {mix.info()}  split {info}")
    assert info["groups"] > 1
    for li in range(len(lats)):
        for j in (0, 1):
            assert torch.equal(mix.outputs[2 * li + j], alone[li].outputs[j])
            assert torch.equal(mix.outputs[2 * li + j], split.outputs[2 * li + j])
        assert torch.equal(mix.combine_outputs[li], alone[li].combine_outputs[0])
    for x in [mix, split] + alone:
        x.close()


def test_batch_on_side_stream():
    import paper_1711_02384_amd as c3pt
    k = c3pt.momentum_list(2)
    lats = _lattices()[1:]
    b = _batch(c3pt, lats, k, 0, combine_pairs=((0, 0), (4, 2)))
    side = torch.cuda.Stream()
    b.run(stream=side.cuda_stream)
    side.synchronize()
    for li, lat in enumerate(lats):
        S_o, I_o = lat.oracle_parts(k)
        assert rel_err(b.outputs[2 * li].cpu().numpy(), S_o) < TOL
        assert rel_err(b.outputs[2 * li + 1].cpu().numpy(), I_o) < TOL
    b.close()


def test_batch_profiled_run_times_each_kernel_and_matches_graph():
    import paper_1711_02384_amd as c3pt
    k = c3pt.momentum_list(3)
    lats = _lattices()
    b = _batch(c3pt, lats, k, 2)
    b.run()
    torch.cuda.synchronize()
    ref = [o.clone() for o in b.outputs + b.combine_outputs]
    for o in b.outputs + b.combine_outputs:
        o.zero_()
    c3pt.profile_read(reset=True)
    c3pt.profile_enable(True)
    b.run()                      # eager: the recorded launches one by one, each timed
    torch.cuda.synchronize()
    c3pt.profile_enable(False)
    prof = c3pt.profile_read(reset=True)
    _say(f"profiled batch: {sorted(prof)}")
    for name in ("batch_reset", "batch_proj_spectator_meson", "batch_proj_spectator_baryon",
                 "batch_proj_insertion", "batch_reduce", "combine"):
        assert prof[name]["count"] >= 1 and prof[name]["total_ms"] > 0
    for o, r in zip(b.outputs + b.combine_outputs, ref):
        assert torch.equal(o, r)
    b.close()


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_batch_factored_variants(variant):
    """The factored batch's tunable forms (32-site tiles for jobs whose L1 is a
    multiple of 32, chunks of about 4096 sites) against the oracle and against
    the default form; lattices with L1 = 32 (meson with the derivative
    operators, baryon, which keeps 16-site tiles) beside ones that keep 16."""
    import paper_1711_02384_amd as c3pt
    k = c3pt.momentum_list(3)
    cls = c3pt.mt_class(len(k))
    lats = [Lattice((32, 6, 24), 6, (5, 1, 9), 2, [0, 2], 5, False, cfg=21),
            Lattice((32, 4, 3), 6, (1, 2, 0), 2, [1], 1, True, cfg=22)] + _lattices()[:1]
    kinds = ("spectator_meson", "spectator_baryon", "insertion")
    before = {kn: c3pt.get_variant(c3pt.KIND[kn], c3pt.MODE["batchfac"], cls) for kn in kinds}
    outs = {}
    try:
        for v in (0, variant):
            for kn in kinds:
                c3pt.set_variant(c3pt.KIND[kn], c3pt.MODE["batchfac"], cls, v)
            _say(f"batch factored variant {v}: create")
            b = _batch(c3pt, lats, k, c3pt.PROJ_FACTORED)
            b.run()
            torch.cuda.synchronize()
            outs[v] = [o.cpu().numpy() for o in b.outputs]
            b.close()
    finally:
        for kn in kinds:
            c3pt.set_variant(c3pt.KIND[kn], c3pt.MODE["batchfac"], cls, before[kn])
    for li, lat in enumerate(lats):
        S_o, I_o = lat.oracle_parts(k)
        S, I = outs[variant][2 * li], outs[variant][2 * li + 1]
        es, ei = rel_err(S, S_o), rel_err(I, I_o)
        _say(f"batch factored variant {variant}: lattice {lat.L} spectator {es:.2e} insertion {ei:.2e}")
        assert es < TOL and ei < TOL
        assert rel_err(S, outs[0][2 * li]) < SAME and rel_err(I, outs[0][2 * li + 1]) < SAME
