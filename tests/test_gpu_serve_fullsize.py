"""Parity of the serving loop at full lattice sizes, in the configuration
bench.py's serve workload runs: its resident pool (u and d propagators and
the stochastic solutions of 16 noise vectors on every timeslice, drawn on the
GPU from seeded generators) for the 64^3 x 128 and 16^3 x 32 lattices, and a
server with its arena, step workspace and request limit.  Three requests in
flight together:

* 64^3 meson, N = 3, |k|^2 <= 9 (123 momenta), timeslices wrapping past T:
  spectator, insertion at the first and last timeslice, and the combine on
  all 245 (p', q) pairs at those timeslices;
* 64^3 nucleon, N = 2: the (u, d) spectator for one noise vector and five
  momenta, and the d insertion at the first timeslice;
* 16^3 meson, N = 16 (the pool's maximum): spectator, insertion at every
  timeslice and the combine.

The FP64 oracle recomputes these from the inputs copied back to the host.
Tolerance 1e-5 relative (Frobenius), the FP32 bar.
"""
import gc

import numpy as np
import pytest

import oracle
from helpers import rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
TOL = 1e-5


def _say(msg):
    print(msg, flush=True)


def _host(t):
    return t.cpu().numpy().astype(np.complex128)


SPECS = [
    {"L": 64, "n2": 9, "kind": "meson", "N": 3, "t_src": 120, "t_f": 2, "n_tau": 11, "r": [5, 61, 33]},
    {"L": 64, "n2": 5, "kind": "nucleon", "N": 2, "t_src": 40, "t_f": 49, "n_tau": 10, "r": [17, 2, 50]},
    {"L": 16, "n2": 3, "kind": "meson", "N": 16, "t_src": 30, "t_f": 6, "n_tau": 9, "r": [3, 14, 9]},
]


@pytest.fixture(scope="module")
def served():
    import bench
    import paper_1711_02384_amd as c3pt
    dev = torch.device("cuda:0")
    _say("serve full size: drawing the resident pool (64^3 x 128, 16^3 x 32)")
    pool = bench.ServePool([64, 16], dev)
    sv = c3pt.Server(proj=c3pt.PROJ_FACTORED, arena_bytes=48 << 30, step_bytes=1024 << 20, max_active=32)
    reqs = [pool.request(c3pt, sp) for sp in SPECS]
    ids = [sv.submit(q) for q in reqs]
    _say(f"serve full size: {len(ids)} requests submitted")
    sv.run_until_done(ids)
    torch.cuda.synchronize()
    res = [{k: [t.cpu().numpy() for t in v] for k, v in sv.result(i).items()} for i in ids]
    _say("serve full size: done")
    yield reqs, res
    for i in ids:
        sv.release(i)
    sv.close()
    # pytest still holds the yielded requests here: drop their tensors and the
    # resident pool (about 120 GiB) so that later modules find the memory free
    for q in reqs:
        q.clear()
    pool.__dict__.clear()
    gc.collect()
    torch.cuda.empty_cache()


def _meson_check(q, got, taus_checked, name):
    L, T, r, k = q["L"], q["T"], q["r"], q["k"]
    tf = q["t_f"]
    taus = [(q["t_src"] + i) % T for i in range((tf - q["t_src"]) % T + 1)]
    S_o = oracle.spectator_meson(_host(q["G_t"][tf]), _host(q["eta"]), L, k, r=r)
    err = rel_err(got["spec"][0], S_o)
    _say(f"{name}: spectator rel err {err:.2e}")
    assert err < TOL
    for tl in taus_checked:
        tau = taus[tl]
        I_o = oracle.insertion({tau: _host(q["G_t"][tau])}, {tau: _host(q["s_t"][tau])}, [tau], L, T, k, r=r)
        err = rel_err(got["ins"][0][:, tl], I_o[:, 0])
        _say(f"{name}: insertion tau={tau} rel err {err:.2e}")
        assert err < TOL
        C_o = oracle.combine(S_o, I_o, pairs=q["pairs"])
        err = rel_err(got["comb"][0][:, tl], C_o[:, 0])
        _say(f"{name}: combine tau={tau} ({len(q['pairs'])} pairs) rel err {err:.2e}")
        assert err < TOL


def test_serve_fullsize_meson64(served):
    reqs, res = served
    q = reqs[0]
    assert q["L"] == (64, 64, 64) and q["t_f"] < q["t_src"]
    _meson_check(q, res[0], (0, 10), "serve meson 64^3")


def test_serve_fullsize_nucleon64(served):
    reqs, res = served
    q, got = reqs[1], res[1]
    L, T, r, k = q["L"], q["T"], q["r"], q["k"]
    tf = q["t_f"]
    sel_m = [0, 1, 7, 20, len(k) - 1]
    want = oracle.spectator_baryon(_host(q["G_t"][tf]), _host(q["G2_t"][tf]), _host(q["eta"])[1:2], L, k[sel_m], r=r)
    err = rel_err(got["spec"][1][1:2, sel_m], want)
    _say(f"serve nucleon 64^3: (u,d) spectator (noise 1, 5 momenta) rel err {err:.2e}")
    assert err < TOL
    tau = q["t_src"]
    I_o = oracle.insertion({tau: _host(q["G2_t"][tau])}, {tau: _host(q["s_t"][tau])}, [tau], L, T, k, r=r)
    err = rel_err(got["ins"][1][:, 0], I_o[:, 0])
    _say(f"serve nucleon 64^3: d insertion tau={tau} rel err {err:.2e}")
    assert err < TOL


def test_serve_fullsize_meson16_all_noise(served):
    reqs, res = served
    q = reqs[2]
    assert q["L"] == (16, 16, 16) and q["eta"].shape[0] == 16
    _meson_check(q, res[2], range(9), "serve meson 16^3")
