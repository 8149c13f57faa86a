"""Pins of the analysis-stage Gamma channels of the oracle.

* meson: the spin-open tensor contracted with Gsnk, Gins, Gsrc equals the
  trace of Eq. (1) evaluated with 12x12 matrix products, for random matrices;
* nucleon: the spin-open tensor contracted by the proton's Wick terms equals a
  brute-force Wick contraction of chi(x') J(y) chibar(r) over quark fields
  (tests/wick.py), for random diquark matrices, projectors and currents, for
  a d and a u current;
* the default matrices: C gamma5 with C = gamma2 gamma4 obeys
  C gamma_mu C^-1 = -gamma_mu^T; the creation matrix of Gamma_n under the
  default source list.
"""
import numpy as np
import pytest

import c3pt_synth as syn
import oracle
from oracle import brute
import wick



def _rand(shape, g):
    return syn.gaussian(shape, g)


def test_meson_channels_equal_trace_of_eq1():
    L = (2, 2, 1)
    V3 = 4
    g = np.random.default_rng(5)
    G1 = _rand((12, 12, V3), g)
    G2 = _rand((V3, V3, 12, 12), g)
    G3 = _rand((12, 12, V3), g)
    kp, q, r = (1, 0, 0), (1, 1, 0), (1, 0, 0)
    C = brute.meson_spin_open(G1, G2, G3, L, kp, q, r=r).reshape(64, 64)
    Gs, Gi, Gc = _rand((3, 4, 4), g), _rand((2, 4, 4), g), _rand((2, 4, 4), g)
    out = oracle.gamma_project_meson(C, Gs, Gi, Gc)
    assert out.shape == (3, 2, 2)
    for i in range(3):
        for j in range(2):
            for l in range(2):
                want = brute.meson_trace(G1, G2, G3, L, kp, q, Gs[i], Gi[j], Gc[l], r=r)
                assert abs(out[i, j, l] - want) < 1e-12 * abs(want)


def test_meson_default_channels():
    g = np.random.default_rng(6)
    C = _rand((2, 64, 64), g)
    out = oracle.gamma_project_meson(C)
    assert out.shape == (2, 16, 16, 16)
    g16 = oracle.gamma_basis16()
    g4 = oracle.GAMMA[3]
    i, j, l = 6, 9, 13
    src = g4 @ g16[l].conj().T @ g4
    want = np.einsum('nBAaxyb,AB,xy,ba->n', C.reshape(2, *(4,) * 6), g16[i], g16[j], src)
    assert np.allclose(out[:, i, j, l], want, rtol=1e-13, atol=0)


def test_charge_conjugation_and_projectors():
    Cm = oracle.charge_conjugation()
    Ci = np.linalg.inv(Cm)
    for gmu in oracle.GAMMA:
        assert np.allclose(Cm @ gmu @ Ci, -gmu.T)
    P = oracle.parity_projectors()
    assert np.allclose(P[0] @ P[0], P[0]) and np.allclose(P[0] @ P[1], 0) and np.allclose(P[0] + P[1], np.eye(4))


def _props(flavours, points, g):
    return {(f, a, b): _rand((4, 3, 4, 3), g) for f, a, b in
            [(f, a, b) for f in flavours for a, b in points]}


@pytest.mark.parametrize("channel", ["d", "u"])
def test_nucleon_channels_equal_wick_contraction(channel):
    """V3 = 2 sites, source at site 0, sums over sink and insertion sites with
    the phases of Eqs. (9)-(10); random A, Abar, projectors and currents."""
    L, V3 = (2, 1, 1), 2
    g = np.random.default_rng(11 if channel == "d" else 12)
    xs = [("x", n) for n in range(V3)]
    ys = [("y", n) for n in range(V3)]
    r = ("r", 0)
    Su = {x: _rand((4, 3, 4, 3), g) for x in xs}                 # <u(x') ubar(r)>
    Sd = {x: _rand((4, 3, 4, 3), g) for x in xs}                 # <d(x') dbar(r)>
    Sxy = {(x, y): _rand((4, 3, 4, 3), g) for x in xs for y in ys}   # active flavour, <q(x') qbar(y)>
    Syr = {y: _rand((4, 3, 4, 3), g) for y in ys}                # active flavour, <q(y) qbar(r)>
    A, Abar = _rand((4, 4), g), _rand((4, 4), g)
    P = _rand((2, 4, 4), g)
    Gi = _rand((3, 4, 4), g)
    kp, q = (1, 0, 0), (1, 0, 0)

    props = {}
    for x in xs:
        props[("u", x, r)] = Su[x]
        props[("d", x, r)] = Sd[x]
        for y in ys:
            props[(channel, x, y)] = Sxy[(x, y)]
    for y in ys:
        props[(channel, y, r)] = Syr[y]
    eps = oracle.EPS.astype(np.complex128)
    want = np.zeros((2, 3), dtype=np.complex128)
    for x in xs:
        for y in ys:
            fields = (wick.proton(x, ("s1", "s2", "g"), ("a", "b", "c"), "snk")
                      + wick.current(y, channel, ("m", "n"), "e")
                      + wick.proton(r, ("t1", "t2", "d"), ("a'", "b'", "c'"), "src", conj=True))
            coeffs = [(eps, ("a", "b", "c")), (A, ("s1", "s2")), (Gi, ("j", "m", "n")),
                      (eps, ("a'", "b'", "c'")), (Abar, ("t2", "t1")), (P, ("p", "d", "g"))]
            ph = np.exp(-2j * np.pi * kp[0] * x[1] / L[0]) * np.exp(2j * np.pi * q[0] * y[1] / L[0])
            want += ph * wick.expectation(fields, coeffs, props, ("p", "j"))

    # the spin-open data of the same propagators
    site = lambda S: S.reshape(12, 12)
    G1 = np.stack([site(Su[x]) for x in xs], axis=-1)
    G2 = np.stack([site(Su[x] if channel == "d" else Sd[x]) for x in xs], axis=-1)
    G5 = np.kron(np.diag([1, 1, -1, -1]), np.eye(3))
    # forward G(y, x') whose gamma5-hermitian conjugate is <q(x') qbar(y)>
    Gact_yx = np.stack([np.stack([G5 @ site(Sxy[(x, y)]).conj().T @ G5 for x in xs]) for y in ys])
    G3 = np.stack([site(Syr[y]) for y in ys], axis=-1)
    T = brute.baryon_spin_open(G1, G2, Gact_yx, G3, L, kp, q).reshape(1024, 64)
    got = oracle.gamma_project_nucleon(T, channel, A=A, Abar=Abar, P=P, g_ins=Gi)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


def test_nucleon_wrong_sign_is_caught():
    """A planted sign flip of one Wick term of the u channel changes the result."""
    g = np.random.default_rng(13)
    T = _rand((1024, 64), g)
    base = oracle.gamma_project_nucleon(T, "u")
    terms = list(oracle.PROTON_TERMS["u"])
    try:
        s, a, b = terms[1]
        oracle.PROTON_TERMS["u"][1] = (-s, a, b)
        flipped = oracle.gamma_project_nucleon(T, "u")
    finally:
        oracle.PROTON_TERMS["u"][:] = terms
    assert np.abs(flipped - base).max() > 1e-3 * np.abs(base).max()
