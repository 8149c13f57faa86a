"""Pins of the creation matrices the Gamma-channel oracle uses by default.

The source operator of a two- or three-point function is the Hermitian
conjugate of the sink (annihilation) operator, Eq. (3): for O = psibar Gamma chi
it is O^dag = chibar Gbar psi with Gbar = gamma4 Gamma^dag gamma4, and for the
proton chi = eps (u^T A d) u the conjugate chibar = chi^dag gamma4 carries the
diquark matrix Abar = gamma4 A^dag gamma4.  The oracle's creation_matrix()
supplies both defaults (the meson source list and the nucleon Abar).  These
tests fix them without writing the formula again:

* c-number spinors: conj(psibar Gamma chi) = chibar M psi for M = creation_matrix(Gamma)
  and random psi, chi, Gamma, with psibar = psi^dag gamma4;
* meson: the Wick contraction of O_snk(x') J(y) O_src(r)^dag, the last built
  field by field as the conjugate of psibar_1 Gamma psi_3 (tests/wick.py),
  equals minus (one fermion loop) the default channel of the spin-open data;
* nucleon: the Wick contraction with the source operator built field by field
  as chi^dag gamma4 of eps (u^T A d) u equals the default channel for random A,
  for the d and the u current;
* planted mistakes in the creation matrix (transposed, not conjugated, no
  gamma4) are caught by every one of them.
"""
import numpy as np
import pytest

import c3pt_synth as syn
import oracle
from oracle import brute
import wick

G4 = oracle.GAMMA[3]

# wrong readings of gamma4 Gamma^dag gamma4 that a mistake could produce
MUTANTS = {
    "transposed": lambda M: G4 @ np.asarray(M).T @ G4,
    "not conjugated": lambda M: G4 @ np.asarray(M) @ G4,
    "no gamma4": lambda M: np.conj(np.asarray(M)).T,
}


def _rand(shape, g):
    return syn.gaussian(shape, g)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_creation_matrix_conjugates_the_bilinear(seed):
    g = np.random.default_rng(100 + seed)
    psi, chi = _rand((4,), g), _rand((4,), g)
    Gam = _rand((4, 4), g)
    bar = lambda v: np.conj(v) @ G4
    lhs = np.conj(bar(psi) @ Gam @ chi)
    assert abs(lhs - bar(chi) @ oracle.creation_matrix(Gam) @ psi) < 1e-13 * abs(lhs)
    for name, mut in MUTANTS.items():
        assert abs(lhs - bar(chi) @ mut(Gam) @ psi) > 1e-3 * abs(lhs), name
    # the 16 basis matrices of the default source list
    for Gn in oracle.gamma_basis16():
        want = np.conj(bar(psi) @ Gn @ chi)
        assert abs(want - bar(chi) @ oracle.creation_matrix(Gn) @ psi) < 1e-13 * max(1.0, abs(want))


def _meson_wick(M1, M2, M3, L, kp, q, Gs, Gi, Gsrc):
    """<O_snk(x') J(y) O_src(r)^dag> summed over x', y with the phases of
    Eqs. (9)-(10); O_snk = qbar_1 Gs q_2, J = qbar_2 Gi q_3, O_src = qbar_1 Gsrc q_3,
    three distinct flavours (one connected contraction)."""
    V3 = M1.shape[0]
    r = ("r", 0)
    props = {}
    for x in range(V3):
        props[("f1", r, ("x", x))] = M1[x].reshape(4, 3, 4, 3)
        props[("f3", ("y", x), r)] = M3[x].reshape(4, 3, 4, 3)
        for y in range(V3):
            props[("f2", ("x", x), ("y", y))] = M2[x, y].reshape(4, 3, 4, 3)
    src_f = wick.bilinear(r, "f1", "f3", ("u1", "u2"), "k", "src")
    src_c = [(Gsrc, ("u1", "u2"))]
    bar_f, bar_c = wick.barred_conjugate(src_f, src_c, None, None, G4)
    fx = brute.phase(L, kp, (0, 0, 0), -1)
    fy = brute.phase(L, q, (0, 0, 0), +1)
    tot = 0j
    for x in range(V3):
        for y in range(V3):
            fields = (wick.bilinear(("x", x), "f1", "f2", ("a", "b"), "i", "snk")
                      + wick.bilinear(("y", y), "f2", "f3", ("c", "d"), "j", "J") + bar_f)
            coeffs = [(Gs, ("a", "b")), (Gi, ("c", "d"))] + bar_c
            tot += fx[x] * fy[y] * wick.expectation(fields, coeffs, props, ())
    return tot


def test_meson_default_source_is_the_conjugate_operator():
    L, V3 = (2, 1, 1), 2
    g = np.random.default_rng(21)
    G1 = _rand((12, 12, V3), g)
    G2 = _rand((V3, V3, 12, 12), g)
    G3 = _rand((12, 12, V3), g)
    kp, q = (1, 0, 0), (1, 0, 0)
    M1 = brute.g5_dagger(brute.site_matrices(G1))        # G1(r, x')
    M2 = brute.g5_dagger(np.swapaxes(G2, 0, 1))           # G2(x', y)
    M3 = brute.site_matrices(G3)                          # G3(y, r)
    C = brute.meson_spin_open(G1, G2, G3, L, kp, q).reshape(64, 64)
    g16 = oracle.gamma_basis16()
    Gs, Gi = _rand((4, 4), g), _rand((4, 4), g)
    default = oracle.gamma_project_meson(C, g_snk=Gs, g_ins=Gi)[0, 0]   # all 16 default sources
    for l in (1, 6, 11, 15):
        want = -_meson_wick(M1, M2, M3, L, kp, q, Gs, Gi, g16[l])
        assert abs(default[l] - want) < 1e-12 * abs(want), l
    # a random source matrix, and the mutants of its creation matrix
    Gr = _rand((4, 4), g)
    want = -_meson_wick(M1, M2, M3, L, kp, q, Gs, Gi, Gr)
    got = oracle.gamma_project_meson(C, Gs, Gi, oracle.creation_matrix(Gr))[0, 0, 0]
    assert abs(got - want) < 1e-12 * abs(want)
    for name, mut in MUTANTS.items():
        bad = oracle.gamma_project_meson(C, Gs, Gi, mut(Gr))[0, 0, 0]
        assert abs(bad - want) > 1e-3 * abs(want), name


def _nucleon_case(channel, seed):
    """Random propagators on V3 = 2 sites and the spin-open nucleon data of them."""
    L, V3 = (2, 1, 1), 2
    g = np.random.default_rng(seed)
    xs = [("x", n) for n in range(V3)]
    ys = [("y", n) for n in range(V3)]
    r = ("r", 0)
    Su = {x: _rand((4, 3, 4, 3), g) for x in xs}
    Sd = {x: _rand((4, 3, 4, 3), g) for x in xs}
    Sxy = {(x, y): _rand((4, 3, 4, 3), g) for x in xs for y in ys}
    Syr = {y: _rand((4, 3, 4, 3), g) for y in ys}
    props = {}
    for x in xs:
        props[("u", x, r)] = Su[x]
        props[("d", x, r)] = Sd[x]
        for y in ys:
            props[(channel, x, y)] = Sxy[(x, y)]
    for y in ys:
        props[(channel, y, r)] = Syr[y]
    site = lambda S: S.reshape(12, 12)
    G1 = np.stack([site(Su[x]) for x in xs], axis=-1)
    G2 = np.stack([site(Su[x] if channel == "d" else Sd[x]) for x in xs], axis=-1)
    G5 = np.kron(np.diag([1, 1, -1, -1]), np.eye(3))
    Gact_yx = np.stack([np.stack([G5 @ site(Sxy[(x, y)]).conj().T @ G5 for x in xs]) for y in ys])
    G3 = np.stack([site(Syr[y]) for y in ys], axis=-1)
    kp, q = (1, 0, 0), (1, 0, 0)
    T = brute.baryon_spin_open(G1, G2, Gact_yx, G3, L, kp, q).reshape(1024, 64)
    return L, xs, ys, r, props, T, kp, q, g


@pytest.mark.parametrize("channel", ["d", "u"])
def test_nucleon_default_abar_is_the_conjugate_operator(channel):
    L, xs, ys, r, props, T, kp, q, g = _nucleon_case(channel, 31 if channel == "d" else 32)
    A = _rand((4, 4), g)
    P = _rand((2, 4, 4), g)
    Gi = _rand((3, 4, 4), g)
    eps = oracle.EPS.astype(np.complex128)
    # chibar(r) = chi(r)^dag gamma4, chi(r)_g = eps (u^T A d) u_g, built field by field
    src_f = wick.proton(r, ("t1", "t2", "g'"), ("a'", "b'", "c'"), "src")
    src_c = [(eps, ("a'", "b'", "c'")), (A, ("t1", "t2"))]
    bar_f, bar_c = wick.barred_conjugate(src_f, src_c, "g'", "d", G4)
    want = np.zeros((2, 3), dtype=np.complex128)
    for x in xs:
        for y in ys:
            fields = (wick.proton(x, ("s1", "s2", "g"), ("a", "b", "c"), "snk")
                      + wick.current(y, channel, ("m", "n"), "e") + bar_f)
            coeffs = [(eps, ("a", "b", "c")), (A, ("s1", "s2")), (Gi, ("j", "m", "n")), (P, ("p", "d", "g"))] + bar_c
            ph = np.exp(-2j * np.pi * kp[0] * x[1] / L[0]) * np.exp(2j * np.pi * q[0] * y[1] / L[0])
            want += ph * wick.expectation(fields, coeffs, props, ("p", "j"))
    got = oracle.gamma_project_nucleon(T, channel, A=A, P=P, g_ins=Gi)     # default Abar
    scale = np.abs(want).max()
    assert np.abs(got - want).max() < 1e-12 * scale
    for name, mut in MUTANTS.items():
        bad = oracle.gamma_project_nucleon(T, channel, A=A, Abar=mut(A), P=P, g_ins=Gi)
        assert np.abs(bad - want).max() > 1e-3 * scale, name


def test_nucleon_default_channel_uses_c_gamma5():
    """The fully default proton channel (A = C gamma5, its conjugate, parity
    projectors, the 16 Gamma_ins) against the conjugate-built Wick contraction
    for one current matrix."""
    channel = "d"
    L, xs, ys, r, props, T, kp, q, g = _nucleon_case(channel, 33)
    A = oracle.charge_conjugation() @ (oracle.GAMMA[0] @ oracle.GAMMA[1] @ oracle.GAMMA[2] @ oracle.GAMMA[3])
    P = oracle.parity_projectors()
    Gi = oracle.gamma_basis16()[3:4]
    eps = oracle.EPS.astype(np.complex128)
    src_f = wick.proton(r, ("t1", "t2", "g'"), ("a'", "b'", "c'"), "src")
    bar_f, bar_c = wick.barred_conjugate(src_f, [(eps, ("a'", "b'", "c'")), (A, ("t1", "t2"))], "g'", "d", G4)
    want = np.zeros((2, 1), dtype=np.complex128)
    for x in xs:
        for y in ys:
            fields = (wick.proton(x, ("s1", "s2", "g"), ("a", "b", "c"), "snk")
                      + wick.current(y, channel, ("m", "n"), "e") + bar_f)
            coeffs = [(eps, ("a", "b", "c")), (A, ("s1", "s2")), (np.stack(Gi), ("j", "m", "n")),
                      (P, ("p", "d", "g"))] + bar_c
            ph = np.exp(-2j * np.pi * kp[0] * x[1] / L[0]) * np.exp(2j * np.pi * q[0] * y[1] / L[0])
            want += ph * wick.expectation(fields, coeffs, props, ("p", "j"))
    got = oracle.gamma_project_nucleon(T, channel)[:, 3:4]
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()
