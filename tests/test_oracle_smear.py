"""Pins of the oracle's gauge-covariant smearing.

* unit links: the smearing is a convolution, diagonal in momentum space with
  eigenvalue ((1 + 2 kappa sum_j cos(2 pi k_j / L_j)) / (1 + 6 kappa))^n, checked
  against numpy's FFT;
* hermiticity of one step with random SU(3) links, <phi, S psi> = <S phi, psi>
  (a link taken at the wrong site or without its dagger breaks it);
* gauge covariance: S[U^g](g psi) = g S[U](psi) for random SU(3) g(x);
* a brute-force loop over sites and directions on a tiny lattice;
* the propagator and vector layouts agree (rows of a propagator are colour
  vectors like noise vectors).
"""
import numpy as np

import c3pt_synth as syn
import oracle
from oracle import c3pt_oracle as core


def _links(L, seed):
    V3 = int(np.prod(L))
    g = np.random.default_rng(seed)
    return syn.haar_su3(4 * V3, g).reshape(4, V3, 3, 3).transpose(0, 2, 3, 1).copy()


def test_unit_links_is_fft_multiplier():
    L = (5, 4, 3)
    V3 = int(np.prod(L))
    kappa, n = 0.3, 7
    psi = syn.gaussian((2, 12, V3), np.random.default_rng(1))
    out = oracle.smear(psi, syn.unit_links(L), L, kappa, n, n_outer=8, n_inner=1)
    k1, k2, k3 = np.meshgrid(*(np.arange(l) for l in L), indexing="ij")
    lam = (1 + 2 * kappa * (np.cos(2 * np.pi * k1 / L[0]) + np.cos(2 * np.pi * k2 / L[1])
                            + np.cos(2 * np.pi * k3 / L[2]))) / (1 + 6 * kappa)
    lam = np.transpose(lam, (2, 1, 0))             # [k3][k2][k1], the order of the site index
    F = np.fft.fftn(psi.reshape(2, 12, L[2], L[1], L[0]), axes=(-3, -2, -1))
    want = np.fft.ifftn(F * lam ** n, axes=(-3, -2, -1)).reshape(2, 12, V3)
    assert np.allclose(out, want, atol=1e-12)


def test_one_step_is_hermitian():
    L = (3, 4, 3)
    V3 = int(np.prod(L))
    U = _links(L, 2)
    g = np.random.default_rng(3)
    a = syn.gaussian((1, 12, V3), g)
    b = syn.gaussian((1, 12, V3), g)
    Sa = oracle.smear(a, U, L, 0.4, 1, 4, 1)
    Sb = oracle.smear(b, U, L, 0.4, 1, 4, 1)
    assert np.isclose(np.vdot(b, Sa), np.vdot(Sb, a), rtol=1e-12)


def test_gauge_covariance():
    L = (4, 3, 3)
    V3 = int(np.prod(L))
    U = _links(L, 4)
    g = np.random.default_rng(5)
    Om = syn.haar_su3(V3, g)                        # [V3][3][3]
    psi = syn.gaussian((12, 12, V3), g)             # propagator slice, rows smeared
    Ug = np.empty_like(U)
    for j in range(3):
        Om_p = core._neighbour(np.moveaxis(Om, 0, -1), L, j, +1)      # [3][3][V3] at x + j
        Ug[j] = np.einsum('abx,bcx,dcx->adx', np.moveaxis(Om, 0, -1), U[j], np.conj(Om_p))
    Ug[3] = U[3]
    rot = lambda f: np.einsum('xcd,sdqx->scqx', Om, f.reshape(4, 3, 12, V3)).reshape(12, 12, V3)
    lhs = oracle.smear(rot(psi), Ug, L, 0.25, 3, 4, 12)
    rhs = rot(oracle.smear(psi, U, L, 0.25, 3, 4, 12))
    assert np.allclose(lhs, rhs, atol=1e-12)


def test_brute_force_loop():
    L = (3, 2, 2)
    V3 = int(np.prod(L))
    U = _links(L, 6)
    psi = syn.gaussian((1, 12, V3), np.random.default_rng(7))
    kappa = 0.35
    x = core.site_coords(L)
    idx = lambda c: int(c[0] % L[0] + L[0] * ((c[1] % L[1]) + L[1] * (c[2] % L[2])))
    v = psi.reshape(4, 3, V3)
    want = np.zeros_like(v)
    for n in range(V3):
        acc = v[:, :, n].copy()
        for j in range(3):
            e = np.zeros(3, dtype=int)
            e[j] = 1
            p, m = idx(x[n] + e), idx(x[n] - e)
            acc += kappa * (v[:, :, p] @ U[j][:, :, n].T + v[:, :, m] @ np.conj(U[j][:, :, m]))
        want[:, :, n] = acc / (1 + 6 * kappa)
    got = oracle.smear(psi, U, L, kappa, 1, 4, 1).reshape(4, 3, V3)
    assert np.allclose(got, want, atol=1e-13)


def test_propagator_rows_equal_vector_layout():
    L = (3, 3, 2)
    V3 = int(np.prod(L))
    U = _links(L, 8)
    G = syn.gaussian((12, 12, V3), np.random.default_rng(9))
    SG = oracle.smear(G, U, L, 0.2, 4, 4, 12)
    vec = np.ascontiguousarray(np.moveaxis(G, 1, 0))             # column q as a vector [q][12][V3]
    Sv = oracle.smear(vec, U, L, 0.2, 4, 48, 1)
    assert np.allclose(np.moveaxis(Sv, 0, 1), SG, atol=1e-13)
