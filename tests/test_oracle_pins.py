"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every test here runs on the CPU.  None of them re-types the oracle's own
formula as its expectation; each compares the factorized oracle with

* the direct trace of Eq. (1) evaluated with 12x12 matrices (oracle.brute),
* closed forms for special inputs (unit propagators, point noise, unit links),
* library routines (numpy FFT) over the full momentum set, and Parseval,
* symmetries: translation covariance, gauge invariance, epsilon symmetry,
* numbers the paper prints (tests/golden/paper_counts.json).
"""
import json
import os

import numpy as np
import pytest

import c3pt_synth as syn
import oracle
from oracle import brute
from oracle import c3pt_oracle as core

HERE = os.path.dirname(os.path.abspath(__file__))
G5 = oracle.GAMMA5_DIAG


def _rand(shape, seed):
    return syn.gaussian(shape, np.random.default_rng(seed))


def _unit_prop(V3):
    G = np.zeros((12, 12, V3), dtype=np.complex128)
    for A in range(12):
        G[A, A] = 1.0
    return G


def _full_momenta(L):
    return np.array([(k1, k2, k3) for k3 in range(L[2]) for k2 in range(L[1]) for k1 in range(L[0])])


# ----------------------------------------------------------------------------
# Conventions
# ----------------------------------------------------------------------------
def test_gamma_clifford_and_gamma5():
    g = oracle.GAMMA
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)
        for nu in range(4):
            ac = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(ac, 2.0 * (mu == nu) * np.eye(4))
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    assert np.allclose(g5, np.diag([1, 1, -1, -1]))
    basis = oracle.gamma_basis16()
    # the 16 products are linearly independent (a basis of 4x4 matrices)
    M = np.array([b.reshape(-1) for b in basis])
    assert np.linalg.matrix_rank(M) == 16


def test_momentum_counts_match_paper():
    with open(os.path.join(HERE, "golden", "paper_counts.json")) as f:
        gold = json.load(f)
    ks = oracle.momenta(gold["n2max"])
    assert len(ks) == gold["n_momenta"]
    assert len(ks) ** 2 == gold["n_combinations"]
    # further counts used by the workloads: |k|^2<=3 -> 27, <=6 -> 81, <=9 -> 123
    assert [len(oracle.momenta(n)) for n in (0, 3, 6, 9)] == [1, 27, 81, 123]
    n2 = (ks ** 2).sum(1)
    assert np.all(np.diff(n2) >= 0)
    assert len({tuple(k) for k in ks}) == len(ks)


# ----------------------------------------------------------------------------
# Projection: k = 0 site sum, FFT over the full momentum set, Parseval
# ----------------------------------------------------------------------------
L_NC = (3, 2, 4)   # non-cubic on purpose: catches swapped axes


def _per_site_spectator(G, eta, L):
    """Unprojected spectator tensor per site, by plain loops (brute force)."""
    V3 = eta.shape[-1]
    N = eta.shape[0]
    P = np.zeros((N, 4, 4, 4, 3, V3), dtype=np.complex128)
    for i in range(N):
        for x in range(V3):
            for bp in range(4):
                for ap in range(4):
                    for a in range(4):
                        for cs in range(3):
                            acc = 0j
                            for c in range(3):
                                # [gamma5 eta]^{b'}_c * [gamma5 G^dag gamma5]^{a' a}_{c cs}
                                acc += (G5[bp] * eta[i, 3 * bp + c, x]) * (
                                    G5[ap] * np.conj(G[3 * ap + c, 3 * a + cs, x]) * G5[a])
                            P[i, bp, ap, a, cs, x] = acc
    return P.reshape(N, 192, V3)


def test_spectator_zero_momentum_is_site_sum():
    V3 = int(np.prod(L_NC))
    G = _rand((12, 12, V3), 1)
    eta = _rand((2, 12, V3), 2)
    S = oracle.spectator_meson(G, eta, L_NC, [[0, 0, 0]])
    P = _per_site_spectator(G, eta, L_NC)
    assert np.allclose(S[:, 0, :], P.sum(-1), rtol=0, atol=1e-12)


def test_spectator_full_momenta_is_fft():
    """With G = 1 the spectator is delta_{a'a} g[b'] (FT^- of eta); over all k in
    [0, L)^3 the sign -1 transform is numpy's forward fftn."""
    L = L_NC
    V3 = int(np.prod(L))
    eta = _rand((1, 12, V3), 3)
    k = _full_momenta(L)
    S = oracle.spectator_meson(_unit_prop(V3), eta, L, k)          # [1][V3][192]
    S = S.reshape(V3, 4, 4, 4, 3)
    e = eta[0].reshape(4, 3, L[2], L[1], L[0])
    F = np.fft.fftn(e, axes=(-3, -2, -1))                          # [b'][c][k3][k2][k1]
    F = F.reshape(4, 3, V3).transpose(2, 0, 1)                      # k index = k1 + L1(k2 + L2 k3)
    for ap in range(4):
        for a in range(4):
            want = (G5[None, :, None] * F) if ap == a else np.zeros_like(F)
            assert np.allclose(S[:, :, ap, a, :], want, atol=1e-11)


def test_insertion_full_momenta_is_inverse_fft():
    """With G = 1 the insertion is delta_{bt b} g[at] (V3 * ifftn of conj s)."""
    L = L_NC
    V3 = int(np.prod(L))
    s = _rand((1, 12, V3), 4)
    k = _full_momenta(L)
    I = oracle.insertion({0: _unit_prop(V3)}, {0: s}, [0], L, 1, k)   # [1][1][1][V3][192]
    I = I[0, 0, 0].reshape(V3, 4, 4, 4, 3)
    e = np.conj(s[0]).reshape(4, 3, L[2], L[1], L[0])
    F = V3 * np.fft.ifftn(e, axes=(-3, -2, -1))
    F = F.reshape(4, 3, V3).transpose(2, 0, 1)
    for bt in range(4):
        for b in range(4):
            want = (G5[None, :, None] * F) if bt == b else np.zeros_like(F)
            assert np.allclose(I[:, :, bt, b, :], want, atol=1e-11)


def test_parseval_spectator_and_insertion():
    L = L_NC
    V3 = int(np.prod(L))
    G = _rand((12, 12, V3), 5)
    eta = _rand((1, 12, V3), 6)
    k = _full_momenta(L)
    S = oracle.spectator_meson(G, eta, L, k)
    P = _per_site_spectator(G, eta, L)
    assert np.isclose((np.abs(S) ** 2).sum(), V3 * (np.abs(P) ** 2).sum(), rtol=1e-12)
    s = _rand((1, 12, V3), 7)
    I = oracle.insertion({0: G}, {0: s}, [0], L, 1, k)
    # per-site insertion via single-site masks and k = 0 (linearity of the site sum)
    tot = 0.0
    for x in range(V3):
        m = np.zeros_like(s)
        m[..., x] = s[..., x]
        tot += (np.abs(oracle.insertion({0: G}, {0: m}, [0], L, 1, [[0, 0, 0]])) ** 2).sum()
    assert np.isclose((np.abs(I) ** 2).sum(), V3 * tot, rtol=1e-12)


def test_point_noise_closed_form():
    """eta = e_A delta_{x,x0}: S is one gamma5-signed conjugated row block of G(x0)
    times the phase at x0."""
    L = (4, 3, 2)
    V3 = int(np.prod(L))
    G = _rand((12, 12, V3), 8)
    x0 = 17
    A = 3 * 2 + 1      # spin 2, colour 1
    eta = np.zeros((1, 12, V3), dtype=np.complex128)
    eta[0, A, x0] = 1.0
    k = oracle.momenta(3)
    r = (1, 2, 0)
    S = oracle.spectator_meson(G, eta, L, k, r).reshape(len(k), 4, 4, 4, 3)
    xc = core.site_coords(L)[x0]
    ph = np.exp(-2j * np.pi * (((xc - np.array(r)) / np.array(L)) @ k.T))
    want = np.zeros((len(k), 4, 4, 4, 3), dtype=np.complex128)
    for ap in range(4):
        for a in range(4):
            for cs in range(3):
                want[:, 2, ap, a, cs] = ph * G5[2] * G5[ap] * G5[a] * np.conj(G[3 * ap + 1, 3 * a + cs, x0])
    assert np.allclose(S, want, atol=1e-13)


# ----------------------------------------------------------------------------
# Brute-force Eq. (1): the factorized estimator reproduces the direct trace
# ----------------------------------------------------------------------------
def _meson_setup(L, N, seed, T=4, n_ops=1, taus=(1, 2)):
    V3 = int(np.prod(L))
    g = np.random.default_rng(seed)
    G1 = syn.gaussian((12, 12, V3), g)
    G3 = {t: syn.gaussian((12, 12, V3), g) for t in range(T)}
    eta = syn.z2z2_noise(L, N, 900 + seed, 0)
    s = {t: syn.gaussian((N, 12, V3), g) for t in range(T)}
    U = {t: syn.haar_su3(4 * V3, g).reshape(4, V3, 3, 3).transpose(0, 2, 3, 1).copy() for t in range(T)}
    return V3, G1, G3, eta, s, U


@pytest.mark.parametrize("L,r", [((2, 3, 2), (0, 0, 0)), ((3, 2, 2), (1, 1, 0))])
def test_factorized_equals_bruteforce_trace(L, r):
    N = 3
    T = 4
    taus = [1, 2]
    V3, G1, G3, eta, s, _ = _meson_setup(L, N, 11)
    w = np.array([0.5, 0.3, 0.2])
    kp = oracle.momenta(1)[:4]
    q = oracle.momenta(2)[[0, 2, 5]]
    S = oracle.spectator_meson(G1, eta, L, kp, r)
    I = oracle.insertion(G3, s, taus, L, T, q, r)
    pairs = [(0, 0), (1, 2), (3, 1)]
    C = oracle.combine(S, I, w=w, pairs=pairs)          # [pair][tau][op][64][64]
    basis = oracle.gamma_basis16()
    rng = np.random.default_rng(5)
    for j, (p, qq) in enumerate(pairs):
        for it, tau in enumerate(taus):
            Ghat = np.einsum('i,iAy,iBx->yxAB', w, s[tau], np.conj(eta))   # G2(y, x')
            Cb = brute.meson_spin_open(G1, Ghat, G3[tau], L, kp[p], q[qq], r)
            Cf = C[j, it, 0].reshape(4, 4, 4, 4, 4, 4)
            assert np.allclose(Cf, Cb, atol=1e-12 * np.abs(Cb).max())
            # and against the plain 12x12 trace of Eq. (1) for random Gammas
            gs, gi, gc = (basis[i] for i in rng.integers(0, 16, 3))
            tr = brute.meson_trace(G1, Ghat, G3[tau], L, kp[p], q[qq], gs, gi, gc, r)
            # C indices: [b'][a'][a][at][bt][b]; trace weights Gsnk^{a'b'} Gins^{at bt} Gsrc^{b a}
            val = np.einsum('qpauts,pq,ut,sa->', Cf, gs, gi, gc)
            assert np.isclose(val, tr, rtol=1e-12, atol=1e-12)


def test_full_dilution_reproduces_exact_propagator():
    """Complete dilution (one unit noise vector per spin, colour and site on t_f,
    w = 1) with s_j = G2 eta_j: the factorized result equals the trace with the
    exact all-to-all G2."""
    L = (2, 2, 2)
    V3 = 8
    g = np.random.default_rng(21)
    G1 = syn.gaussian((12, 12, V3), g)
    G3 = syn.gaussian((12, 12, V3), g)
    G2 = syn.gaussian((V3, V3, 12, 12), g)          # exact G2(y, x') [y][x'][A][B]
    N = 12 * V3
    eta = np.zeros((N, 12, V3), dtype=np.complex128)
    for j in range(N):
        eta[j, j % 12, j // 12] = 1.0
    s = np.einsum('yxAB,jBx->jAy', G2, eta)
    kp = oracle.momenta(1)
    q = oracle.momenta(1)
    S = oracle.spectator_meson(G1, eta, L, kp)
    I = oracle.insertion({0: G3}, {0: s}, [0], L, 1, q)
    C = oracle.combine(S, I, w=np.ones(N), pairs=[(2, 5), (0, 0)])
    for j, (p, qq) in enumerate([(2, 5), (0, 0)]):
        Cb = brute.meson_spin_open(G1, G2, G3, L, kp[p], q[qq])
        assert np.allclose(C[j, 0, 0].reshape((4,) * 6), Cb, atol=1e-12 * np.abs(Cb).max())


# ----------------------------------------------------------------------------
# Derivative insertion
# ----------------------------------------------------------------------------
def test_derivative_unit_links_is_central_difference():
    L = (3, 4, 2)
    T = 4
    V3, _, G3, _, s, _ = _meson_setup(L, 2, 31)
    U1 = {t: syn.unit_links(L) for t in range(T)}
    k = oracle.momenta(2)
    I = oracle.insertion(G3, s, [1, 3], L, T, k, U_t=U1, n_ops=5)
    for it, tau in enumerate([1, 3]):
        for nu in range(4):
            if nu < 3:
                arr = G3[tau].reshape(12, 12, L[2], L[1], L[0])
                ax = {0: -1, 1: -2, 2: -3}[nu]
                Gp = np.roll(arr, -1, axis=ax).reshape(12, 12, V3)
                Gm = np.roll(arr, +1, axis=ax).reshape(12, 12, V3)
            else:
                Gp, Gm = G3[(tau + 1) % T], G3[(tau - 1) % T]
            Ip = oracle.insertion({0: Gp}, {0: s[tau]}, [0], L, 1, k)
            Im = oracle.insertion({0: Gm}, {0: s[tau]}, [0], L, 1, k)
            assert np.allclose(I[:, it, 1 + nu], 0.5 * (Ip - Im)[:, 0, 0], atol=1e-12)


def test_derivative_matches_matrix_form():
    """The oracle's covariant derivative equals the explicit kron(1, U) matrix form."""
    L = (3, 2, 2)
    T = 3
    V3, _, G3, _, _, U = _meson_setup(L, 1, 41, T=T)
    for nu in range(4):
        D = oracle.covariant_derivative(G3, U, L, T, 1, nu)
        Db = brute.derivative_field(G3, U, L, T, 1, nu)
        assert np.allclose(np.moveaxis(D, -1, 0), Db, atol=1e-13)


def test_derivative_trace_against_bruteforce():
    L = (2, 2, 3)
    T = 4
    N = 2
    V3, G1, G3, eta, s, U = _meson_setup(L, N, 51, T=T)
    kp = oracle.momenta(1)[[0, 3]]
    q = oracle.momenta(1)[[1, 4]]
    S = oracle.spectator_meson(G1, eta, L, kp)
    I = oracle.insertion(G3, s, [2], L, T, q, U_t=U, n_ops=5)
    C = oracle.combine(S, I, pairs=[(1, 0), (0, 1)])
    w = np.full(N, 1.0 / N)
    Ghat = np.einsum('i,iAy,iBx->yxAB', w, s[2], np.conj(eta))
    for j, (p, qq) in enumerate([(1, 0), (0, 1)]):
        for nu in range(4):
            DG = brute.derivative_field(G3, U, L, T, 2, nu)           # [V3][12][12]
            Cb = brute.meson_spin_open(G1, Ghat, np.moveaxis(DG, 0, -1), L, kp[p], q[qq])
            assert np.allclose(C[j, 0, 1 + nu].reshape((4,) * 6), Cb, atol=1e-12 * np.abs(Cb).max())


def _left_derivative_G2(Ghat_t, U, L, T, tau, nu):
    """(D_nu G2)(y, x') on the y index of G2(y, x') = [V3_y][V3_x'][12][12] per
    timeslice, through brute.derivative_field with (x', column) as the columns."""
    V3 = Ghat_t[tau].shape[0]
    F = {t: np.ascontiguousarray(g.transpose(2, 1, 3, 0).reshape(12, V3 * 12, V3)) for t, g in Ghat_t.items()}
    D = brute.derivative_field(F, U, L, T, tau, nu)                   # [V3_y][12][V3_x' * 12]
    return D.reshape(V3, 12, V3, 12).transpose(0, 2, 1, 3)


@pytest.mark.parametrize("r", [(0, 0, 0), (1, 0, 1)])
def test_symmetric_derivative_trace_against_bruteforce(r):
    """<->D_nu = 1/2 (->D_nu - <-D_nu): the left derivative acts on the end of
    G_f2(x', y) at the insertion, (G_f2 <-D)(x', y) = 1/2 [G_f2(x', y+nu) U_nu(y)^dag
    - G_f2(x', y-nu) U_nu(y-nu)], built here on the stochastic estimate of G2 with
    explicit neighbour lookups and kron(1, U) matrices, then traced as Eq. (1)."""
    L = (3, 3, 3)
    T = 4
    N = 2
    V3, G1, G3, eta, s, U = _meson_setup(L, N, 57, T=T)
    kp = oracle.momenta(1)[[0, 2]]
    q = oracle.momenta(1)[[3, 5]]
    tau = 3
    S = oracle.spectator_meson(G1, eta, L, kp, r)
    I = oracle.insertion(G3, s, [tau], L, T, q, r=r, U_t=U, n_ops=9)
    C = oracle.combine(S, I, pairs=[(1, 0), (0, 1)])
    w = np.full(N, 1.0 / N)
    Ghat = {t: np.einsum('i,iAy,iBx->yxAB', w, s[t], np.conj(eta)) for t in range(T)}
    for j, (p, qq) in enumerate([(1, 0), (0, 1)]):
        for nu in range(4):
            DG3 = np.moveaxis(brute.derivative_field(G3, U, L, T, tau, nu), 0, -1)
            right = brute.meson_spin_open(G1, Ghat[tau], DG3, L, kp[p], q[qq], r=r)
            left = brute.meson_spin_open(G1, _left_derivative_G2(Ghat, U, L, T, tau, nu), G3[tau], L, kp[p],
                                         q[qq], r=r)
            Cb = 0.5 * (right - left)
            got = C[j, 0, 5 + nu].reshape((4,) * 6)
            assert np.allclose(got, Cb, atol=1e-12 * np.abs(Cb).max())
            assert np.allclose(C[j, 0, 1 + nu].reshape((4,) * 6), right, atol=1e-12 * np.abs(right).max())


def test_symmetric_derivative_total_derivative_identity():
    """Summation by parts over a periodic direction: at insertion momentum
    q_nu = 0 the site sum of ->D_nu + <-D_nu vanishes (a total derivative), so
    <->D_nu = ->D_nu there; at q_nu != 0 it does not."""
    L = (3, 4, 3)
    T = 4
    V3, _, G3, _, s, U = _meson_setup(L, 2, 59, T=T)
    q = np.array([[0, 0, 0], [0, 1, 0], [1, 0, 2], [2, 3, 0]])
    I = oracle.insertion(G3, s, [2], L, T, q, U_t=U, n_ops=9)
    for m, qm in enumerate(q):
        for nu in range(3):
            fwd, sym = I[:, 0, 1 + nu, m], I[:, 0, 5 + nu, m]
            if qm[nu] == 0:
                assert np.allclose(sym, fwd, atol=1e-12 * np.abs(fwd).max())
            else:
                assert not np.allclose(sym, fwd, atol=1e-3 * np.abs(fwd).max())


def test_two_derivatives_trace_against_bruteforce():
    """Ops 5 + 4 rho + nu = D_nu D_rho: the brute-force matrix form of the
    covariant derivative applied twice (to a dict of once-derived slices),
    traced as Eq. (1) against the factorized estimator."""
    L = (3, 2, 3)
    T = 6
    N = 2
    V3, G1, G3, eta, s, U = _meson_setup(L, N, 53, T=T)
    kp = oracle.momenta(1)[[0, 4]]
    q = oracle.momenta(1)[[2, 6]]
    tau = 2
    S = oracle.spectator_meson(G1, eta, L, kp)
    I = oracle.insertion(G3, s, [tau], L, T, q, U_t=U, n_ops=21)
    C = oracle.combine(S, I, pairs=[(1, 0), (0, 1)])
    w = np.full(N, 1.0 / N)
    Ghat = np.einsum('i,iAy,iBx->yxAB', w, s[tau], np.conj(eta))
    for rho in range(4):
        D1 = {t: np.ascontiguousarray(np.moveaxis(brute.derivative_field(G3, U, L, T, t, rho), 0, -1))
              for t in (tau - 1, tau, tau + 1)}
        for nu in range(4):
            DD = brute.derivative_field(D1, U, L, T, tau, nu)          # [V3][12][12]
            for j, (p, qq) in enumerate([(1, 0), (0, 1)]):
                Cb = brute.meson_spin_open(G1, Ghat, np.moveaxis(DD, 0, -1), L, kp[p], q[qq])
                got = C[j, 0, 5 + 4 * rho + nu].reshape((4,) * 6)
                assert np.allclose(got, Cb, atol=1e-12 * np.abs(Cb).max())


def test_symmetrized_two_derivatives_trace_against_bruteforce():
    """Ops 21 + 4 mu + nu = <->D_mu <->D_nu = 1/4 (->->  - ->D_mu <-D_nu - <-D_mu ->D_nu + <-<-):
    every term traced as Eq. (1) with the right derivatives on G_f3 and the left
    ones on the end of G_f2(x', y) at the insertion (matrix form, applied to
    the stochastic estimate of G2 in the order they act)."""
    L = (3, 3, 2)
    T = 7
    N = 2
    V3, G1, G3, eta, s, U = _meson_setup(L, N, 56, T=T)
    kp = oracle.momenta(1)[[0, 5]]
    q = oracle.momenta(1)[[1, 6]]
    tau = 3
    S = oracle.spectator_meson(G1, eta, L, kp)
    I = oracle.insertion(G3, s, [tau], L, T, q, U_t=U, n_ops=37)
    C = oracle.combine(S, I, pairs=[(1, 0), (0, 1)])
    w = np.full(N, 1.0 / N)
    Ghat = {t: np.einsum('i,iAy,iBx->yxAB', w, s[t], np.conj(eta)) for t in range(T)}
    DG3 = {nu: {t: np.ascontiguousarray(np.moveaxis(brute.derivative_field(G3, U, L, T, t, nu), 0, -1))
                for t in (tau - 1, tau, tau + 1)} for nu in range(4)}
    # left derivative mu on G2's y end, on the slices next to tau
    DG2 = {mu: {t: _left_derivative_G2(Ghat, U, L, T, t, mu) for t in (tau - 1, tau, tau + 1)} for mu in range(4)}
    for mu in range(4):
        for nu in range(4):
            DDG3 = np.moveaxis(brute.derivative_field(DG3[nu], U, L, T, tau, mu), 0, -1)   # D_mu D_nu G3
            DDG2 = _left_derivative_G2(DG2[mu], U, L, T, tau, nu)                          # <-D_mu then <-D_nu
            for j, (p, qq) in enumerate([(1, 0), (0, 1)]):
                args = (L, kp[p], q[qq])
                rr = brute.meson_spin_open(G1, Ghat[tau], DDG3, *args)
                lr = brute.meson_spin_open(G1, DG2[mu][tau], DG3[nu][tau], *args)
                rl = brute.meson_spin_open(G1, DG2[nu][tau], DG3[mu][tau], *args)
                ll = brute.meson_spin_open(G1, DDG2, G3[tau], *args)
                Cb = 0.25 * (rr - lr - rl + ll)
                got = C[j, 0, 21 + 4 * mu + nu].reshape((4,) * 6)
                assert np.allclose(got, Cb, atol=1e-12 * np.abs(Cb).max())


def test_symmetrized_two_derivatives_summation_by_parts():
    """At insertion momentum with q_mu = q_nu = 0 (spatial mu, nu) a left
    derivative moves onto the right with a minus sign, so
    <->D_mu <->D_nu = 1/4 (3 D_mu D_nu + D_nu D_mu) there (random links: the two
    orders differ)."""
    L = (3, 4, 3)
    T = 7
    V3, _, G3, _, s, U = _meson_setup(L, 2, 58, T=T)
    q = np.array([[0, 0, 0], [0, 0, 1]])
    I = oracle.insertion(G3, s, [3], L, T, q, U_t=U, n_ops=37)[:, 0]
    for m, qm in enumerate(q):
        for mu in range(3):
            for nu in range(3):
                if qm[mu] or qm[nu]:
                    continue
                dd = I[:, 5 + 4 * nu + mu, m]          # D_mu D_nu
                dd_rev = I[:, 5 + 4 * mu + nu, m]      # D_nu D_mu
                want = 0.25 * (3 * dd + dd_rev)
                assert np.allclose(I[:, 21 + 4 * mu + nu, m], want, atol=1e-12 * np.abs(want).max())


def test_two_derivatives_commute_with_unit_links():
    """With unit links the lattice derivatives are commuting difference
    operators: D_nu D_rho = D_rho D_nu, and D_nu D_nu is the second difference
    over two sites, (G(y+2nu) - 2 G(y) + G(y-2nu)) / 4."""
    L = (4, 5, 4)
    T = 6
    V3, _, G3, _, s, _ = _meson_setup(L, 1, 54, T=T)
    U1 = {t: syn.unit_links(L) for t in range(T)}
    k = oracle.momenta(2)
    I = oracle.insertion(G3, s, [2], L, T, k, U_t=U1, n_ops=21)[:, 0]
    for rho in range(4):
        for nu in range(4):
            assert np.allclose(I[:, 5 + 4 * rho + nu], I[:, 5 + 4 * nu + rho], atol=1e-12)
    for nu in range(4):
        if nu < 3:
            arr = G3[2].reshape(12, 12, L[2], L[1], L[0])
            ax = {0: -1, 1: -2, 2: -3}[nu]
            Gp2 = np.roll(arr, -2, axis=ax).reshape(12, 12, V3)
            Gm2 = np.roll(arr, +2, axis=ax).reshape(12, 12, V3)
        else:
            Gp2, Gm2 = G3[4], G3[0]
        D2 = (Gp2 - 2 * G3[2] + Gm2) / 4
        want = oracle.insertion({0: D2}, {0: s[2]}, [0], L, 1, k)[:, 0, 0]
        assert np.allclose(I[:, 5 + 5 * nu], want, atol=1e-12)


def test_vector_derivative_matches_propagator_derivative():
    """D_nu on the colour vectors of s equals D_nu on a propagator whose columns are them."""
    L = (3, 2, 2)
    T = 3
    V3, _, _, _, s, U = _meson_setup(L, 2, 58, T=T)
    for nu in range(4):
        Dv = oracle.covariant_derivative_vector(s, U, L, T, 1, nu)         # [N][12][V3]
        Gs = {t: np.ascontiguousarray(np.moveaxis(v, 0, 1)) for t, v in s.items()}   # [12][N][V3]
        Dg = brute.derivative_field(Gs, U, L, T, 1, nu)                    # [V3][12][N]
        assert np.allclose(np.moveaxis(Dv, -1, 0), np.moveaxis(Dg, 2, 1), atol=1e-13)


# ----------------------------------------------------------------------------
# Symmetries: translation covariance and gauge invariance
# ----------------------------------------------------------------------------
def _shift_field(f, L, d):
    """f'(x) = f(x - d) (periodic), f[..., V3]."""
    arr = f.reshape(f.shape[:-1] + (L[2], L[1], L[0]))
    arr = np.roll(arr, shift=(d[2], d[1], d[0]), axis=(-3, -2, -1))
    return arr.reshape(f.shape)


def test_translation_covariance():
    L = (4, 3, 2)
    T = 4
    N = 2
    V3, G1, G3, eta, s, U = _meson_setup(L, N, 61, T=T)
    G1b = syn.gaussian((12, 12, V3), np.random.default_rng(3))
    k = oracle.momenta(3)
    r = (1, 0, 1)
    d = (2, 1, 1)
    r2 = tuple((r[j] + d[j]) for j in range(3))
    sh = lambda f: _shift_field(f, L, d)
    S = oracle.spectator_meson(G1, eta, L, k, r)
    S2 = oracle.spectator_meson(sh(G1), sh(eta), L, k, r2)
    assert np.allclose(S, S2, atol=1e-12)
    B = oracle.spectator_baryon(G1, G1b, eta, L, k[:5], r)
    B2 = oracle.spectator_baryon(sh(G1), sh(G1b), sh(eta), L, k[:5], r2)
    assert np.allclose(B, B2, atol=1e-11)
    I = oracle.insertion(G3, s, [1, 2], L, T, k, r, U_t=U, n_ops=5)
    I2 = oracle.insertion({t: sh(G3[t]) for t in G3}, {t: sh(s[t]) for t in s}, [1, 2], L, T, k, r2,
                          U_t={t: sh(U[t]) for t in U}, n_ops=5)
    assert np.allclose(I, I2, atol=1e-11)
    # absolute phases instead: the shift shows up as exp(-+ 2 pi i k.d / L)
    S0 = oracle.spectator_meson(sh(G1), sh(eta), L, k, r)
    fac = np.exp(-2j * np.pi * (k @ (np.array(d) / np.array(L))))
    assert np.allclose(S0, S * fac[None, :, None], atol=1e-12)


def _gauge_transform(L, T, G1, G1b, G3, eta, s, U, seed):
    V3 = int(np.prod(L))
    g = np.random.default_rng(seed)
    Om = {t: syn.haar_su3(V3, g) for t in range(T)}      # [V3][3][3] per slice
    Omr = syn.haar_su3(1, g)[0]                          # at the source point

    def prop(G, t):
        Gr = G.reshape(4, 3, 4, 3, V3)
        x = np.einsum('xce,sejdx->scjdx', Om[t], Gr)
        x = np.einsum('scjdx,fd->scjfx', x, np.conj(Omr))   # G Om(r)^dag: col colour
        return x.reshape(12, 12, V3)

    def vec(v, t):
        vr = v.reshape(v.shape[0], 4, 3, V3)
        return np.einsum('xce,isex->iscx', Om[t], vr).reshape(v.shape)

    def links(Ut, t):
        out = np.empty_like(Ut)
        for mu in range(4):
            if mu < 3:
                e = [0, 0, 0]
                e[mu] = 1
                # Om(x + mu): value at x of the field shifted by -mu
                Omp = np.moveaxis(_shift_field(np.moveaxis(Om[t], 0, -1), L, [-v for v in e]), -1, 0)
            else:
                Omp = Om[(t + 1) % T]
            out[mu] = np.einsum('xce,edx,xfd->cfx', Om[t], Ut[mu], np.conj(Omp))
        return out

    t_f = T - 1
    return (prop(G1, t_f), prop(G1b, t_f), {t: prop(G3[t], t) for t in G3}, vec(eta, t_f),
            {t: vec(s[t], t) for t in s}, {t: links(U[t], t) for t in U})


def test_gauge_invariance_of_combine():
    L = (2, 3, 2)
    T = 4
    N = 2
    V3, G1, G3, eta, s, U = _meson_setup(L, N, 71, T=T)
    G1b = syn.gaussian((12, 12, V3), np.random.default_rng(72))
    kp = oracle.momenta(2)[:4]
    q = oracle.momenta(2)[3:7]
    taus = [0, 1, 2]

    def run(G1, G1b, G3, eta, s, U):
        S = oracle.spectator_meson(G1, eta, L, kp)
        B = oracle.spectator_baryon(G1, G1b, eta, L, kp)
        I = oracle.insertion(G3, s, taus, L, T, q, U_t=U, n_ops=9)
        return oracle.combine(S, I), oracle.combine(B, I), S, I

    C, CB, S, I = run(G1, G1b, G3, eta, s, U)
    C2, CB2, S2, I2 = run(*_gauge_transform(L, T, G1, G1b, G3, eta, s, U, 73))
    assert np.allclose(C, C2, atol=1e-12 * np.abs(C).max())
    assert np.allclose(CB, CB2, atol=1e-12 * np.abs(CB).max())
    # the parts alone are not invariant (their source colour rotates)
    assert not np.allclose(S, S2, atol=1e-6)
    assert not np.allclose(I, I2, atol=1e-6)


# ----------------------------------------------------------------------------
# Baryon
# ----------------------------------------------------------------------------
def test_baryon_unit_propagators_closed_form():
    """G1 = G2 = 1: sum_{ab} eps_abc eps_abc' = 2 delta_cc', so
    S^B = 2 delta_{a1'a1} delta_{a2'a2} sum_x phi g[b'] eta[(b', c')]."""
    L = (3, 2, 2)
    V3 = 12
    eta = _rand((2, 12, V3), 81)
    k = oracle.momenta(2)
    B = oracle.spectator_baryon(_unit_prop(V3), _unit_prop(V3), eta, L, k).reshape(2, len(k), 4, 4, 4, 4, 4, 3)
    ph = oracle.phase_matrix(L, k, (0, 0, 0), -1)
    fe = np.einsum('mx,iAx->imA', ph, eta).reshape(2, len(k), 4, 3) * G5[None, None, :, None]
    want = np.zeros_like(B)
    for a1 in range(4):
        for a2 in range(4):
            want[:, :, a1, a1, a2, a2] = 2.0 * fe
    assert np.allclose(B, want, atol=1e-12)


def test_baryon_exchange_symmetry():
    L = (2, 2, 3)
    V3 = 12
    G1 = _rand((12, 12, V3), 82)
    G2 = _rand((12, 12, V3), 83)
    eta = _rand((1, 12, V3), 84)
    k = oracle.momenta(1)
    B12 = oracle.spectator_baryon(G1, G2, eta, L, k).reshape(1, len(k), 4, 4, 4, 4, 4, 3)
    B21 = oracle.spectator_baryon(G2, G1, eta, L, k).reshape(1, len(k), 4, 4, 4, 4, 4, 3)
    assert np.allclose(B12, B21.transpose(0, 1, 4, 5, 2, 3, 6, 7), atol=1e-12)


def test_baryon_factorized_equals_bruteforce():
    L = (2, 2, 2)
    V3 = 8
    N = 2
    g = np.random.default_rng(91)
    G1 = syn.gaussian((12, 12, V3), g)
    G2 = syn.gaussian((12, 12, V3), g)
    G3 = syn.gaussian((12, 12, V3), g)
    eta = syn.z2z2_noise(L, N, 92, 0)
    s = syn.gaussian((N, 12, V3), g)
    w = np.array([0.7, 0.3])
    kp = oracle.momenta(1)[[0, 2]]
    q = oracle.momenta(1)[[4, 1]]
    B = oracle.spectator_baryon(G1, G2, eta, L, kp)
    I = oracle.insertion({0: G3}, {0: s}, [0], L, 1, q)
    C = oracle.combine(B, I, w=w, pairs=[(0, 1), (1, 0)])
    Ghat = np.einsum('i,iAy,iBx->yxAB', w, s, np.conj(eta))
    for j, (p, qq) in enumerate([(0, 1), (1, 0)]):
        Cb = brute.baryon_spin_open(G1, G2, Ghat, G3, L, kp[p], q[qq])
        assert np.allclose(C[j, 0, 0].reshape((4,) * 8), Cb, atol=1e-12 * np.abs(Cb).max())


# ----------------------------------------------------------------------------
# Combine bookkeeping
# ----------------------------------------------------------------------------
def test_combine_linear_in_weights_and_pairs_subset():
    L = (2, 2, 2)
    V3, G1, G3, eta, s, U = _meson_setup(L, 3, 101, T=3)
    k = oracle.momenta(1)
    S = oracle.spectator_meson(G1, eta, L, k)
    I = oracle.insertion(G3, s, [0, 1], L, 3, k, U_t=U, n_ops=5)
    w1 = np.array([1.0, 0.0, 0.0])
    w2 = np.array([0.0, 2.0, -1.0])
    Ca = oracle.combine(S, I, w=w1 + w2)
    assert np.allclose(Ca, oracle.combine(S, I, w=w1) + oracle.combine(S, I, w=w2), atol=1e-13)
    pairs = [(3, 1), (0, 6), (6, 6)]
    Cp = oracle.combine(S, I, pairs=pairs, op_begin=1, op_end=4)
    Call = oracle.combine(S, I)
    for j, (p, q) in enumerate(pairs):
        assert np.allclose(Cp[j], Call[p * 7 + q][:, 1:4], atol=1e-14)


# ----------------------------------------------------------------------------
# The pins have teeth: a planted mistake in the oracle is caught.
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("mutation", ["no_gamma5", "no_conj", "wrong_sign"])
def test_planted_mistake_fails_bruteforce(monkeypatch, mutation):
    L = (3, 2, 3)      # L = 2 would make every phase real and hide a sign flip
    N = 2
    V3, G1, G3, eta, s, _ = _meson_setup(L, N, 111, T=2)
    kp = oracle.momenta(1)[[1]]
    q = oracle.momenta(1)[[2]]
    if mutation == "no_gamma5":
        monkeypatch.setattr(core, "GAMMA5_DIAG", np.ones(4))
    elif mutation == "no_conj":
        monkeypatch.setattr(core.np, "conj", lambda x: x)
    else:
        orig = core.phase_matrix
        monkeypatch.setattr(core, "phase_matrix", lambda L, k, r, sg, sites=None: orig(L, k, r, -sg, sites))
    S = oracle.spectator_meson(G1, eta, L, kp)
    I = oracle.insertion(G3, s, [1], L, 2, q)
    C = oracle.combine(S, I)
    monkeypatch.undo()
    w = np.full(N, 1.0 / N)
    Ghat = np.einsum('i,iAy,iBx->yxAB', w, s[1], np.conj(eta))
    Cb = brute.meson_spin_open(G1, Ghat, G3[1], L, kp[0], q[0])
    assert not np.allclose(C[0, 0, 0].reshape((4,) * 6), Cb, atol=1e-6 * np.abs(Cb).max())


# ----------------------------------------------------------------------------
# Forward and backward diagrams with time-partitioned noise
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("t_fwd,t_src,t_bwd", [(1, 3, 5), (4, 0, 2)])
def test_two_sink_full_dilution_reproduces_both_diagrams(t_fwd, t_src, t_bwd):
    """Noise on the two sink slices only, fully diluted one slice at a time
    (unit vectors on x'_4 for the first 12 V3 noise vectors, on x''_4 for the
    rest; w = 1); the solution of each is the exact propagator's column to its
    sink.  The forward result must equal the direct trace with the exact
    G2(y, x') for x' on x'_4 at every tau from x'_4 to r_4, the backward one
    with x'' on x''_4 from r_4 to x''_4 (second case wraps around T)."""
    L, T = (2, 2, 2), 6
    V3 = 8
    g = np.random.default_rng(41)
    n_fwd = (t_src - t_fwd) % T + 1
    n_bwd = (t_bwd - t_src) % T + 1
    taus = [(t_fwd + j) % T for j in range(n_fwd + n_bwd - 1)]
    G1f = syn.gaussian((12, 12, V3), g)
    G1b = syn.gaussian((12, 12, V3), g)
    G3 = {t: syn.gaussian((12, 12, V3), g) for t in taus}
    G2f = {t: syn.gaussian((V3, V3, 12, 12), g) for t in taus}   # exact G2(y on t, x' on x'_4)
    G2b = {t: syn.gaussian((V3, V3, 12, 12), g) for t in taus}   # exact G2(y on t, x'' on x''_4)
    M = 12 * V3
    eta_f = np.zeros((2 * M, 12, V3), dtype=np.complex128)
    eta_b = np.zeros((2 * M, 12, V3), dtype=np.complex128)
    for j in range(M):
        eta_f[j, j % 12, j // 12] = 1.0
        eta_b[M + j, j % 12, j // 12] = 1.0
    s = {t: np.einsum('yxAB,jBx->jAy', G2f[t], eta_f) + np.einsum('yxAB,jBx->jAy', G2b[t], eta_b) for t in taus}
    kp = oracle.momenta(1)
    q = oracle.momenta(1)
    pairs = [(2, 5), (0, 0)]
    res = oracle.two_sink_meson(G1f, eta_f, t_fwd, G1b, eta_b, t_bwd, t_src, G3, s, L, T, kp, w=np.ones(2 * M),
                                pairs=pairs)
    assert res["taus"] == taus and res["fwd"].shape[1] == n_fwd and res["bwd"].shape[1] == n_bwd
    for j, (p, qq) in enumerate(pairs):
        for it in range(n_fwd):
            t = taus[it]
            Cb = brute.meson_spin_open(G1f, G2f[t], G3[t], L, kp[p], kp[qq])
            assert np.allclose(res["fwd"][j, it, 0].reshape((4,) * 6), Cb, atol=1e-12 * np.abs(Cb).max())
        for it in range(n_bwd):
            t = taus[n_fwd - 1 + it]
            Cb = brute.meson_spin_open(G1b, G2b[t], G3[t], L, kp[p], kp[qq])
            assert np.allclose(res["bwd"][j, it, 0].reshape((4,) * 6), Cb, atol=1e-12 * np.abs(Cb).max())
