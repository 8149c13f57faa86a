"""Direct evaluation of the three-point trace on tiny lattices.

TEST INFRASTRUCTURE ONLY.

This is the second, independent form of the oracle.  It never forms the
spectator or insertion parts: it builds the three propagators of the trace of
Eq. (1) as 12x12 matrices per site pair and multiplies them out.

* G_f1(r, x') and G_f2(x', y) are obtained from the forward propagators by
  gamma5-hermiticity, G(a, b) = Gamma5 G(b, a)^dag Gamma5 with
  Gamma5 = gamma5 (x) 1_colour, written as plain matrix algebra;
* G_f2(y, x') is either an exact all-to-all propagator or its stochastic
  estimate sum_i w_i s_i(y) eta_i(x')^dag (Eq. (5));
* the derivative insertion replaces G_f3(y, r) by (D_nu G_f3)(y, r) built from
  kron(1_spin, U) matrices.

Cost is O(V3^2) per momentum pair, so only L <= 4 is practical.
"""
from __future__ import annotations

import itertools

import numpy as np

from .c3pt_oracle import GAMMA5, EPS, site_coords

_G5 = np.kron(GAMMA5, np.eye(3))   # Gamma5 on (spin, colour), A = 3*spin + colour


def site_matrices(G) -> np.ndarray:
    """[12][12][V3] -> [V3][12][12]."""
    return np.ascontiguousarray(np.moveaxis(np.asarray(G, dtype=np.complex128), -1, 0))


def g5_dagger(M) -> np.ndarray:
    """Gamma5 M^dag Gamma5 for a stack [..., 12, 12]."""
    return _G5 @ np.conj(np.swapaxes(M, -1, -2)) @ _G5


def stochastic_all_to_all(s, eta, w) -> np.ndarray:
    """Ghat(y, x') = sum_i w_i s_i(y) eta_i(x')^dag  as [V3_y][V3_x'][12][12]  (Eq. (5))."""
    s = np.asarray(s, dtype=np.complex128)
    eta = np.asarray(eta, dtype=np.complex128)
    return np.einsum('i,iAy,iBx->yxAB', np.asarray(w, dtype=np.float64), s, np.conj(eta))


def phase(L, k, r, sigma):
    x = site_coords(L)
    d = (x - np.asarray(r[:3])[None, :]) / np.asarray(L[:3], dtype=np.float64)[None, :]
    return np.exp(1j * sigma * 2.0 * np.pi * (d @ np.asarray(k, dtype=np.float64)))


def meson_spin_open(G1_tf, G2_yx, G3_tau, L, kp, q, r=(0, 0, 0)) -> np.ndarray:
    """C[b'][a'][a][at][bt][b] = sum_{x',y} e^{-ip'(x'-r)} e^{iq(y-r)}
         sum_{a,a',at} G1(r,x')[(a,c),(a',c')] G2(x',y)[(b',c'),(at,ct)] G3(y,r)[(bt,ct),(b,c)].

    G1_tf: forward propagator slice at the sink, G1(x', r); G2_yx: forward
    all-to-all G2(y, x') as [V3_y][V3_x'][12][12]; G3_tau: forward slice G3(y, r)."""
    M1 = g5_dagger(site_matrices(G1_tf))              # G1(r, x')  [x'][12][12]
    M2 = g5_dagger(np.swapaxes(G2_yx, 0, 1))          # G2(x', y)  [x'][y][12][12]
    M3 = site_matrices(G3_tau)                        # G3(y, r)   [y][12][12]
    fx = phase(L, kp, r, -1)
    fy = phase(L, q, r, +1)
    M1r = M1.reshape(-1, 4, 3, 4, 3)                  # [x'][a][c][a'][c']
    M2r = M2.reshape(M2.shape[0], M2.shape[1], 4, 3, 4, 3)   # [x'][y][b'][c'][at][ct]
    M3r = M3.reshape(-1, 4, 3, 4, 3)                  # [y][bt][ct][b][c]
    A = np.einsum('x,xacpd->xacpd', fx, M1r)
    B = np.einsum('y,ytesf->ytesf', fy, M3r)
    # a: source spin, c: source colour, p/d: sink spin/colour of G1, q: b',
    # u/e: insertion spin/colour on the active line, t/s: bt, b.
    return np.einsum('xacpd,xyqdue,ytesc->qpauts', A, M2r, B, optimize=True)


def meson_trace(G1_tf, G2_yx, G3_tau, L, kp, q, g_snk, g_ins, g_src, r=(0, 0, 0)) -> complex:
    """sum_{x',y} phases * tr[G1(r,x') Gsnk G2(x',y) Gins G3(y,r) Gsrc]   (Eq. (1)),
    with 12x12 matrix products; Gamma acts as Gamma (x) 1_colour."""
    M1 = g5_dagger(site_matrices(G1_tf))
    M2 = g5_dagger(np.swapaxes(G2_yx, 0, 1))
    M3 = site_matrices(G3_tau)
    Gs, Gi, Gc = (np.kron(np.asarray(m), np.eye(3)) for m in (g_snk, g_ins, g_src))
    fx = phase(L, kp, r, -1)
    fy = phase(L, q, r, +1)
    tot = 0j
    for x in range(M1.shape[0]):
        left = M1[x] @ Gs
        for y in range(M3.shape[0]):
            tot += fx[x] * fy[y] * np.trace(left @ M2[x, y] @ Gi @ M3[y] @ Gc)
    return tot


def derivative_field(G_t, U_t, L, T, tau, nu) -> np.ndarray:
    """(D_nu G)(y) = 1/2 [U_nu(y) G(y+nu) - U_nu(y-nu)^dag G(y-nu)] as [V3][12][M]
    for G_t: t -> [12][M][V3] (row index at y), using explicit neighbour lookup
    and kron(1_spin, U) matrices."""
    L1, L2, L3 = (int(v) for v in L)
    x = site_coords(L)
    V3 = x.shape[0]
    out = np.zeros((V3, 12, np.asarray(G_t[tau]).shape[1]), dtype=np.complex128)

    def idx(c):
        return int(c[0] % L1 + L1 * ((c[1] % L2) + L2 * (c[2] % L3)))

    for n in range(V3):
        e = np.zeros(3, dtype=int)
        if nu < 3:
            e[nu] = 1
            np_, nm = idx(x[n] + e), idx(x[n] - e)
            Gp = np.asarray(G_t[tau])[:, :, np_]
            Gm = np.asarray(G_t[tau])[:, :, nm]
            Uy = np.asarray(U_t[tau])[nu][:, :, n]
            Um = np.asarray(U_t[tau])[nu][:, :, nm]
        else:
            Gp = np.asarray(G_t[(tau + 1) % T])[:, :, n]
            Gm = np.asarray(G_t[(tau - 1) % T])[:, :, n]
            Uy = np.asarray(U_t[tau])[3][:, :, n]
            Um = np.asarray(U_t[(tau - 1) % T])[3][:, :, n]
        KU = np.kron(np.eye(4), Uy)
        KUm = np.kron(np.eye(4), Um)
        out[n] = 0.5 * (KU @ Gp - np.conj(KUm).T @ Gm)
    return out


def baryon_spin_open(G1_tf, G2_tf, Gact_yx, G3_tau, L, kp, q, r=(0, 0, 0)) -> np.ndarray:
    """Nucleon-type three-point function with open spins, evaluated directly.

    C[a1'][a1][a2'][a2][b'][at][bt][b] = sum_{x',y} e^{-ip'(x'-r)} e^{iq(y-r)}
       eps_{abc} eps_{a'b'c'} G1(x',r)[(a1',a),(a1,a')] G2(x',r)[(a2',b),(a2,b')]
       Gact(x',y)[(b',c),(at,ct)] G3(y,r)[(bt,ct),(b,c')]

    where Gact(x', y) = Gamma5 Gact(y, x')^dag Gamma5 is the active quark's
    propagator from the insertion to the sink, and Gact_yx is the forward
    G(y, x') as [V3_y][V3_x'][12][12]."""
    M1 = site_matrices(G1_tf).reshape(-1, 4, 3, 4, 3)   # [x'][a1'][a][a1][a']
    M2 = site_matrices(G2_tf).reshape(-1, 4, 3, 4, 3)   # [x'][a2'][b][a2][b']
    Ma = g5_dagger(np.swapaxes(Gact_yx, 0, 1)).reshape(M1.shape[0], -1, 4, 3, 4, 3)
    M3 = site_matrices(G3_tau).reshape(-1, 4, 3, 4, 3)  # [y][bt][ct][b][c']
    fx = phase(L, kp, r, -1)
    fy = phase(L, q, r, +1)
    tot = np.zeros((4, 4, 4, 4, 4, 4, 4, 4), dtype=np.complex128)
    for (a, b, c) in itertools.permutations(range(3)):
        for (a_, b_, c_) in itertools.permutations(range(3)):
            s = EPS[a, b, c] * EPS[a_, b_, c_]
            # sink side for fixed colours: [x'][a1'][a1][a2'][a2]
            D = np.einsum('x,xpq,xrs->xpqrs', fx, M1[:, :, a, :, a_], M2[:, :, b, :, b_])
            # active line and insertion: [x'][b'][at][bt][b]
            E = np.einsum('xyuve,y,ykej->xuvkj', Ma[:, :, :, c, :, :], fy,
                          M3[:, :, :, :, c_], optimize=True)
            tot += s * np.einsum('xpqrs,xuvkj->pqrsuvkj', D, E, optimize=True)
    return tot
