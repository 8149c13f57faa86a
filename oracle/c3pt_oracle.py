"""FP64 CPU oracle: factorized spin-open three-point function.

TEST INFRASTRUCTURE ONLY -- never called by the product path.

Follows Bali et al., "Baryonic and mesonic 3-point functions with open spin
indices" (Lattice 2017):

* the spectator part, Eq. (9), and the insertion part, Eq. (10), obtained from
  the factorization Eq. (8) of the trace Eq. (1) once one propagator is
  replaced by its stochastic estimate Eq. (5);
* the momentum projection of both parts with p = 2 pi k / L (Sec. 3), and the
  source offset of Sec. 2.1 (x -> x - r);
* the noise-weighted product of the two parts (the estimate of Eq. (5) inserted
  into Eq. (8)), with the source colour delta of Eq. (1) summed.

Readings where the paper is silent:

* gamma basis: DeGrand-Rossi, so gamma5 = diag(1, 1, -1, -1) and is real;
* memory orders: A = 3*spin + colour; propagator G[A_row][A_col][site] with the
  row at the field point and the column at the source; site n = x1 + L1(x2 + L2 x3);
* baryon spectator: epsilon-tensor colour contraction at sink and source with
  all five spins and the source colour of the active quark open; the active
  (stochastic) line carries gamma5 eta at the sink exactly as for the meson;
* derivative insertion: D_nu psi(y) = 1/2 [U_nu(y) psi(y+nu) - U_nu(y-nu)^dag psi(y-nu)]
  acting on the propagator G_f3, periodic boundaries in all directions;
* noise weights w_i, default 1/N (Eq. (5) carries 1/N, Eq. (8) drops it);
* two sinks: the noise lives on x'_4 and x''_4, the forward diagram takes the
  insertion timeslices from x'_4 to r_4, the backward one those from r_4 to
  x''_4 (both inclusive, forward in time modulo T);
* symmetrized derivative 1/2 (->D - <-D), the left derivative acting on the
  insertion's antiquark (D applied to s in the factorized form); two
  derivatives D_nu D_rho act on the quark field, D_rho first;
* Gamma channels: the creation operator carries gamma4 Gamma^dag gamma4
  (Eq. (3)); the proton is eps (u^T C gamma5 d) u with C = gamma2 gamma4,
  its conjugate chi^dag gamma4, connected Wick contractions, tr[P G];
* smearing: Wuppertal form, spatial, periodic, kappa and the step count free.

Everything is complex128.  Sums over sites are done as a phase-matrix product
(numpy matmul) over site chunks; colour sums as einsum.
"""
from __future__ import annotations

import itertools

import numpy as np

# --------------------------------------------------------------------------
# Gamma matrices (DeGrand-Rossi basis, the QDP++/Chroma convention).
# --------------------------------------------------------------------------
_i = 1j
GAMMA = [
    np.array([[0, 0, 0, _i], [0, 0, _i, 0], [0, -_i, 0, 0], [-_i, 0, 0, 0]], dtype=np.complex128),
    np.array([[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]], dtype=np.complex128),
    np.array([[0, 0, _i, 0], [0, 0, 0, -_i], [-_i, 0, 0, 0], [0, _i, 0, 0]], dtype=np.complex128),
    np.array([[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]], dtype=np.complex128),
]
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
GAMMA5_DIAG = np.real(np.diagonal(GAMMA5)).copy()


def gamma_basis16():
    """Gamma_n = g1^b0 g2^b1 g3^b2 g4^b3 for n = b0 + 2 b1 + 4 b2 + 8 b3."""
    out = []
    for n in range(16):
        m = np.eye(4, dtype=np.complex128)
        for mu in range(4):
            if (n >> mu) & 1:
                m = m @ GAMMA[mu]
        out.append(m)
    return out


# Levi-Civita tensor for the baryon colour contractions.
EPS = np.zeros((3, 3, 3))
for (_a, _b, _c), _s in (((0, 1, 2), 1), ((1, 2, 0), 1), ((2, 0, 1), 1),
                         ((0, 2, 1), -1), ((2, 1, 0), -1), ((1, 0, 2), -1)):
    EPS[_a, _b, _c] = _s


# --------------------------------------------------------------------------
# Momenta and phases (Eqs. (9)-(10), Sec. 3: p = 2 pi k / L, integer k).
# --------------------------------------------------------------------------
def momenta(n2max: int) -> np.ndarray:
    """All integer k with |k|^2 <= n2max, ordered by (|k|^2, k1, k2, k3)."""
    r = int(np.floor(np.sqrt(n2max)))
    ks = [k for k in itertools.product(range(-r, r + 1), repeat=3)
          if k[0] * k[0] + k[1] * k[1] + k[2] * k[2] <= n2max]
    ks.sort(key=lambda k: (k[0] * k[0] + k[1] * k[1] + k[2] * k[2], k[0], k[1], k[2]))
    return np.array(ks, dtype=np.int64).reshape(-1, 3)


def site_coords(L) -> np.ndarray:
    """[V3][3] coordinates (x1, x2, x3) of site n = x1 + L1 (x2 + L2 x3)."""
    L1, L2, L3 = (int(v) for v in L)
    n = np.arange(L1 * L2 * L3)
    return np.stack([n % L1, (n // L1) % L2, n // (L1 * L2)], axis=1)


def phase_matrix(L, k, r, sigma: int, sites=None) -> np.ndarray:
    """phi[m][x] = exp(sigma * 2 pi i * sum_j k_mj (x_j - r_j) / L_j).

    sigma = -1 for the spectator (Eq. (9)), +1 for the insertion (Eq. (10));
    r is the spatial source position (Sec. 2.1, x -> x - r)."""
    x = site_coords(L) if sites is None else site_coords(L)[sites]
    k = np.asarray(k, dtype=np.float64).reshape(-1, 3)
    Lf = np.asarray(L[:3], dtype=np.float64)
    d = (x - np.asarray(r[:3], dtype=np.float64)[None, :]) / Lf[None, :]
    arg = 2.0 * np.pi * (k @ d.T)
    return np.exp(1j * sigma * arg)


# --------------------------------------------------------------------------
# Spectator parts.
# --------------------------------------------------------------------------
def spectator_meson(G, eta, L, k, r=(0, 0, 0)) -> np.ndarray:
    """Meson spectator, Eq. (9).

    S_i(p')[b'][a'][a][c_src] = sum_x' phi^-_p'(x') sum_c [gamma5 eta_i(x')]^{b'}_c
                                  [gamma5 G(x',r)^dag gamma5]^{a' a}_{c c_src}

    where the daggered propagator element with sink spin a', sink colour c,
    source spin a and source colour c_src is g[a'] g[a] conj(G[(a',c)][(a,c_src)]).
    G: [12][12][V3] (slice at the sink time), eta: [N][12][V3].
    Returns [N][n_mom][192] in the order (b', a', a, c_src)."""
    G = np.asarray(G, dtype=np.complex128)
    eta = np.asarray(eta, dtype=np.complex128)
    N, V3 = eta.shape[0], eta.shape[-1]
    g = GAMMA5_DIAG
    Gr = G.reshape(4, 3, 4, 3, V3)                 # [a'][c][a][c_src][x]
    er = eta.reshape(N, 4, 3, V3) * g[None, :, None, None]   # gamma5 eta
    Gd = np.conj(Gr) * g[:, None, None, None, None] * g[None, None, :, None, None]
    out = np.zeros((N, 192, len(np.asarray(k).reshape(-1, 3))), dtype=np.complex128)
    chunk = 4096
    for s0 in range(0, V3, chunk):
        s1 = min(V3, s0 + chunk)
        P = np.einsum('ibcx,pcqax->ibpqax', er[..., s0:s1], Gd[..., s0:s1], optimize=True)
        ph = phase_matrix(L, k, r, -1, sites=np.arange(s0, s1))
        out += P.reshape(N, 192, s1 - s0) @ ph.T
    return np.ascontiguousarray(out.transpose(0, 2, 1))


def baryon_diquark(G1, G2) -> np.ndarray:
    """Q[a1'][a1][a2'][a2][c][c'][x] = sum eps_{abc} eps_{a'b'c'}
    G1[(a1',a)][(a1,a')] G2[(a2',b)][(a2,b')]   (colour indices a,b,a',b' summed)."""
    V3 = np.asarray(G1).shape[-1]
    return _diquark(np.asarray(G1, dtype=np.complex128).reshape(4, 3, 4, 3, V3),
                    np.asarray(G2, dtype=np.complex128).reshape(4, 3, 4, 3, V3))


def _diquark(G1r, G2r):
    # Written out with explicit epsilon sums (a,b | c) and (a',b' | c').
    V3 = G1r.shape[-1]
    Q = np.zeros((4, 4, 4, 4, 3, 3, V3), dtype=np.complex128)
    for a, b, c in itertools.permutations(range(3)):
        s1 = EPS[a, b, c]
        for a_, b_, c_ in itertools.permutations(range(3)):
            s2 = EPS[a_, b_, c_]
            # G1[a1'][a][a1][a'] * G2[a2'][b][a2][b']
            Q[:, :, :, :, c, c_, :] += (s1 * s2) * (
                G1r[:, a, :, a_, None, None, :] * G2r[None, None, :, b, :, b_, :])
    return Q


def spectator_baryon(G1, G2, eta, L, k, r=(0, 0, 0)) -> np.ndarray:
    """Nucleon-type spectator with epsilon-tensor colour contraction.

    The paper times a baryon measurement but prints no formula for it (Sec. 2
    shows only mesons).  Reading: two spectator quarks run forward from the
    source r to the sink x' (propagators G1, G2 with sink (spin, colour) rows and
    source (spin, colour) columns); the third, active quark leaves the sink on
    the stochastic line, which contributes [gamma5 eta_i(x')]^{b'}_c exactly as
    in the meson case.  Colours are contracted with eps at the sink and at the
    source; the source colour c' of the active quark stays open and meets the
    insertion part's source colour in the combine.

    S^B_i(p')[a1'][a1][a2'][a2][b'][c'] = sum_x' phi^-_p'(x') sum_{c} g[b'] eta_i(x')[(b',c)]
        sum_{a,b,a',b'} eps_{abc} eps_{a'b'c'} G1[(a1',a)][(a1,a')] G2[(a2',b)][(a2,b')]

    Returns [N][n_mom][3072] in the order (a1', a1, a2', a2, b', c')."""
    eta = np.asarray(eta, dtype=np.complex128)
    N, V3 = eta.shape[0], eta.shape[-1]
    g = GAMMA5_DIAG
    G1r = np.asarray(G1, dtype=np.complex128).reshape(4, 3, 4, 3, V3)
    G2r = np.asarray(G2, dtype=np.complex128).reshape(4, 3, 4, 3, V3)
    er = eta.reshape(N, 4, 3, V3) * g[None, :, None, None]
    n_mom = len(np.asarray(k).reshape(-1, 3))
    out = np.zeros((N, 3072, n_mom), dtype=np.complex128)
    chunk = 512
    for s0 in range(0, V3, chunk):
        s1 = min(V3, s0 + chunk)
        Q = _diquark(G1r[..., s0:s1], G2r[..., s0:s1])       # [a1'][a1][a2'][a2][c][c'][x]
        P = np.einsum('ibcx,pqrscfx->ipqrsbfx', er[..., s0:s1], Q, optimize=True)
        ph = phase_matrix(L, k, r, -1, sites=np.arange(s0, s1))
        out += P.reshape(N, 3072, s1 - s0) @ ph.T
    return np.ascontiguousarray(out.transpose(0, 2, 1))


# --------------------------------------------------------------------------
# Insertion part.
# --------------------------------------------------------------------------
def _neighbour(f, L, mu: int, sign: int):
    """f(x + sign * mu_hat) on one timeslice, periodic; f[..., V3], mu in 0..2."""
    L1, L2, L3 = (int(v) for v in L)
    arr = f.reshape(f.shape[:-1] + (L3, L2, L1))
    axis = {0: -1, 1: -2, 2: -3}[mu]
    return np.roll(arr, -sign, axis=axis).reshape(f.shape)


def covariant_derivative(G_t, U_t, L, T: int, tau: int, nu: int) -> np.ndarray:
    """(D_nu G)(y) = 1/2 [U_nu(y) G(y+nu) - U_nu(y-nu)^dag G(y-nu)] on slice tau.

    The insertion operator may contain local derivatives (Sec. 2.1); this is the
    standard symmetric lattice covariant derivative acting on the quark field
    psi_f2 (the propagator G_f3's sink side), with links U_nu(y) on the link
    y -> y + nu and periodic boundaries.  U_t: dict t -> [4][3][3][V3].
    Returns [12][12][V3]."""
    V3 = G_t[tau].shape[-1]
    if nu < 3:
        Gp = _neighbour(G_t[tau], L, nu, +1)
        Gm = _neighbour(G_t[tau], L, nu, -1)
        Uy = U_t[tau][nu]
        Um = _neighbour(U_t[tau][nu], L, nu, -1)
    else:
        Gp = G_t[(tau + 1) % T]
        Gm = G_t[(tau - 1) % T]
        Uy = U_t[tau][3]
        Um = U_t[(tau - 1) % T][3]
    Gp = np.asarray(Gp, dtype=np.complex128).reshape(4, 3, 12, V3)
    Gm = np.asarray(Gm, dtype=np.complex128).reshape(4, 3, 12, V3)
    fwd = np.einsum('cdx,sdqx->scqx', Uy, Gp)
    bwd = np.einsum('dcx,sdqx->scqx', np.conj(Um), Gm)
    return (0.5 * (fwd - bwd)).reshape(12, 12, V3)


def _insertion_local(G, s, L, k, r):
    """I_i(q)[at][bt][b][c_src] = sum_y phi^+_q(y) sum_c [gamma5 s_i(y)]*^{at}_c G(y,r)^{bt b}_{c c_src}.

    Eq. (10): the sink colour of G equals the colour of s (delta a~ b~), the
    source indices (b, c_src) stay open.  Returns [N][n_mom][192]."""
    s = np.asarray(s, dtype=np.complex128)
    N, V3 = s.shape[0], s.shape[-1]
    g = GAMMA5_DIAG
    sb = np.conj(s.reshape(N, 4, 3, V3)) * g[None, :, None, None]
    Gr = np.asarray(G, dtype=np.complex128).reshape(4, 3, 12, V3)
    n_mom = len(np.asarray(k).reshape(-1, 3))
    out = np.zeros((N, 192, n_mom), dtype=np.complex128)
    chunk = 4096
    for s0 in range(0, V3, chunk):
        s1 = min(V3, s0 + chunk)
        P = np.einsum('iacx,bcqx->iabqx', sb[..., s0:s1], Gr[..., s0:s1], optimize=True)
        ph = phase_matrix(L, k, r, +1, sites=np.arange(s0, s1))
        out += P.reshape(N, 192, s1 - s0) @ ph.T
    return np.ascontiguousarray(out.transpose(0, 2, 1))


def covariant_derivative_vector(v_t, U_t, L, T: int, tau: int, nu: int) -> np.ndarray:
    """(D_nu v)(y) = 1/2 [U_nu(y) v(y+nu) - U_nu(y-nu)^dag v(y-nu)] for the
    colour vectors v_t: t -> [N][12][V3] (spin and noise index untouched), the
    same lattice derivative as covariant_derivative.  Returns [N][12][V3]."""
    v = np.asarray(v_t[tau], dtype=np.complex128)
    N, V3 = v.shape[0], v.shape[-1]
    if nu < 3:
        vp = _neighbour(v_t[tau], L, nu, +1)
        vm = _neighbour(v_t[tau], L, nu, -1)
        Uy = U_t[tau][nu]
        Um = _neighbour(U_t[tau][nu], L, nu, -1)
    else:
        vp = v_t[(tau + 1) % T]
        vm = v_t[(tau - 1) % T]
        Uy = U_t[tau][3]
        Um = U_t[(tau - 1) % T][3]
    vp = np.asarray(vp, dtype=np.complex128).reshape(N, 4, 3, V3)
    vm = np.asarray(vm, dtype=np.complex128).reshape(N, 4, 3, V3)
    fwd = np.einsum('cdx,isdx->iscx', Uy, vp)
    bwd = np.einsum('dcx,isdx->iscx', np.conj(Um), vm)
    return (0.5 * (fwd - bwd)).reshape(N, 12, V3)


def insertion(G_t, s_t, taus, L, T: int, k, r=(0, 0, 0), U_t=None, n_ops: int = 1) -> np.ndarray:
    """Insertion part, Eq. (10), at every tau in ``taus``.

    G_t: mapping t -> [12][12][V3] propagator slice; s_t: t -> [N][12][V3];
    U_t: t -> [4][3][3][V3] (needed when n_ops > 1).
    Operators: op 0 is local (all 16 Gamma stay open in (at, bt)); ops 1..4 are
    the derivative D_nu for nu = x, y, z, t applied to G before the same
    contraction (gamma_mu D_nu follows by contracting (at, bt) with gamma_mu);
    with n_ops = 21, ops 5 + 4 rho + nu are the two-derivative operators
    D_nu D_rho (D_rho applied first; G needed on tau +- 2 for rho = nu = t);
    with n_ops = 37, ops 21 + 4 mu + nu are in addition the symmetrized
    <->D_mu <->D_nu (s needed on tau +- 2 as well);
    with n_ops = 9, ops 5..8 are the symmetrized derivative
    <->D_nu = 1/2 (->D_nu - <-D_nu).  The left derivative acts on the
    antiquark field of the insertion, whose factorized form is the conjugated
    gamma5 s (Eq. (10)); moving it there turns it into D_nu applied to s, so
    <-D_nu is the local contraction of G(y) with D_nu s (s needed on tau +- 1
    for nu = t).
    Returns [N][n_tau][n_ops][n_mom][192]."""
    assert n_ops in (1, 5, 9, 21, 37)
    taus = list(taus)
    N = np.asarray(s_t[taus[0]]).shape[0]
    n_mom = len(np.asarray(k).reshape(-1, 3))
    out = np.zeros((N, len(taus), n_ops, n_mom, 192), dtype=np.complex128)
    for j, tau in enumerate(taus):
        out[:, j, 0] = _insertion_local(G_t[tau], s_t[tau], L, k, r)
        if n_ops >= 5:
            for nu in range(4):
                DG = covariant_derivative(G_t, U_t, L, T, tau, nu)
                out[:, j, 1 + nu] = _insertion_local(DG, s_t[tau], L, k, r)
        if n_ops == 9:
            for nu in range(4):
                Ds = covariant_derivative_vector(s_t, U_t, L, T, tau, nu)
                left = _insertion_local(G_t[tau], Ds, L, k, r)
                out[:, j, 5 + nu] = 0.5 * (out[:, j, 1 + nu] - left)
        if n_ops >= 21:
            for rho in range(4):
                # D_rho G on tau and its two neighbouring slices, then D_nu of that field
                DG = {t % T: covariant_derivative(G_t, U_t, L, T, t % T, rho) for t in (tau - 1, tau, tau + 1)}
                for nu in range(4):
                    DDG = covariant_derivative(DG, U_t, L, T, tau, nu)
                    out[:, j, 5 + 4 * rho + nu] = _insertion_local(DDG, s_t[tau], L, k, r)
        if n_ops == 37:
            # <->D_mu <->D_nu = 1/4 (->D_mu ->D_nu - ->D_mu <-D_nu - <-D_mu ->D_nu + <-D_mu <-D_nu);
            # left derivatives act on the antiquark: D applied to s, <-D_mu first
            Ds = {mu: {t % T: covariant_derivative_vector(s_t, U_t, L, T, t % T, mu) for t in (tau - 1, tau, tau + 1)}
                  for mu in range(4)}
            DG = {nu: covariant_derivative(G_t, U_t, L, T, tau, nu) for nu in range(4)}
            for mu in range(4):
                for nu in range(4):
                    rr = out[:, j, 5 + 4 * nu + mu]                       # D_mu (D_nu G)
                    lr = _insertion_local(DG[nu], Ds[mu][tau], L, k, r)   # (psibar <-D_mu)(->D_nu psi)
                    rl = _insertion_local(DG[mu], Ds[nu][tau], L, k, r)   # (psibar <-D_nu)(->D_mu psi)
                    ll = _insertion_local(G_t[tau], covariant_derivative_vector(Ds[mu], U_t, L, T, tau, nu),
                                          L, k, r)
                    out[:, j, 21 + 4 * mu + nu] = 0.25 * (rr - lr - rl + ll)
    return out


# --------------------------------------------------------------------------
# Combine: noise-weighted product of the two parts.
# --------------------------------------------------------------------------
def all_pairs(n_p: int, n_q: int) -> np.ndarray:
    return np.array([(a, b) for a in range(n_p) for b in range(n_q)], dtype=np.int64).reshape(-1, 2)


def combine(S, I, w=None, pairs=None, op_begin: int = 0, op_end=None) -> np.ndarray:
    """C[pair][tau][op][s][t] = sum_i w_i sum_c S_i(p')[s][c] I_i(q, tau)[op][t][c].

    Eq. (5) inserted in Eq. (8): the noise average of spectator x insertion,
    with the source colour delta of Eq. (1) summed over c.  S: [N][n_p][spin*3]
    (spin = 64 meson, 1024 baryon; source colour last), I: [N][n_tau][n_ops][n_q][192].
    w defaults to 1/N.  pairs: [n_pairs][2] of (p' index, q index), default all.
    Returns [n_pairs][n_tau][op_end-op_begin][spin][64]."""
    S = np.asarray(S, dtype=np.complex128)
    I = np.asarray(I, dtype=np.complex128)
    N, n_p, sc = S.shape
    n_q = I.shape[3]
    n_ops = I.shape[2]
    op_end = n_ops if op_end is None else op_end
    if w is None:
        w = np.full(N, 1.0 / N)
    w = np.asarray(w, dtype=np.float64)
    if pairs is None:
        pairs = all_pairs(n_p, n_q)
    pairs = np.asarray(pairs).reshape(-1, 2)
    spin = sc // 3
    Sr = S.reshape(N, n_p, spin, 3) * w[:, None, None, None]
    Ir = I[:, :, op_begin:op_end].reshape(N, I.shape[1], op_end - op_begin, n_q, 64, 3)
    out = np.empty((len(pairs), I.shape[1], op_end - op_begin, spin, 64), dtype=np.complex128)
    for j, (p, q) in enumerate(pairs):
        out[j] = np.einsum('isc,ijouc->josu', Sr[:, p], Ir[:, :, :, q], optimize=True)
    return out


# --------------------------------------------------------------------------
# Forward and backward diagrams of one measurement (Sec. 2.3, Fig. 6).
# --------------------------------------------------------------------------
def two_sink_meson(G1_fwd, eta_fwd, t_fwd, G1_bwd, eta_bwd, t_bwd, t_src, G_t, s_t, L, T: int, k,
                   r=(0, 0, 0), U_t=None, n_ops: int = 1, w=None, pairs=None) -> dict:
    """The noise is time partitioned: zero except on the sink timeslices x'_4
    (t_fwd) and x''_4 (t_bwd) around the source timeslice r_4 (t_src), so one
    solution s per noise vector serves the forward diagram (sink x'_4,
    insertion between x'_4 and r_4) and the backward one (sink x''_4,
    insertion between r_4 and x''_4), estimated together.  Each diagram is a
    spectator at its sink (Eq. (9) with that sink's propagator and noise
    slice), the insertion (Eq. (10)) on its timeslices, and their noise
    average (Eq. (5) in Eq. (8)).  Timeslices run forward in time modulo T:
    forward t_fwd .. t_src, backward t_src .. t_bwd; the source timeslice is
    in both.  Returns spec [2][N][n_mom][192] (forward, backward), ins on the
    span t_fwd .. t_bwd, and fwd / bwd as combine() returns them."""
    n_fwd = (t_src - t_fwd) % T + 1
    n_bwd = (t_bwd - t_src) % T + 1
    taus = [(t_fwd + j) % T for j in range(n_fwd + n_bwd - 1)]
    S_f = spectator_meson(G1_fwd, eta_fwd, L, k, r=r)
    S_b = spectator_meson(G1_bwd, eta_bwd, L, k, r=r)
    I = insertion(G_t, s_t, taus, L, T, k, r=r, U_t=U_t, n_ops=n_ops)
    return {"spec": np.stack([S_f, S_b]), "ins": I, "taus": taus,
            "fwd": combine(S_f, I[:, :n_fwd], w=w, pairs=pairs),
            "bwd": combine(S_b, I[:, n_fwd - 1:], w=w, pairs=pairs)}


# --------------------------------------------------------------------------
# Analysis stage: Gamma channels of the spin-open data (Sec. 1 and Sec. 3:
# every source / sink Gamma and every Gamma_ins follow from one measurement).
# --------------------------------------------------------------------------
def creation_matrix(G) -> np.ndarray:
    """gamma4 G^dag gamma4: the matrix of the creation operator, Eq. (3)."""
    return GAMMA[3] @ np.conj(np.asarray(G, dtype=np.complex128)).T @ GAMMA[3]


def charge_conjugation() -> np.ndarray:
    """C = gamma2 gamma4, for which C gamma_mu C^-1 = -gamma_mu^T in this basis."""
    return GAMMA[1] @ GAMMA[3]


def _mats(m, default):
    if m is None:
        m = default
    return np.asarray(m, dtype=np.complex128).reshape(-1, 4, 4)


def gamma_project_meson(C, g_snk=None, g_ins=None, g_src=None) -> np.ndarray:
    """Eq. (1) with the spins of the combine output contracted:
    out[..., i, j, l] = sum Gsnk_i^{a' b'} Gins_j^{at bt} Gsrc_l^{b a} C[..., b', a', a, at, bt, b].

    C: [..., 64, 64], rows (b', a', a), columns (at, bt, b) as combine()
    returns them for the meson.  Defaults: Gsnk = Gins = the 16 Gamma_n of
    gamma_basis16(); Gsrc_l = gamma4 Gamma_l^dag gamma4 (the creation operator
    of Eq. (3) with Gamma = Gamma_l)."""
    C = np.asarray(C, dtype=np.complex128)
    g16 = gamma_basis16()
    Gs = _mats(g_snk, g16)
    Gi = _mats(g_ins, g16)
    Gc = _mats(g_src, [creation_matrix(g) for g in g16])
    T6 = C.reshape(C.shape[:-2] + (4,) * 6)
    return np.einsum('...BAaxyb,iAB,jxy,lba->...ijl', T6, Gs, Gi, Gc, optimize=True)


# Wick contractions of the proton three-point function with the spin-open
# nucleon data.  Proton chi_g = eps_abc (u_a^T A d_b) u_c^g, its conjugate
# chibar_d = chi^dag gamma4 = eps_abc ubar_c^d (dbar_b Abar ubar_a^T) with
# Abar = gamma4 A^dag gamma4; current J = qbar Gamma q; connected diagrams.
# The data C[a1'][a1][a2'][a2][b'][at][bt][b] carry the sink (a1', a2', b') and
# source (a1, a2, b) spins of the spectator lines G1, G2 and of the active line.
# A term is (sign, sink roles, source roles): the sink roles name the tensor
# spins of (u_a, d_b, u_c) -- the two diquark spins of A, then the nucleon
# spin -- and the source roles those of (dbar_b, ubar_a, ubar_c).
#   "d": spectators (G1, G2) = (u, u), the d quark active (two u pairings);
#   "u": spectators (G1, G2) = (u, d), a u quark active (four pairings).
PROTON_TERMS = {
    "d": [(+1, ("a1'", "b'", "a2'"), ("b", "a1", "a2")),
          (+1, ("a1'", "b'", "a2'"), ("b", "a2", "a1"))],
    "u": [(+1, ("b'", "a2'", "a1'"), ("a2", "b", "a1")),
          (+1, ("b'", "a2'", "a1'"), ("a2", "a1", "b")),
          (+1, ("a1'", "a2'", "b'"), ("a2", "b", "a1")),
          (+1, ("a1'", "a2'", "b'"), ("a2", "a1", "b"))],
}
_NUC_LABEL = {"a1'": 'A', "a1": 'B', "a2'": 'C', "a2": 'D', "b'": 'E', "b": 'H'}


def parity_projectors() -> np.ndarray:
    """(1 + gamma4)/2 and (1 - gamma4)/2."""
    one = np.eye(4, dtype=np.complex128)
    return np.stack([(one + GAMMA[3]) / 2, (one - GAMMA[3]) / 2])


def gamma_project_nucleon(C, channel: str, A=None, Abar=None, P=None, g_ins=None) -> np.ndarray:
    """out[..., p, j] = tr[P_p G_j] with G_j[g][d] = <chi_g(x') J_j(y) chibar_d(r)>,
    J_j = qbar Gamma_j q, summed over the Wick terms of PROTON_TERMS[channel]:
    sum_t sign_t sum A[s1][s2] Abar[r1][r2] P_p[d][g] Gins_j[at][bt] C[...].

    C: [..., 1024, 64] as combine() returns it for the nucleon.  Defaults:
    A = C gamma5, Abar = gamma4 A^dag gamma4, P = the two parity projectors,
    Gins = the 16 Gamma_n."""
    C = np.asarray(C, dtype=np.complex128)
    A = charge_conjugation() @ GAMMA5 if A is None else np.asarray(A, dtype=np.complex128)
    Abar = creation_matrix(A) if Abar is None else np.asarray(Abar, dtype=np.complex128)
    Ps = parity_projectors() if P is None else np.asarray(P, dtype=np.complex128).reshape(-1, 4, 4)
    Gi = _mats(g_ins, gamma_basis16())
    T8 = C.reshape(C.shape[:-2] + (4,) * 8)      # [a1'][a1][a2'][a2][b'][at][bt][b]
    out = np.zeros(C.shape[:-2] + (len(Ps), len(Gi)), dtype=np.complex128)
    for sign, snk, src in PROTON_TERMS[channel]:
        s1, s2, sn = (_NUC_LABEL[x] for x in snk)
        r1, r2, rn = (_NUC_LABEL[x] for x in src)
        expr = f'...ABCDEFGH,{s1}{s2},{r1}{r2},p{rn}{sn},jFG->...pj'
        out += sign * np.einsum(expr, T8, A, Abar, Ps, Gi, optimize=True)
    return out


# --------------------------------------------------------------------------
# Quark smearing of the inputs (Sec. 2.1: A and C may contain quark smearing;
# Sec. 3: the spectator's propagators are smeared at source and sink).
# --------------------------------------------------------------------------
def smear(field, U, L, kappa: float, n_iter: int, n_outer: int, n_inner: int) -> np.ndarray:
    """Gauge-covariant (Wuppertal-type) smearing of colour vectors on one timeslice,
    applied n_iter times:
        psi'(x) = [psi(x) + kappa sum_{j=1..3} (U_j(x) psi(x+j) + U_j(x-j)^dag psi(x-j))] / (1 + 6 kappa).
    The paper names smearing but gives no kernel or parameters; this is the
    usual choice.  field: n_outer * 3 * n_inner * V3 values laid out as
    [n_outer][3 colour][n_inner][V3] (a propagator slice [12][12][V3] smeared on
    its row index is n_outer = 4 spins, n_inner = 12 columns; noise or solution
    vectors [N][12][V3] are n_outer = 4 N, n_inner = 1).  U: [4][3][3][V3]."""
    V3 = int(np.prod(L))
    psi = np.asarray(field, dtype=np.complex128).reshape(n_outer, 3, n_inner, V3).copy()
    U = np.asarray(U, dtype=np.complex128)
    Um = [_neighbour(U[j], L, j, -1) for j in range(3)]
    norm = 1.0 / (1.0 + 6.0 * kappa)
    for _ in range(n_iter):
        hop = np.zeros_like(psi)
        for j in range(3):
            fwd = _neighbour(psi, L, j, +1)
            bwd = _neighbour(psi, L, j, -1)
            hop += np.einsum('cdx,odix->ocix', U[j], fwd)
            hop += np.einsum('dcx,odix->ocix', np.conj(Um[j]), bwd)
        psi = norm * (psi + kappa * hop)
    return psi.reshape(np.asarray(field).shape)
