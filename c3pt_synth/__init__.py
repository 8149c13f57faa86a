"""Seeded synthetic inputs for the spin-open three-point contractions.

This module holds random draws and array plumbing only: none of the method's
arithmetic (no contraction, no phase, no projection, no combine).  Both the
CPU oracle and the GPU path take their inputs from here, so the two sides see
identical numbers.

Shapes and memory orders (complex arrays, site index last):

* propagator slice  G[A_row][A_col][site],  A = 3*spin + colour, 12x12 per site;
  the row belongs to the field point, the column to the source point;
* noise / stochastic solution  v[noise][A][site];
* gauge links  U[mu][c][d][site], mu = 0..3 for x, y, z, t;
* site n = x1 + L1*(x2 + L2*x3), time is the slice index.

Distributions (the paper fixes only the noise moments of its noise equations,
zero mean and unit covariance; the rest are stated choices):

* propagators and stochastic solutions: i.i.d. unit complex Gaussians,
  re, im ~ N(0, 1/2), so E|z|^2 = 1;
* noise: Z2 x Z2, each component (+-1 +- i)/sqrt(2) with independent fair signs;
* links: Haar SU(3) from the QR decomposition of a complex Gaussian matrix with
  the diagonal of R made real positive (Mezzadri 2007), then divided by the
  cube root of its determinant.

Seeds: numpy PCG64 from SeedSequence([1711, 2384, cfg, field_id, index]).
"""
from __future__ import annotations

import numpy as np

FIELD_G3 = 1   # propagator used on the insertion side (also "u" for the nucleon)
FIELD_G1 = 2   # propagator used on the spectator side (also "d" for the nucleon)
FIELD_ETA = 3
FIELD_S = 4
FIELD_U = 5

NC = 3
NS = 4
NSC = 12


def rng(cfg: int, field_id: int, index: int) -> np.random.Generator:
    ss = np.random.SeedSequence([1711, 2384, int(cfg), int(field_id), int(index) & 0xFFFFFFFF])
    return np.random.Generator(np.random.PCG64(ss))


def volume(L) -> int:
    return int(L[0]) * int(L[1]) * int(L[2])


def gaussian(shape, g: np.random.Generator, dtype=np.complex128) -> np.ndarray:
    """i.i.d. complex Gaussian with E|z|^2 = 1, drawn as interleaved (re, im)."""
    x = g.standard_normal(tuple(shape) + (2,), dtype=np.float64)
    x *= np.sqrt(0.5)
    z = x.view(np.complex128)[..., 0]
    return z.astype(dtype, copy=False)


def propagator_slice(L, cfg: int, field_id: int, t: int, dtype=np.complex128) -> np.ndarray:
    """One timeslice of a point-to-all propagator, [12][12][V3]."""
    return gaussian((NSC, NSC, volume(L)), rng(cfg, field_id, t), dtype)


def solution_slice(L, n_noise: int, cfg: int, t: int, dtype=np.complex128) -> np.ndarray:
    """Stochastic solutions s_i on one timeslice, [N][12][V3]."""
    return gaussian((n_noise, NSC, volume(L)), rng(cfg, FIELD_S, t), dtype)


def z2z2_noise(L, n_noise: int, cfg: int, t: int, dtype=np.complex128) -> np.ndarray:
    """Z2 x Z2 noise vectors on one timeslice, [N][12][V3]."""
    g = rng(cfg, FIELD_ETA, t)
    bits = g.integers(0, 2, size=(n_noise, NSC, volume(L), 2), dtype=np.int8)
    sgn = 1.0 - 2.0 * bits.astype(np.float64)
    z = (sgn[..., 0] + 1j * sgn[..., 1]) / np.sqrt(2.0)
    return z.astype(dtype, copy=False)


def haar_su3(n: int, g: np.random.Generator) -> np.ndarray:
    """n Haar-distributed SU(3) matrices, [n][3][3]."""
    z = gaussian((n, NC, NC), g)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    q = q / (det ** (1.0 / 3.0))[:, None, None]
    return q


def link_slice(L, cfg: int, t: int, dtype=np.complex128) -> np.ndarray:
    """Gauge links U_mu(x) for mu = x, y, z, t on one timeslice, [4][3][3][V3]."""
    V3 = volume(L)
    u = haar_su3(4 * V3, rng(cfg, FIELD_U, t)).reshape(4, V3, NC, NC)
    return np.ascontiguousarray(u.transpose(0, 2, 3, 1)).astype(dtype, copy=False)


def unit_links(L, dtype=np.complex128) -> np.ndarray:
    V3 = volume(L)
    u = np.zeros((4, NC, NC, V3), dtype=dtype)
    for c in range(NC):
        u[:, c, c, :] = 1.0
    return u


def round_to_c64(a: np.ndarray) -> np.ndarray:
    """Values as a complex64 device buffer holds them, promoted back to complex128.

    Reduced-precision runs feed the oracle these rounded values, so that the
    measured error is that of the computation, not of the input cast."""
    return a.astype(np.complex64).astype(np.complex128)


def random_source(L, T, cfg: int, index: int):
    """Seeded source position (r1, r2, r3, r4)."""
    g = rng(cfg, 99, index)
    return [int(g.integers(0, L[0])), int(g.integers(0, L[1])), int(g.integers(0, L[2])),
            int(g.integers(0, T))]
