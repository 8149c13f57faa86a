"""Brute-force Wick contraction of products of quark fields (test pin).

An independent route to correlators of hadron operators: the fields of the
product are written out one by one, every complete pairing of each quark
field with an antiquark field of the same flavour is enumerated, each pairing
gets the sign of the permutation that brings its pairs next to each other
(Grassmann fields), and the propagators of its pairs are contracted with the
c-number coefficients of the operators by einsum.

    <q(x)_{s c} qbar(y)_{s' c'}> = S[flavour, x, y][s, c, s', c']

No factorization, no spin-open tensor and no role table is involved.
"""
from __future__ import annotations

import itertools

import numpy as np


class Field:
    def __init__(self, bar: bool, flavour: str, point, spin: str, colour: str, group: str):
        self.bar, self.flavour, self.point = bar, flavour, point
        self.spin, self.colour, self.group = spin, colour, group


def _parity(seq) -> int:
    inv = sum(1 for i in range(len(seq)) for j in range(i + 1, len(seq)) if seq[i] > seq[j])
    return -1 if inv % 2 else 1


def expectation(fields, coeffs, props, free, skip_same_group=("J",)):
    """<prod fields> with coefficients.

    fields: list of Field in operator order.
    coeffs: list of (array, labels) c-number tensors; labels are index names.
    props: dict (flavour, point_q, point_qbar) -> array [4, 3, 4, 3].
    free: output index names, in order.
    Pairings that join a quark and an antiquark of one group in
    skip_same_group (a current's own loop) are left out: connected diagrams."""
    names = {}

    def lab(n):
        return names.setdefault(n, len(names))

    qs = [i for i, f in enumerate(fields) if not f.bar]
    qbs = [i for i, f in enumerate(fields) if f.bar]
    total = None
    for perm in itertools.permutations(qbs):
        pairs = list(zip(qs, perm))
        if any(fields[a].flavour != fields[b].flavour for a, b in pairs):
            continue
        if any(fields[a].group == fields[b].group and fields[a].group in skip_same_group for a, b in pairs):
            continue
        order = [i for pr in pairs for i in pr]
        sign = _parity(order)
        ops = []
        for arr, labels in coeffs:
            ops += [arr, [lab(x) for x in labels]]
        for a, b in pairs:
            fa, fb = fields[a], fields[b]
            S = props[(fa.flavour, fa.point, fb.point)]
            ops += [S, [lab(fa.spin), lab(fa.colour), lab(fb.spin), lab(fb.colour)]]
        val = sign * np.einsum(*ops, [lab(x) for x in free], optimize='greedy')
        total = val if total is None else total + val
    return total


def proton(point, spins, colours, group, conj=False):
    """Fields of chi = eps_abc u_a^s1 A_{s1 s2} d_b^s2 u_c^s3 (conj=False, order
    u_a d_b u_c) or of chibar = eps_abc ubar_c^s3 dbar_b^s2 Abar_{s2 s1} ubar_a^s1
    (conj=True, order ubar_c dbar_b ubar_a).  spins = (s1, s2, s3) names the
    spins of (u_a, d_b, u_c) or (ubar_a, dbar_b, ubar_c); colours = (a, b, c)."""
    (s1, s2, s3), (a, b, c) = spins, colours
    if not conj:
        return [Field(False, "u", point, s1, a, group), Field(False, "d", point, s2, b, group),
                Field(False, "u", point, s3, c, group)]
    return [Field(True, "u", point, s3, c, group), Field(True, "d", point, s2, b, group),
            Field(True, "u", point, s1, a, group)]


def current(point, flavour, spins, colour, group="J"):
    """qbar^s1 Gamma_{s1 s2} q^s2 with one colour index (summed)."""
    s1, s2 = spins
    return [Field(True, flavour, point, s1, colour, group), Field(False, flavour, point, s2, colour, group)]


def barred_conjugate(fields, coeffs, free_spin, bar_spin, gamma4):
    """Fields and coefficients of Obar = O^dag gamma4 for an operator
    O_{free_spin} = coeffs * prod(fields), built field by field from
    qbar = q^dag gamma4 alone:

    * the product is reversed and every coefficient is complex conjugated
      ((AB)^dag = B^dag A^dag);
    * a quark field q_s becomes q^dag_s = sum_t qbar_t (gamma4^-1)_{t s};
    * an antiquark field qbar_s becomes (qbar_s)^dag = sum_t conj(gamma4)_{t s} q_t;
    * the free spin is barred: Obar_{bar_spin} = sum_g (O_g)^dag gamma4_{g, bar_spin}
      (free_spin None: a scalar operator, whose conjugate O^dag is returned).

    No matrix of the hadron operators (A, Gamma) is transformed as a whole:
    whatever the correct creation matrix is follows from the contraction."""
    inv4 = np.linalg.inv(gamma4)
    out_f = []
    out_c = [(np.conj(arr), labels) for arr, labels in coeffs]
    for f in reversed(fields):
        t = f.spin + "~"
        out_f.append(Field(not f.bar, f.flavour, f.point, t, f.colour, f.group))
        out_c.append((np.conj(gamma4) if f.bar else inv4, (t, f.spin)))
    if free_spin is not None:
        out_c.append((gamma4, (free_spin, bar_spin)))
    return out_f, out_c


def bilinear(point, flavour_bar, flavour, spins, colour, group):
    """qbar_{flavour_bar}^s1 M_{s1 s2} q_{flavour}^s2 (one colour, summed): the fields."""
    s1, s2 = spins
    return [Field(True, flavour_bar, point, s1, colour, group), Field(False, flavour, point, s2, colour, group)]
