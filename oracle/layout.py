"""The seven-box amplitude layout, mapped to determinants (oracle side).

Test infrastructure.  The HIP library exposes its amplitude vectors in this
layout (it is the interface both sides agree on); this module is the
oracle's own implementation of it.  It defines each stored amplitude as an
excitation-operator string acting on the closed shell, in the spin-orbital
notation of the paper's first-order wave function (same-spin T and
mixed-spin S amplitudes).  TOP t is occupied orbital 0 (largest singular
value) and its partner t' is virtual 0.

  box  name   stored index                       operator string (acting on |Phi>)
  0    T2     (i<j), (a<b)                         a+_{a u} a+_{b u} a_{j u} a_{i u}
  1    S2     i, j, a, b                           a+_{a u} a+_{b d} a_{j d} a_{i u}
  2    T3L    (j<k) in 1.., (b<c) in 1..           a+_{t' u} a+_{b u} a+_{c u} a_{k u} a_{j u} a_{t u}
  3    H1P1   (j<k), (b<c)                         a+_{t' u} a+_{b d} a+_{c d} a_{k d} a_{j d} a_{t u}
  4    H1P2   (j<k), a in 1.., c in 1..            a+_{a u} a+_{t' d} a+_{c d} a_{k d} a_{j d} a_{t u}
  5    H2P1   i in 1.., k in 1.., (b<c)            a+_{t' u} a+_{b d} a+_{c d} a_{k d} a_{t d} a_{i u}
  6    H2P2   i in 1.., k in 1.., a in 1.., c in 1..   a+_{a u} a+_{t' d} a+_{c d} a_{k d} a_{t d} a_{i u}

(u = spin up, d = spin down; pairs "(p<q)" are stored packed, row-major over
the strict upper triangle; all other index groups are dense row-major; the
occupied pair is the outer index, the virtual pair the inner one.)

Every box except S2 stands for a spin-flip pair of determinants with equal
amplitudes (singlet): weight w = 2.  S2 stores every up-down determinant
separately (w = 1); the vector it represents is the flip-symmetrised one,
Psi = sum_S2 x_mu (|mu> + |flip mu>)/2 + sum_others x_nu (|nu> + |flip nu>),
so that every stored vector maps to a singlet-symmetric wave function.
"""
from __future__ import annotations

from itertools import combinations

import numpy as np

from . import fermion as fm

BOX_NAMES = ("T2", "S2", "T3L", "H1P1", "H1P2", "H2P1", "H2P2")
WEIGHTS = (2.0, 1.0, 2.0, 2.0, 2.0, 2.0, 2.0)


def pairs(lo, hi):
    return list(combinations(range(lo, hi), 2))


def box_sizes(no, nv):
    c2 = lambda m: m * (m - 1) // 2
    return [c2(no) * c2(nv), no * no * nv * nv, c2(no - 1) * c2(nv - 1),
            c2(no) * c2(nv), c2(no) * (nv - 1) ** 2,
            (no - 1) ** 2 * c2(nv), (no - 1) ** 2 * (nv - 1) ** 2]


def box_offsets(no, nv):
    s = box_sizes(no, nv)
    return list(np.concatenate([[0], np.cumsum(s)]).astype(np.int64))


def enumerate_ops(no, nv):
    """Yield (box, ops) in layout order.  ops: list of (kind, spin, orbital)
    with orbital in the full index space (virtual a -> no + a)."""
    V = lambda a: no + a
    t, tp = 0, 0
    for (i, j) in pairs(0, no):
        for (a, b) in pairs(0, nv):
            yield 0, [("c", 0, V(a)), ("c", 0, V(b)), ("a", 0, j), ("a", 0, i)]
    for i in range(no):
        for j in range(no):
            for a in range(nv):
                for b in range(nv):
                    yield 1, [("c", 0, V(a)), ("c", 1, V(b)), ("a", 1, j), ("a", 0, i)]
    for (j, k) in pairs(1, no):
        for (b, c) in pairs(1, nv):
            yield 2, [("c", 0, V(tp)), ("c", 0, V(b)), ("c", 0, V(c)),
                      ("a", 0, k), ("a", 0, j), ("a", 0, t)]
    for (j, k) in pairs(0, no):
        for (b, c) in pairs(0, nv):
            yield 3, [("c", 0, V(tp)), ("c", 1, V(b)), ("c", 1, V(c)),
                      ("a", 1, k), ("a", 1, j), ("a", 0, t)]
    for (j, k) in pairs(0, no):
        for a in range(1, nv):
            for c in range(1, nv):
                yield 4, [("c", 0, V(a)), ("c", 1, V(tp)), ("c", 1, V(c)),
                          ("a", 1, k), ("a", 1, j), ("a", 0, t)]
    for i in range(1, no):
        for k in range(1, no):
            for (b, c) in pairs(0, nv):
                yield 5, [("c", 0, V(tp)), ("c", 1, V(b)), ("c", 1, V(c)),
                          ("a", 1, k), ("a", 1, t), ("a", 0, i)]
    for i in range(1, no):
        for k in range(1, no):
            for a in range(1, nv):
                for c in range(1, nv):
                    yield 6, [("c", 0, V(a)), ("c", 1, V(tp)), ("c", 1, V(c)),
                              ("a", 1, k), ("a", 1, t), ("a", 0, i)]


def _det_of(ops, phi, n, flip=False):
    so = [(k, ((1 - s) if flip else s) * n + p) for (k, s, p) in ops]
    return fm.apply_string(phi, so)


def rep_map(no, nv, spin=0):
    """For every stored amplitude: list of (det, sign * factor) it contributes
    to the wave function, and (det, sign) of its own (unflipped) determinant.
    spin = 0: the spin-flip partner carries the same amplitude (singlet);
    spin = 1: the opposite one (the M_s = 0 triplet, antisymmetric under the
    flip of every spin)."""
    n = no + nv
    phi = sum(1 << p for p in range(no)) | sum(1 << (n + p) for p in range(no))
    fs = -1.0 if spin else 1.0
    out = []
    for box, ops in enumerate_ops(no, nv):
        s0, d0 = _det_of(ops, phi, n)
        s1, d1 = _det_of(ops, phi, n, flip=True)
        if box == 1:
            contrib = [(d0, 0.5 * s0), (d1, 0.5 * fs * s1)]
        else:
            contrib = [(d0, float(s0)), (d1, fs * float(s1))]
        out.append((box, contrib, (d0, s0)))
    return out


def weights(no, nv):
    s = box_sizes(no, nv)
    return np.concatenate([np.full(m, w) for m, w in zip(s, WEIGHTS)])
