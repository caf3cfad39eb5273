"""Slater-determinant algebra on bit strings (oracle, test infrastructure).

A determinant over 2N spin-orbitals is a Python int.  Spin-orbital index:
alpha orbital p -> p, beta orbital p -> N + p.  The phase convention is
|D> = a+_{s1} a+_{s2} ... a+_{sn} |vac> with s1 < s2 < ... < sn, i.e. the
alpha string first and then the beta string, each in ascending order.
"""
from __future__ import annotations


def _parity_below(det: int, p: int) -> int:
    return (det & ((1 << p) - 1)).bit_count() & 1


def annihilate(det: int, p: int):
    """a_p |det> -> (sign, det') or None."""
    if not (det >> p) & 1:
        return None
    s = -1 if _parity_below(det, p) else 1
    return s, det ^ (1 << p)


def create(det: int, p: int):
    """a+_p |det> -> (sign, det') or None."""
    if (det >> p) & 1:
        return None
    s = -1 if _parity_below(det, p) else 1
    return s, det | (1 << p)


def apply_string(det: int, ops):
    """Apply a product of operators, rightmost first.

    ``ops`` is a sequence of ('c'|'a', spin-orbital) read left to right as
    written in the operator product; the rightmost acts first.
    Returns (sign, det') or None.
    """
    sign = 1
    for kind, p in reversed(ops):
        r = create(det, p) if kind == 'c' else annihilate(det, p)
        if r is None:
            return None
        s, det = r
        sign *= s
    return sign, det


def occupied(det: int, nso: int):
    return [p for p in range(nso) if (det >> p) & 1]


def apply_one_body(vec: dict, h, n: int) -> dict:
    """sum_{pq,sigma} h[p,q] a+_{p sigma} a_{q sigma} applied to a vector {det: c}."""
    out: dict = {}
    for det, c in vec.items():
        for q in occupied(det, 2 * n):
            spin, qq = divmod(q, n)
            r1 = annihilate(det, q)
            s1, d1 = r1
            for pp in range(n):
                hv = h[pp, qq]
                if hv == 0.0:
                    continue
                r2 = create(d1, spin * n + pp)
                if r2 is None:
                    continue
                s2, d2 = r2
                out[d2] = out.get(d2, 0.0) + c * hv * s1 * s2
    return out


def apply_two_body(vec: dict, eri, n: int) -> dict:
    """(1/2) sum (pq|rs) a+_{p s} a+_{r t} a_{s' t} a_{q s} applied to {det: c}.

    ``eri[p, q, r, s]`` is the chemists'-notation integral (pq|rs).
    """
    out: dict = {}
    for det, c in vec.items():
        occ = occupied(det, 2 * n)
        for q in occ:
            sq, qq = divmod(q, n)
            s1, d1 = annihilate(det, q)
            for s in occ:
                if s == q:
                    continue
                ss, sp = divmod(s, n)
                s2, d2 = annihilate(d1, s)
                for rr in range(n):
                    r3 = create(d2, ss * n + rr)
                    if r3 is None:
                        continue
                    s3, d3 = r3
                    for pp in range(n):
                        v = eri[pp, qq, rr, sp]
                        if v == 0.0:
                            continue
                        r4 = create(d3, sq * n + pp)
                        if r4 is None:
                            continue
                        s4, d4 = r4
                        out[d4] = out.get(d4, 0.0) + 0.5 * c * v * s1 * s2 * s3 * s4
    return out
