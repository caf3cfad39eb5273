"""Algorithmic work of one sigma = (H0 - E0) x application (size arithmetic only).

Counted as 2 flops (one multiply-add) per Fock coupling through a free
index of a unique amplitude, over that index's range (a pinned-index box
transfer counts as one more element of the range).  S2 is counted over its
flip-unique amplitudes, (n_o^2 n_v^2 + n_o n_v)/2.  The O(dim) couplings of
the pinned TOP pair and the f_ov doubles <-> triples terms are not counted,
so the figure is a slight undercount.  The virtual-index part is the
N_o^2 N_v^3 work done by the Sylvester kernel; the occupied part is
N_o^3 N_v^2.
"""


def _c2(m):
    return m * (m - 1) // 2


def boxes(no, nv):
    """(unique amplitudes, virtual ranges, occupied ranges) per box."""
    return [
        (_c2(no) * _c2(nv), (nv, nv), (no, no)),                          # T2
        ((no * no * nv * nv + no * nv) // 2, (nv, nv), (no, no)),         # S2
        (_c2(no - 1) * _c2(nv - 1), (nv - 1, nv - 1), (no - 1, no - 1)),  # T3L
        (_c2(no) * _c2(nv), (nv, nv), (no, no)),                          # H1P1
        (_c2(no) * (nv - 1) ** 2, (nv, nv - 1), (no, no)),                # H1P2
        ((no - 1) ** 2 * _c2(nv), (nv, nv), (no, no - 1)),                # H2P1
        ((no - 1) ** 2 * (nv - 1) ** 2, (nv, nv - 1), (no, no - 1)),      # H2P2
    ]


def sigma_flops(no, nv):
    """(virtual-index flops, occupied-index flops) of one sigma application."""
    vv = sum(u * 2 * (v[0] + v[1]) for u, v, _ in boxes(no, nv))
    oo = sum(u * 2 * (o[0] + o[1]) for u, _, o in boxes(no, nv))
    return vv, oo


def amplitudes(no, nv):
    """Stored amplitudes (the library's layout)."""
    return (_c2(no) * _c2(nv) + no * no * nv * nv + _c2(no - 1) * _c2(nv - 1) + _c2(no) * _c2(nv)
            + _c2(no) * (nv - 1) ** 2 + (no - 1) ** 2 * _c2(nv) + (no - 1) ** 2 * (nv - 1) ** 2)
