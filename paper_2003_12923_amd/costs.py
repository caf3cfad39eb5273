"""Algorithmic work of one sigma = (H0 - E0) x application (size arithmetic only).

The algorithmic flop count is 2 x nnz of (H0 - E0) restricted to doubles +
L-triples, in the representative basis the amplitude vectors use (one row
per stored amplitude: a spin-flip pair of determinants per row, the two
members of an S2 flip pair (i, j, a, b) ~ (j, i, b, a) in one row): every
structural Fock coupling is one multiply-add.  Padding, Pauli zeros,
antisymmetric duplicates and the redundant half of S2 do not count.

The nonzeros fall into four classes by the one spin-orbital replacement
that links the two determinants (the index kinds a contraction runs over,
paper Sec. III.B, Table I):

  vir   a particle replaced by another virtual: the virtual-index Fock
        contractions (the N_o^2 N_v^3 terms; the Sylvester products);
  occ   a hole replaced by another occupied orbital (N_o^3 N_v^2);
  ov    a change of excitation level through f_ov, doubles <-> L-triples
        (N_o^2 N_v^2);
  diag  the diagonal.

Per box, for a representative row (t = occupied 0, t' = virtual 0; a
replacement that removes the pinned t or t' leaves the L-triples unless the
other spin of the same spatial orbital is still there, which makes it a box
transfer):

  T2    2 (V-2) particle and 2 (O-2) hole replacements;
  S2    summed over the flip-unique rows: O^2 V^2 (V-1) and O^2 V^2 (O-1);
  T3L   2 (V-3) and 2 (O-3) (removing t or t' leaves L);
  H1P1  2 (V-2) + (V-1) [b = t': t'up -> any] and 2 (O-2) + (O-1) [j = t];
  H1P2  (V-1) + (V-2) and 2 (O-2) + (O-1) [j = t];
  H2P1  2 (V-2) + (V-1) [b = t'] and (O-1) + (O-2);
  H2P2  (V-1) + (V-2) and (O-1) + (O-2);
  f_ov  9 doubles per T3L row, 5 per mixed-spin row, counted both ways.

Every closed form here is checked against an enumeration of the explicit
operator (oracle, test infrastructure) at several sizes.
"""


def _c2(m):
    return m * (m - 1) // 2


def sigma_nnz(no, nv):
    """Nonzeros of (H0 - E0) on doubles + L-triples in the representative basis,
    by class: dict with keys diag, vir, occ, ov, total."""
    O, V = no, nv
    po, pv, po1, pv1 = _c2(O), _c2(V), _c2(O - 1), _c2(V - 1)
    o1, v1 = O - 1, V - 1
    rows = po * pv + (O * O * V * V + O * V) // 2 + po1 * pv1 + po * pv + po * v1 * v1 + o1 * o1 * pv \
        + o1 * o1 * v1 * v1
    vir = (po * pv * 2 * (V - 2)                                 # T2
           + O * O * V * V * (V - 1)                             # S2
           + po1 * pv1 * 2 * (V - 3)                             # T3L
           + po * pv * 2 * (V - 2) + po * v1 * v1                # H1P1 (+ t' up -> any, b = t')
           + po * v1 * v1 * (2 * V - 3)                          # H1P2
           + o1 * o1 * pv * 2 * (V - 2) + o1 * o1 * v1 * v1      # H2P1 (+ b = t')
           + o1 * o1 * v1 * v1 * (2 * V - 3))                    # H2P2
    occ = (po * pv * 2 * (O - 2)
           + O * O * V * V * (O - 1)
           + po1 * pv1 * 2 * (O - 3)
           + po * pv * 2 * (O - 2) + o1 * pv * o1                # H1P1 (+ t up -> any, j = t)
           + po * v1 * v1 * 2 * (O - 2) + o1 * v1 * v1 * o1      # H1P2 (+ j = t)
           + o1 * o1 * pv * (2 * O - 3)                          # H2P1
           + o1 * o1 * v1 * v1 * (2 * O - 3))                    # H2P2
    ov = 2 * (9 * po1 * pv1 + 5 * (po * pv + po * v1 * v1 + o1 * o1 * pv + o1 * o1 * v1 * v1))
    return dict(diag=rows, vir=vir, occ=occ, ov=ov, total=rows + vir + occ + ov)


def sigma_flops(no, nv):
    """(virtual-index flops, all other flops) of one sigma application: 2 x the
    vir nonzeros (the Sylvester products' work) and 2 x the rest."""
    z = sigma_nnz(no, nv)
    return 2 * z["vir"], 2 * (z["total"] - z["vir"])


def amplitudes(no, nv):
    """Stored amplitudes (the library's layout)."""
    return (_c2(no) * _c2(nv) + no * no * nv * nv + _c2(no - 1) * _c2(nv - 1) + _c2(no) * _c2(nv)
            + _c2(no) * (nv - 1) ** 2 + (no - 1) ** 2 * _c2(nv) + (no - 1) ** 2 * (nv - 1) ** 2)
