"""Structural size of the operator (H0 - E0) on doubles + L-triples (oracle).

Test infrastructure.  Counts, by enumeration of the explicit (tier-1)
operator, the nonzero couplings of sigma = (H0 - E0) x in the representative
basis the amplitude vectors use: one row per stored amplitude, the two
determinants of a spin-flip pair in one row, the two members of an S2 flip
pair (i, j, a, b) ~ (j, i, b, a) in one row (the flip-unique S2 reading).
Each nonzero is one multiply-add of sigma, so 2 x nnz is its algorithmic
flop count.

The Fock matrix is generic (every element nonzero) so that no coupling
vanishes by accident.  Each nonzero is classified by the one spin-orbital
replacement that links the two determinants (paper Sec. III.B / Table I
sort the contractions the same way, by the index kinds they run over):

* ``diag`` -- the same determinant (orbital-energy differences and E0);
* ``vir``  -- a particle replaced by another virtual (the virtual-index
  Fock contractions, N_o^2 N_v^3 in total);
* ``occ``  -- a hole replaced by another occupied orbital (N_o^3 N_v^2);
* ``ov``   -- a change of excitation level through f_ov (doubles <->
  L-triples, N_o^2 N_v^2).
"""
from __future__ import annotations

import numpy as np

from .explicit import ExplicitESMP2
from .layout import rep_map


def _generic_problem(no, nv, seed):
    n = no + nv
    rng = np.random.default_rng(seed)
    F = rng.uniform(0.5, 1.5, (n, n)) * rng.choice([-1.0, 1.0], (n, n))
    F = F + F.T
    lam = np.sort(rng.uniform(0.2, 1.0, no))[::-1]
    lam /= np.linalg.norm(lam)
    return F, lam


def rep_nnz(no, nv, seed=0):
    """Nonzeros of (H0 - E0) on D + L in the representative basis, by class:
    dict with keys diag, vir, occ, ov, total, and dim (the number of rows)."""
    n = no + nv
    F, lam = _generic_problem(no, nv, seed)
    ex = ExplicitESMP2(F, np.zeros((n, n, n, n)), lam, no)
    A = ex.fock_matrix().tocoo()
    rep = {}
    for g, (box, contrib, _) in enumerate(rep_map(no, nv)):
        for d, _ in contrib:
            rep[d] = min(rep.get(d, g), g)
    dl = ex.DL
    assert set(rep) == set(dl), "the layout covers exactly the determinants of D + L"
    occ_mask = ex.phi
    pairs = {}
    for r, c in zip(A.row, A.col):
        dr, dc = dl[r], dl[c]
        x = dr ^ dc
        if x == 0:
            cls = "diag"
        else:
            p, q = [k for k in range(2 * n) if (x >> k) & 1]
            kp, kq = (occ_mask >> p) & 1, (occ_mask >> q) & 1
            cls = "occ" if kp and kq else ("vir" if not kp and not kq else "ov")
        key = (rep[dr], rep[dc])
        prev = pairs.get(key)
        assert prev is None or prev == cls, "a representative pair linked by couplings of two kinds"
        pairs[key] = cls
    out = dict(diag=0, vir=0, occ=0, ov=0)
    for cls in pairs.values():
        out[cls] += 1
    out["total"] = sum(out.values())
    out["dim"] = len(set(rep.values()))
    return out
