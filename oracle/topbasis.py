"""Rotation to the transition-orbital-pair (TOP) basis (oracle, test infrastructure).

Paper, Sec. II.A (zeroth-order wave function): the singles coefficient matrix
is factored by a singular value decomposition C = U Lambda V^T, and an
occupied-occupied rotation (by U) plus a virtual-virtual rotation (by V)
turn the reference into a sum of n_occ pair excitations, one per singular
value.  The paper leaves the remaining virtual orbitals (the AVOs) otherwise
unspecified; this oracle fixes them as the orthonormal complement of the TOP
virtuals that diagonalises the Fock matrix inside that complement
(semicanonical AVOs, ascending energy).  Without that choice the diagonal
zeroth-order Hamiltonian of the S-triples would depend on an arbitrary basis.

Sign convention (both sides implement it): every occupied TOP orbital and
every AVO is signed so that its largest-magnitude coefficient in the input
orbital basis is positive; a TOP virtual takes the sign that makes its
singular value positive.  Singular values are in descending order.

Orbital order of the TOP basis: occupied TOP orbitals 0..n_occ-1 (by
descending singular value), then virtual index a = 0..n_vir-1 where a < n_occ
is the TOP partner of occupied a and a >= n_occ are the AVOs.
"""
from __future__ import annotations

import numpy as np


def _fix_sign(M):
    """Sign each column so that its largest-|entry| is positive."""
    idx = np.argmax(np.abs(M), axis=0)
    s = np.sign(M[idx, np.arange(M.shape[1])])
    s[s == 0] = 1.0
    return M * s, s


def top_rotation(F, C, n_occ):
    """Return (lam, R) with R (N x N) orthogonal: new orbital k = sum_p R[p,k] old p."""
    n_vir = C.shape[1]
    U, lam, Vt = np.linalg.svd(C, full_matrices=False)       # C = U diag(lam) Vt
    U, s = _fix_sign(U)
    V = Vt.T * s                                               # keep u_l^T C v_l = lam_l > 0
    # orthonormal complement of span(V) in the virtual space
    Q, _ = np.linalg.qr(V, mode="complete")
    Q2 = Q[:, n_occ:]
    Fvv = F[n_occ:, n_occ:]
    w, Y = np.linalg.eigh(Q2.T @ Fvv @ Q2)
    avo, _ = _fix_sign(Q2 @ Y)
    W = np.concatenate([V, avo], axis=1)
    n = n_occ + n_vir
    R = np.zeros((n, n))
    R[:n_occ, :n_occ] = U
    R[n_occ:, n_occ:] = W
    return lam, R


def rotate(F, B, R):
    """F~ = R^T F R and B~[Q] = R^T B[Q] R."""
    Ft = R.T @ F @ R
    Bt = np.einsum("pk,Qpq,ql->Qkl", R, B, R, optimize=True)
    return Ft, Bt


def eri_from_factor(Bt):
    """(pq|rs) = sum_Q B[Q,p,q] B[Q,r,s] (full tensor; tiny sizes only)."""
    return np.einsum("Qpq,Qrs->pqrs", Bt, Bt, optimize=True)


def pinned_semicanonical(Ft, n_occ):
    """Rotation (To, Tv) of the occupied orbitals other than t = 0 and of the
    virtuals other than t' = 0 that diagonalises their Fock blocks
    Ft[1:no, 1:no] and Ft[no+1:, no+1:] (t and t' fixed).  Doubles +
    L-triples are mapped onto themselves by such rotations (an L-triple
    keeps t among its holes and t' among its particles, Sec. II.B).
    Eigenvalues ascending; each eigenvector signed so that its
    largest-magnitude component is positive (the library's convention).
    New orbital P' = sum_P T[P, P'] P."""
    no = n_occ
    nv = Ft.shape[0] - no
    To, Tv = np.eye(no), np.eye(nv)
    To[1:, 1:] = _fix_sign(np.linalg.eigh(Ft[1:no, 1:no])[1])[0]
    Tv[1:, 1:] = _fix_sign(np.linalg.eigh(Ft[no + 1:, no + 1:])[1])[0]
    return To, Tv
