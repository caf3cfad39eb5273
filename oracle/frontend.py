"""The Fock operator of the reference's density (oracle, test infrastructure).

Paper, Sec. II.C: the zeroth-order Hamiltonian uses the Fock operator built
from the one-body density matrix of the ESMF reference.  Given the one-
electron operator h (input orbital basis), the factor B of the two-electron
integrals, (pq|rs) = sum_Q B[Q,p,q] B[Q,r,s], and the singles coefficients C
of Psi0 = sum_ia C_ia (E^up_ai + E^dn_ai)/sqrt(2) |Phi> (||C||_F = 1):

  gamma (spin-summed):  gamma_ij = 2 delta_ij - (C C^T)_ij,  gamma_ab = (C^T C)_ab,
                        gamma_ia = 0 (Psi0 has no closed-shell component),
  F = h + G[gamma],     G[g]_pq = sum_rs g_rs ((pq|rs) - (ps|rq)/2).

``density_explicit`` builds gamma from the determinant expansion of Psi0 (tiny
sizes) and pins the closed form.
"""
from __future__ import annotations

import numpy as np

from . import fermion as fm


def density(C, n_occ):
    """Spin-summed one-body density of Psi0 in the input orbital basis."""
    n_vir = C.shape[1]
    n = n_occ + n_vir
    g = np.zeros((n, n))
    g[:n_occ, :n_occ] = 2.0 * np.eye(n_occ) - C @ C.T
    g[n_occ:, n_occ:] = C.T @ C
    return g


def g_matrix(gam, B):
    """G[gamma]_pq = sum_rs gamma_rs ((pq|rs) - (ps|rq)/2) from the factor B."""
    J = np.einsum("Qpq,Qrs,rs->pq", B, B, gam, optimize=True)
    K = np.einsum("Qps,rs,Qrq->pq", B, gam, B, optimize=True)
    return J - 0.5 * K


def fock_from_core(h, B, C, n_occ):
    """F = h + G[gamma(Psi0)]."""
    return h + g_matrix(density(C, n_occ), B)


def density_explicit(C, n_occ):
    """gamma_pq = sum_spin <Psi0| a+_p a_q |Psi0> from the determinant expansion."""
    n_vir = C.shape[1]
    n = n_occ + n_vir
    phi = sum(1 << p for p in range(n_occ)) | sum(1 << (n + p) for p in range(n_occ))
    psi = {}
    for i in range(n_occ):
        for a in range(n_vir):
            for spin in (0, 1):
                r = fm.apply_string(phi, [("c", spin * n + n_occ + a), ("a", spin * n + i)])
                s, d = r
                psi[d] = psi.get(d, 0.0) + s * C[i, a] / np.sqrt(2.0)
    g = np.zeros((n, n))
    for p in range(n):
        for q in range(n):
            acc = 0.0
            for spin in (0, 1):
                for d, c in psi.items():
                    r = fm.apply_string(d, [("c", spin * n + p), ("a", spin * n + q)])
                    if r is None:
                        continue
                    s, d2 = r
                    acc += s * c * psi.get(d2, 0.0)
            g[p, q] = acc
    return g
