"""Tier 2 of the oracle: the modified-H0 problem in the seven-box layout.

Test infrastructure.  Plain FP64 numpy.  Each box is held internally as a
dense tensor over its free indices (antisymmetric pairs unpacked); the
Fock operator acts on every index slot, exactly as a one-body operator acts
on an excitation string:

  sigma^{A..}_{I..} = sum_slots sum_E f_{A_s E} t^{..E..} - sum_slots sum_M f_{M I_s} t_{..M..}
                      + (E_Phi - E0) t + f_vo excitation (doubles -> triples)
                      + f_ov de-excitation (triples -> doubles),

restricted to doubles + L-triples (paper Sec. II.C, the modified Q F Q);
a slot whose replacement leaves L is dropped, one that moves a pinned TOP
index to another box is a box transfer.  E_Phi - E0 = -omega with
omega = sum_l lambda_l^2 (f_{l'l'} - f_{ll}).  The de-excitation terms are
the adjoint (in the weighted inner product) of the excitation terms, since
the operator is symmetric.

Singlet (spin = 0) or the M_s = 0 triplet (spin = 1, beta singles of Psi0
negated): for the triplet the first-order amplitudes are antisymmetric under
the flip of every spin, so every term that reaches a stored amplitude through
the flip partner of another picks up a factor -1.

The right-hand side is <mu|H|Psi0> for the single-excitation reference
(singles -> doubles: f^Phi_{ov} and the integrals with one TOP index;
singles -> triples: antisymmetrised (ov|ov)).  E2_S is the direct
inversion of the diagonal S-triple block.  Everything is pinned against the
explicit determinant tier (``explicit``) by brute force at tiny sizes.
"""
from __future__ import annotations

import numpy as np

from .layout import box_sizes, box_offsets, WEIGHTS


# ---------------------------------------------------------------------------
# packing between the stored layout and dense per-box tensors
# ---------------------------------------------------------------------------
def _triu(m, lo=0):
    iu = np.triu_indices(m - lo, 1)
    return iu[0] + lo, iu[1] + lo


def _unpack_anti(vec2d, m, lo=0):
    """rows of packed strict-upper vectors -> dense antisymmetric (.., m-lo, m-lo)."""
    k = m - lo
    r, c = np.triu_indices(k, 1)
    out = np.zeros(vec2d.shape[:-1] + (k, k))
    out[..., r, c] = vec2d
    out[..., c, r] = -vec2d
    return out


def _pack_anti(dense):
    k = dense.shape[-1]
    r, c = np.triu_indices(k, 1)
    return dense[..., r, c]


class Boxes:
    """Dense per-box tensors of one amplitude vector."""

    def __init__(self, no, nv):
        self.no, self.nv = no, nv

    def unpack(self, x):
        no, nv = self.no, self.nv
        off = box_offsets(no, nv)
        g = lambda k: x[off[k]:off[k + 1]]
        npo = no * (no - 1) // 2
        npo1 = (no - 1) * (no - 2) // 2
        d = {}
        # T2: [pair(i<j)][pair(a<b)] -> T[i,j,a,b]
        c2v = nv * (nv - 1) // 2
        c2v1 = (nv - 1) * (nv - 2) // 2
        t = _unpack_anti(g(0).reshape(npo, c2v), nv)            # (npo, nv, nv)
        d["T2"] = self._unpack_occ(t, no, 0)
        d["S2"] = g(1).reshape(no, no, nv, nv).copy()
        t = _unpack_anti(g(2).reshape(npo1, c2v1), nv, 1)          # (npo1, nv-1, nv-1)
        d["T3L"] = self._unpack_occ(t, no, 1)
        t = _unpack_anti(g(3).reshape(npo, c2v), nv)
        d["H11"] = self._unpack_occ(t, no, 0)
        t = g(4).reshape(npo, nv - 1, nv - 1)
        d["H12"] = self._unpack_occ(t, no, 0)
        d["H21"] = _unpack_anti(g(5).reshape((no - 1) * (no - 1), c2v), nv).reshape(no - 1, no - 1, nv, nv)
        d["H22"] = g(6).reshape(no - 1, no - 1, nv - 1, nv - 1).copy()
        return d

    @staticmethod
    def _unpack_occ(t, no, lo):
        k = no - lo
        r, c = np.triu_indices(k, 1)
        out = np.zeros((k, k) + t.shape[1:])
        out[r, c] = t
        out[c, r] = -t
        return out

    def pack(self, d):
        no = self.no
        parts = []
        r, c = np.triu_indices(no, 1)
        parts.append(_pack_anti(d["T2"][r, c]).ravel())
        parts.append(d["S2"].ravel())
        r1, c1 = np.triu_indices(no - 1, 1)
        parts.append(_pack_anti(d["T3L"][r1, c1]).ravel())
        parts.append(_pack_anti(d["H11"][r, c]).ravel())
        parts.append(d["H12"][r, c].ravel())
        parts.append(_pack_anti(d["H21"]).ravel())
        parts.append(d["H22"].ravel())
        return np.concatenate(parts)


def _anti_occ(x):
    """antisymmetrise over the two leading (occupied) indices."""
    return x - x.transpose(1, 0, *range(2, x.ndim))


# ---------------------------------------------------------------------------
# the operator
# ---------------------------------------------------------------------------
class Structured:
    """sigma = (H0 - E0) x on doubles + L-triples, in the seven-box layout."""

    def __init__(self, f, lam, n_occ, omega=None, spin=0):
        """f: Fock matrix in the TOP basis, or in any basis that differs from
        it by a rotation of the occupied orbitals other than t and of the
        virtuals other than t'; then omega (computed in the TOP basis) must be
        given, since it reads the TOP orbitals' diagonal Fock elements.
        spin = 0: singlet reference; 1: the M_s = 0 triplet (Sec. II.A: the
        beta singles enter Psi0 with the opposite sign), whose first-order
        amplitudes are antisymmetric under the flip of every spin: a stored
        amplitude's flip partner carries the amplitude times sg = -1."""
        f = np.asarray(f, dtype=np.float64)
        self.spin = spin
        self.sg = -1.0 if spin else 1.0
        self.no = no = n_occ
        self.nv = nv = f.shape[0] - n_occ
        self.lam = np.asarray(lam, dtype=np.float64)
        self.fo = f[:no, :no]
        self.fv = f[no:, no:]
        self.fov = f[:no, no:]          # fov[i, a] = f_{i a} = f_{a i}
        if omega is None:
            omega = np.sum(self.lam ** 2 * (np.diag(self.fv)[:no] - np.diag(self.fo)))
        self.omega = float(omega)
        self.E0 = float(2.0 * np.trace(self.fo) + self.omega)
        # diagonal constant of the pinned TOP pair in every L box
        self.kappa = self.fv[0, 0] - self.fo[0, 0] - self.omega
        self.boxes = Boxes(no, nv)
        self.w = np.concatenate([np.full(m, w) for m, w in zip(box_sizes(no, nv), WEIGHTS)])
        self.dim = int(sum(box_sizes(no, nv)))

    # -- helpers -------------------------------------------------------------
    @staticmethod
    def _vv(F1, F2, X):
        """sum_E F1[a,E] X[..,E,c] + sum_E F2[c,E] X[..,a,E]"""
        return np.einsum("ae,...ec->...ac", F1, X) + np.einsum("ce,...ae->...ac", F2, X)

    @staticmethod
    def _oo(F1, F2, X):
        """sum_M F1[M,i] X[M,k,..] + sum_M F2[M,k] X[i,M,..]"""
        return np.einsum("mi,mk...->ik...", F1, X) + np.einsum("mk,im...->ik...", F2, X)

    def sigma_boxes(self, d):
        fo, fv, fov = self.fo, self.fv, self.fov
        fo1, fv1 = fo[1:, 1:], fv[1:, 1:]
        om, ka = self.omega, self.kappa
        T2, T3, H11, H12, H21, H22 = d["T2"], d["T3L"], d["H11"], d["H12"], d["H21"], d["H22"]
        S = 0.5 * (d["S2"] + self.sg * d["S2"].transpose(1, 0, 3, 2))     # flip-(anti)symmetrised S2
        o = {}
        # ---- diagonal-block (same box) Fock action ------------------------
        o["T2"] = self._vv(fv, fv, T2) - self._oo(fo, fo, T2) - om * T2
        o["S2"] = self._vv(fv, fv, S) - self._oo(fo, fo, S) - om * S
        o["T3L"] = self._vv(fv1, fv1, T3) - self._oo(fo1, fo1, T3) + ka * T3
        o["H11"] = self._vv(fv, fv, H11) - self._oo(fo, fo, H11) + ka * H11
        o["H12"] = self._vv(fv1, fv1, H12) - self._oo(fo, fo, H12) + ka * H12
        o["H21"] = self._vv(fv, fv, H21) - self._oo(fo1, fo1, H21) + ka * H21
        o["H22"] = self._vv(fv1, fv1, H22) - self._oo(fo1, fo1, H22) + ka * H22
        # ---- box transfers (pinned index moved by one Fock element) -------
        # up particle t' -> E: H1P1 (down pair holding t') <-> H1P2, H2P1 <-> H2P2
        v = np.einsum("e,jkec->jkc", fv[0, 1:], H12)
        o["H11"][:, :, 0, 1:] += v
        o["H11"][:, :, 1:, 0] -= v
        o["H12"] += fv[1:, 0][None, None, :, None] * H11[:, :, 0, 1:][:, :, None, :]
        v = np.einsum("e,ikec->ikc", fv[0, 1:], H22)
        o["H21"][:, :, 0, 1:] += v
        o["H21"][:, :, 1:, 0] -= v
        o["H22"] += fv[1:, 0][None, None, :, None] * H21[:, :, 0, 1:][:, :, None, :]
        # up hole t -> M: H1P1 (down pair holding t) <-> H2P1, H1P2 <-> H2P2
        v = np.einsum("m,mk...->k...", fo[1:, 0], H21)
        o["H11"][0, 1:] -= v
        o["H11"][1:, 0] += v
        o["H21"] -= fo[0, 1:][:, None, None, None] * H11[0, 1:][None]
        v = np.einsum("m,mk...->k...", fo[1:, 0], H22)
        o["H12"][0, 1:] -= v
        o["H12"][1:, 0] += v
        o["H22"] -= fo[0, 1:][:, None, None, None] * H12[0, 1:][None]
        # ---- doubles -> L-triples (f_vo) -------------------------------------
        self._excite(o, T2, S)
        # ---- L-triples -> doubles (f_ov), adjoint of the above -------------
        self._deexcite(o, T3, H11, H12, H21, H22)
        return o

    def _excite(self, o, T2, S):
        fov = self.fov
        # T3L <- T2 (up up up from up up)
        u = T2[1:, 1:, 1:, 1:]
        al = T2[0, 1:, 1:, 1:]                     # T2[t k][b c]
        be = T2[1:, 1:, 0, 1:]                     # T2[j k][t' c]
        ga = T2[0, 1:, 0, 1:]                      # T2[t k][t' c]
        ft_o = fov[1:, 0]                          # f_{t' j}
        fo_t = fov[0, 1:]                          # f_{b t}
        fjb = fov[1:, 1:]                          # f_{b j} as [j, b]
        x = fov[0, 0] * u
        x -= _anti_occ(ft_o[:, None, None, None] * al[None])
        bt = fo_t[None, None, :, None] * be[:, :, None, :]
        x -= bt - bt.transpose(0, 1, 3, 2)
        g4 = fjb[:, None, :, None] * ga[None, :, None, :]          # f_{bj} ga[k,c] -> [j,k,b,c]
        g4 = g4 - g4.transpose(1, 0, 2, 3)
        g4 = g4 - g4.transpose(0, 1, 3, 2)
        x += g4
        o["T3L"] += x
        # S3 boxes <- T2 (down-down copy = flip partner of T2, amplitude sg T2; up pair = f_{a i})
        sg = self.sg
        o["H11"] += sg * fov[0, 0] * T2
        o["H12"] += sg * fov[0, 1:][None, None, :, None] * T2[:, :, 0, 1:][:, :, None, :]
        o["H21"] += sg * fov[1:, 0][:, None, None, None] * T2[0, 1:][None]
        o["H22"] += sg * fov[1:, 1:][:, None, :, None] * T2[0, 1:, 0, 1:][None, :, None, :]
        # S3 boxes <- S2 (down pair = f_{b j}), S = flip-symmetrised S2
        s = S[0, :, 0, :]                                           # s[k, c] = S[t k t' c]
        h = fov.T[None, None, :, :] * 0                              # placeholder shape check
        g = fov[:, None, :, None] * s[None, :, None, :]              # f_{bj} s[k,c] -> [j,k,b,c]
        g = g - g.transpose(1, 0, 2, 3)
        g = g - g.transpose(0, 1, 3, 2)
        o["H11"] += g
        # H1P2: i=t, b=t'; a,c in 1..
        A = fov[:, 0][:, None, None, None] * S[0, :, 1:, 1:][None]   # f_{t' j} S[t k a c] -> [j,k,a,c]
        o["H12"] += A - A.transpose(1, 0, 2, 3)
        Bm = -fov[:, 1:][:, None, None, :] * S[0, :, 1:, 0][None, :, :, None]  # -f_{c j} S[t k a t']
        o["H12"] += Bm - Bm.transpose(1, 0, 2, 3)
        # H2P1: a=t', j=t; i,k in 1..; b<c all
        C1 = fov[0, :][None, None, :, None] * S[1:, 1:, 0, :][:, :, None, :]   # f_{b t} S[i k t' c]
        C2 = -fov[1:, :][None, :, :, None] * S[1:, 0, 0, :][:, None, None, :]  # -f_{b k} S[i t t' c]
        Cs = C1 + C2
        o["H21"] += Cs - Cs.transpose(0, 1, 3, 2)
        # H2P2: i,k in 1..; a,c in 1..
        o["H22"] += fov[0, 0] * S[1:, 1:, 1:, 1:]
        o["H22"] -= fov[1:, 0][None, :, None, None] * S[1:, 0, 1:, 1:][:, None, :, :]
        o["H22"] -= fov[0, 1:][None, None, None, :] * S[1:, 1:, 1:, 0][:, :, :, None]
        o["H22"] += fov[1:, 1:][None, :, None, :] * S[1:, 0, 1:, 0][:, None, :, None]
        del h

    def _deexcite(self, o, T3, H11, H12, H21, H22):
        fov = self.fov
        no = self.no
        t2 = np.zeros_like(o["T2"])
        # from T3L
        t2[1:, 1:, 1:, 1:] += fov[0, 0] * T3
        v = -np.einsum("j,jkbc->kbc", fov[1:, 0], T3)               # T2[t k][b c]
        t2[0, 1:, 1:, 1:] += v
        t2[1:, 0, 1:, 1:] -= v
        v = -np.einsum("b,jkbc->jkc", fov[0, 1:], T3)               # T2[j k][t' c]
        t2[1:, 1:, 0, 1:] += v
        t2[1:, 1:, 1:, 0] -= v
        v = np.einsum("jb,jkbc->kc", fov[1:, 1:], T3)                # T2[t k][t' c]
        t2[0, 1:, 0, 1:] += v
        t2[1:, 0, 0, 1:] -= v
        t2[0, 1:, 1:, 0] -= v
        t2[1:, 0, 1:, 0] += v
        o["T2"] += t2
        # from the S3 boxes, through their flip partners (down-down copy of T2): sg
        t2 = np.zeros_like(o["T2"])
        t2 += fov[0, 0] * H11
        v = np.einsum("a,jkac->jkc", fov[0, 1:], H12)               # T2[j k][t' c]
        t2[:, :, 0, 1:] += v
        t2[:, :, 1:, 0] -= v
        v = np.einsum("i,ikbc->kbc", fov[1:, 0], H21)               # T2[t k][b c]
        t2[0, 1:] += v
        t2[1:, 0] -= v
        v = np.einsum("ia,ikac->kc", fov[1:, 1:], H22)               # T2[t k][t' c]
        t2[0, 1:, 0, 1:] += v
        t2[1:, 0, 0, 1:] -= v
        t2[0, 1:, 1:, 0] -= v
        t2[1:, 0, 1:, 0] += v
        o["T2"] += self.sg * t2
        # S2 <- S3 boxes: d = E^T x (per determinant), sigma_S2 += d + flip(d)
        d = np.zeros_like(o["S2"])
        d[0, :, 0, :] += np.einsum("jb,jkbc->kc", fov, H11)
        d[0, :, 1:, 1:] += np.einsum("j,jkac->kac", fov[:, 0], H12)
        d[0, :, 1:, 0] -= np.einsum("jc,jkac->ka", fov[:, 1:], H12)
        d[1:, 1:, 0, :] += np.einsum("b,ikbc->ikc", fov[0, :], H21)
        d[1:, 0, 0, :] -= np.einsum("kb,ikbc->ic", fov[1:, :], H21)
        d[1:, 1:, 1:, 1:] += fov[0, 0] * H22
        d[1:, 0, 1:, 1:] -= np.einsum("k,ikac->iac", fov[1:, 0], H22)
        d[1:, 1:, 1:, 0] -= np.einsum("c,ikac->ika", fov[0, 1:], H22)
        d[1:, 0, 1:, 0] += np.einsum("kc,ikac->ia", fov[1:, 1:], H22)
        o["S2"] += d + self.sg * d.transpose(1, 0, 3, 2)

    def sigma(self, x):
        return self.boxes.pack(self.sigma_boxes(self.boxes.unpack(x)))

    # -- diagonal ------------------------------------------------------------
    def diagonal(self):
        """D_mu = <mu|F|mu> - E0 (the Jacobi preconditioner)."""
        eo, ev = np.diag(self.fo), np.diag(self.fv)
        no, nv, om = self.no, self.nv, self.omega
        d = {}
        d["T2"] = ev[None, None, :, None] + ev[None, None, None, :] - eo[:, None, None, None] - eo[None, :, None, None] - om
        d["S2"] = d["T2"].copy()
        base = ev[0] - eo[0] - om
        d["T3L"] = base + ev[None, None, 1:, None] + ev[None, None, None, 1:] - eo[1:, None, None, None] - eo[None, 1:, None, None]
        d["H11"] = base + ev[None, None, :, None] + ev[None, None, None, :] - eo[:, None, None, None] - eo[None, :, None, None]
        d["H12"] = base + ev[None, None, 1:, None] + ev[None, None, None, 1:] - eo[:, None, None, None] - eo[None, :, None, None]
        d["H21"] = base + ev[None, None, :, None] + ev[None, None, None, :] - eo[1:, None, None, None] - eo[None, 1:, None, None]
        d["H22"] = base + ev[None, None, 1:, None] + ev[None, None, None, 1:] - eo[1:, None, None, None] - eo[None, 1:, None, None]
        return self.boxes.pack(d)

    def dot(self, x, y):
        return float(np.sum(self.w * x * y))


# ---------------------------------------------------------------------------
# right-hand side b = <mu|H|Psi0>, and E2_S
# ---------------------------------------------------------------------------
# index ranges (occupied, virtual) of the free indices of each box: 0 = all
# orbitals of the kind, 1 = all but the pinned TOP orbital (t or t')
BOX_RANGES = {"T2": (0, 0), "S2": (0, 0), "T3L": (1, 1), "H11": (0, 0), "H12": (0, 1), "H21": (1, 0),
              "H22": (1, 1)}


def transform_amplitudes(x, no, nv, To, Tv):
    """Amplitudes after the orbital rotation that fixes t and t': new orbital
    P' = sum_P To[P, P'] P (occupied, To[0] = e_0), likewise Tv for the
    virtuals.  Every free index of every box is contracted with the matching
    block of To or Tv.  D + L is invariant under such rotations, so this is an
    orthogonal map of the first-order space onto itself."""
    bx = Boxes(no, nv)
    d = bx.unpack(x)
    out = {}
    for k, X in d.items():
        lo_o, lo_v = BOX_RANGES[k]
        U, V = To[lo_o:, lo_o:], Tv[lo_v:, lo_v:]
        out[k] = np.einsum("ijab,iI,jJ,aA,bB->IJAB", X, U, U, V, V, optimize=True)
    return bx.pack(out)


def _anti2(x):
    """P(ij) P(ab) on a [i,j,a,b] tensor."""
    x = x - x.transpose(1, 0, 2, 3)
    return x - x.transpose(0, 1, 3, 2)


class RHS:
    """Integral blocks in the TOP basis and the right-hand side.

    Ft: TOP-basis Fock (N x N); Bt: TOP-basis factor (n_aux x N x N);
    (pq|rs) = sum_Q Bt[Q,p,q] Bt[Q,r,s].
    """

    def __init__(self, Ft, Bt, lam, n_occ, spin=0):
        no = n_occ
        self.no, self.nv = no, Ft.shape[0] - no
        nv = self.nv
        self.lam = np.asarray(lam, dtype=np.float64)
        self.c = self.lam / np.sqrt(2.0)
        self.sg = -1.0 if spin else 1.0       # sign of the beta singles in Psi0
        self.op = Structured(Ft, lam, n_occ, spin=spin)
        Bov = Bt[:, :no, no:]
        self.V = np.einsum("Qia,Qjb->iajb", Bov, Bov, optimize=True)           # (ia|jb)
        self.W = np.einsum("Qal,Qjb->albj", Bt[:, no:, no:2 * no], Bov, optimize=True)  # (a l'|b j)
        self.Z = np.einsum("Qli,Qjb->libj", Bt[:, :no, :no], Bov, optimize=True)        # (l i|b j)
        # f^Phi_ov = F~_ov - G[gamma - gamma_Phi]_ov
        l2 = self.lam ** 2
        idx = np.arange(no)
        Bvv_d = Bt[:, no + idx, no + idx]                 # (Q, l): B[l'l']
        Boo_d = Bt[:, idx, idx]                           # (Q, l): B[ll]
        J = np.einsum("Qia,Ql,l->ia", Bov, Bvv_d - Boo_d, l2, optimize=True)
        Kv = np.einsum("Qil,Qla,l->ia", Bt[:, :no, no:2 * no], Bt[:, no:2 * no, no:], l2, optimize=True)
        Ko = np.einsum("Qil,Qla,l->ia", Bt[:, :no, :no], Bt[:, :no, no:], l2, optimize=True)
        self.fphi_ov = Ft[:no, no:] - (J - 0.5 * Kv + 0.5 * Ko)

    def rhs_boxes(self):
        no, nv = self.no, self.nv
        c = self.c
        V, W, Z, fp = self.V, self.W, self.Z, self.fphi_ov
        cv = np.zeros(nv)
        cv[:no] = c                                        # c_a for a TOP virtual a
        dlt = np.zeros((no, nv))
        dlt[np.arange(no), np.arange(no)] = 1.0            # delta(a == i)
        g = (c[:, None] * dlt)[:, None, :, None] * fp[None, :, None, :]        # c_i d(a,i) fphi[j,b]
        h = c[:, None, None, None] * W.transpose(1, 3, 0, 2)                  # c_i W[a,i,b,j] -> [i,j,a,b]
        zz = np.zeros((no, no, nv, nv))
        zz[:, :, :no, :] = Z.transpose(1, 3, 0, 2)[:, :, :, :]                # Z[a,i,b,j] -> [i,j,a,b], a < no
        k = -cv[None, None, :, None] * zz
        m = g + h + k
        sg = self.sg
        d = {}
        d["T2"] = _anti2(m)
        d["S2"] = m + sg * m.transpose(1, 0, 3, 2)       # second term: the beta singles
        # triples
        c0 = c[0]
        Vx = V.transpose(0, 2, 1, 3)                                           # [j,k,b,c] = (jb|kc)
        AS = Vx - Vx.transpose(1, 0, 2, 3)                                     # (bj|ck) - (bk|cj)
        e_tt = V[0, 0]                                                         # (t t'|k c) as [k,c]
        e_kt = V[:, 0, 0, :]                                                   # (k t'|t c) as [k,c]
        # T3L
        q = (c[:, None] * dlt)[1:, None, 1:, None] * (e_tt - e_kt)[None, 1:, None, 1:]
        d["T3L"] = c0 * AS[1:, 1:, 1:, 1:] + _anti2(q)
        q = (c[:, None] * dlt)[:, None, :, None] * e_tt[None, :, None, :]
        d["H11"] = c0 * AS + sg * _anti2(q)                 # alpha single t -> t'; beta singles
        # H1P2 [j,k,a,c], a,c in 1..
        r = np.zeros((no, no, nv - 1, nv - 1))
        r[0] += c0 * V[0, 1:, :, 1:].transpose(1, 0, 2)                      # d(j,t) c_t (a t|c k)
        r -= (c[:, None] * dlt[:, 1:])[:, None, None, :] * V[0, 1:, :, 0].T[None, :, :, None]
        d["H12"] = sg * (r - r.transpose(1, 0, 2, 3))     # beta singles only
        # H2P1 [i,k,b,c], i,k in 1..
        s = np.zeros((no - 1, no - 1, nv, nv))
        s[:, :, 0, :] += c0 * V[1:, 0, 1:, :]
        s -= (c[:, None] * dlt)[None, 1:, :, None] * V[1:, 0, 0, :][:, None, None, :]
        d["H21"] = sg * (s - s.transpose(0, 1, 3, 2))     # beta singles only
        # H2P2 [i,k,a,c]
        u = (c[:, None] * dlt)[1:, None, 1:, None] * (e_tt - e_kt)[None, 1:, None, 1:]      # alpha single i -> i'
        w = c0 * V[1:, 1:, 1:, 1:].transpose(0, 2, 1, 3)                                    # beta singles
        w = w + (c[:, None] * dlt)[None, 1:, None, 1:] * V[1:, 1:, 0, 0][:, None, :, None]
        d["H22"] = u + sg * w
        return d

    def rhs(self):
        return self.op.boxes.pack(self.rhs_boxes())

    # -- E2_S: direct inversion over the S-triples --------------------------
    def e2_s(self):
        """-sum over S-triple determinants of b^2 / D (both spin-flip partners)."""
        return -sum(2.0 * np.sum(b * b / D) for b, D in self.s_terms())

    def s_terms(self):
        """(b, D) arrays over the S-triple determinants, chunk by chunk in a
        fixed order; each determinant stands for itself and its spin-flip
        partner, which has the same b and D."""
        no, nv = self.no, self.nv
        c, V = self.c, self.V
        eo, ev = np.diag(self.op.fo), np.diag(self.op.fv)
        om = self.op.omega
        # ---- same-spin sector (up up up; x2 for down down down) --------------
        # enumerated by the smallest TOP l contained; t = 0 excluded.
        for l in range(1, no):
            occ = [m for m in range(no) if m != l]
            vir = [a for a in range(nv) if a != l]
            jk = np.array([(j, k) for ii, j in enumerate(occ) for k in occ[ii + 1:]]).reshape(-1, 2)
            bc = np.array([(b, cc) for ii, b in enumerate(vir) for cc in vir[ii + 1:]]).reshape(-1, 2)
            if len(jk) == 0 or len(bc) == 0:
                continue
            J = jk[:, 0][:, None]
            K = jk[:, 1][:, None]
            Bb = bc[:, 0][None, :]
            Cc = bc[:, 1][None, :]
            keep = np.ones((len(jk), len(bc)), dtype=bool)
            for m in range(l):
                keep &= ~(((J == m) | (K == m)) & ((Bb == m) | (Cc == m)))
            I = np.sort(np.stack(np.broadcast_arrays(np.full(J.shape, l), J, K), -1), -1)
            A = np.sort(np.stack(np.broadcast_arrays(np.full(Bb.shape, l), Bb, Cc), -1), -1)
            I = np.broadcast_to(I, keep.shape + (3,))[keep]
            A = np.broadcast_to(A, keep.shape + (3,))[keep]
            b = np.zeros(len(I))
            for p in range(3):
                for qq in range(3):
                    hit = A[:, p] == I[:, qq]
                    if not hit.any():
                        continue
                    ap = [x for x in range(3) if x != p]
                    iq = [x for x in range(3) if x != qq]
                    a1, a2 = A[hit][:, ap[0]], A[hit][:, ap[1]]
                    i1, i2 = I[hit][:, iq[0]], I[hit][:, iq[1]]
                    anti = V[i1, a1, i2, a2] - V[i2, a1, i1, a2]
                    b[hit] += (-1) ** (p + qq) * c[I[hit][:, qq]] * anti
            D = ev[A].sum(1) - eo[I].sum(1) - om
            yield b, D
        # ---- mixed sector (up; down down), x2 for its flip ---------------------
        occ_pairs = np.array([(j, k) for j in range(no) for k in range(j + 1, no)]).reshape(-1, 2)
        vir_pairs = np.array([(b, cc) for b in range(nv) for cc in range(b + 1, nv)]).reshape(-1, 2)
        for i in range(no):
            for a in range(nv):
                J = occ_pairs[:, 0][:, None]
                K = occ_pairs[:, 1][:, None]
                Bb = vir_pairs[:, 0][None, :]
                Cc = vir_pairs[:, 1][None, :]
                up_top = (a == i)
                dn_top = (Bb == J) | (Bb == K) | (Cc == J) | (Cc == K)
                if up_top:
                    if i == 0:
                        continue                      # contains t: L
                    keep = np.ones(dn_top.shape, dtype=bool)
                else:
                    keep = dn_top
                has_t_h = (i == 0) | (J == 0) | (K == 0)
                has_t_p = (a == 0) | (Bb == 0) | (Cc == 0)
                keep = keep & ~(has_t_h & has_t_p)
                if not keep.any():
                    continue
                jj = np.broadcast_to(J, keep.shape)[keep]
                kk = np.broadcast_to(K, keep.shape)[keep]
                bb = np.broadcast_to(Bb, keep.shape)[keep]
                cc = np.broadcast_to(Cc, keep.shape)[keep]
                bd = np.zeros(len(jj))                # from the beta singles (down TOP pairs)
                m = bb == jj
                bd[m] += c[jj[m]] * V[i, a, kk[m], cc[m]]
                m = bb == kk
                bd[m] -= c[kk[m]] * V[i, a, jj[m], cc[m]]
                m = cc == jj
                bd[m] -= c[jj[m]] * V[i, a, kk[m], bb[m]]
                m = cc == kk
                bd[m] += c[kk[m]] * V[i, a, jj[m], bb[m]]
                b = self.sg * bd
                if up_top:                            # the alpha single i -> i'
                    b = b + c[i] * (V[jj, bb, kk, cc] - V[kk, bb, jj, cc])
                D = ev[a] + ev[bb] + ev[cc] - eo[i] - eo[jj] - eo[kk] - om
                yield b, D


# ---------------------------------------------------------------------------
# Jacobi-preconditioned conjugate gradient and the energy
# ---------------------------------------------------------------------------
def pcg(op, b, tol=1e-8, max_iter=200, x0=None, history=None):
    """Solve A x = -b with A = (H0 - E0) on D + L (weighted inner product).

    The paper solves the first-order equation by conjugate gradient; the
    preconditioner (the diagonal D), x0 = 0 and the stopping rule
    ||b + A x||_W / ||b||_W <= tol are this implementation's choices.
    """
    D = op.diagonal()
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = -b - op.sigma(x) if x0 is not None else -b.copy()
    z = r / D
    p = z.copy()
    rho = op.dot(r, z)
    bn = np.sqrt(op.dot(b, b))
    it = 0
    rel = np.sqrt(op.dot(r, r)) / bn
    while rel > tol and it < max_iter:
        q = op.sigma(p)
        pq = op.dot(p, q)
        if pq <= 0:
            raise FloatingPointError("operator not positive definite")
        alpha = rho / pq
        x += alpha * p
        r -= alpha * q
        it += 1
        rel = np.sqrt(op.dot(r, r)) / bn
        if history is not None:
            history.append((rel, op.dot(b, x) - op.dot(x, r)))
        z = r / D
        rho_new = op.dot(r, z)
        p = z + (rho_new / rho) * p
        rho = rho_new
    return x, r, it, rel


def solve(Ft, Bt, lam, n_occ, tol=1e-8, max_iter=200, spin=0):
    rh = RHS(Ft, Bt, lam, n_occ, spin=spin)
    op = rh.op
    b = rh.rhs()
    x, r, it, rel = pcg(op, b, tol=tol, max_iter=max_iter)
    e2_dl = op.dot(b, x) - op.dot(x, r)          # Hylleraas form
    e2_s = rh.e2_s()
    return dict(e2=e2_dl + e2_s, e2_dl=e2_dl, e2_s=e2_s, e0=op.E0, iters=it, rel=rel,
                x=x, b=b)


def solve_problem(prob, tol=1e-8, max_iter=200, spin=0):
    from .topbasis import top_rotation, rotate
    lam, R = top_rotation(prob.F, prob.C, prob.n_occ)
    Ft, Bt = rotate(prob.F, prob.B, R)
    out = solve(Ft, Bt, lam, prob.n_occ, tol=tol, max_iter=max_iter, spin=spin)
    out["lam"] = lam
    return out
