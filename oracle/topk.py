"""ESMP2-TOP(k): several transition-orbital pairs treated as large (oracle).

Test infrastructure (see the package docstring).  Paper Sec. II.C: the
L-triples are the triples that contain a *large* TOP, and how many TOPs are
large is a choice -- one ("TOP(1)"), a few, up to all of them ("TOP(all)",
the N^6 limit of Sec. III.B, Table II).  With the spatial reading R1 a
triple contains TOP l when spatial occupied l is among its holes and spatial
virtual l' among its particles.  L = triples containing any of the large
TOPs 0 .. k-1; S = triples containing only smaller TOPs (diagonal block,
inverted directly); N = the rest.

Layout (the interface the HIP library implements too): the doubles (T2, S2)
of the one-TOP layout, then, for every large TOP s = 0 .. k-1, the five
L-boxes of the one-TOP layout written for TOP s in place of TOP 0 (occupied
orbitals 0 and s swapped, virtuals 0' and s' swapped).  A triple that also
contains a larger TOP r < s belongs to set r: its slot in set s is held at
zero ("masked").

Storage convention: every element is the coefficient of its own determinant
(the one the one-TOP layout's operator string creates, with the relabelled
orbitals) in the canonical order -- spin-orbitals alpha then beta, each
ascending.  A spin-flip partner outside S2 carries sg times it (sg = +1
singlet, -1 M_s = 0 triplet); S2 stores both members of a pair and enters
the operator flip-symmetrised.

The operator is applied on determinants: for the determinant D0 of an
element, (F - E0) Psi at D0 collects the diagonal and every single
spin-orbital replacement D' of D0 that lies in D + L, with the matrix
element f_uv (-1)^(n(u) + n(v) - [u < v]), n(.) = occupied spin-orbitals of
D0 below.  The right-hand side and the S-triple energy come from the
one-TOP oracle (tier 2) applied to the relabelled problems:
  E2_S(TOP(k)) = E2_S(TOP(1)) + sum over L-triples outside L_0 of b^2 / D,
since those are exactly the TOP(1) S-triples that TOP(k) moves into L.
"""
from __future__ import annotations

import numpy as np

from . import fermion as fm
from . import structured
from .layout import enumerate_ops

SENT = 1023          # empty slot of a double in a key


def _relabel_orbital(o, no, s):
    """Swap occupied 0 <-> s and virtual 0' <-> s' (full orbital index)."""
    if o < no:
        return s if o == 0 else (0 if o == s else o)
    a = o - no
    return no + (s if a == 0 else (0 if a == s else a))


def relabel_problem(Ft, Bt, lam, no, s):
    """The problem with TOP s renamed to TOP 0 (and 0 to s)."""
    n = Ft.shape[0]
    perm = np.array([_relabel_orbital(o, no, s) for o in range(n)])
    lam_s = np.array(lam, dtype=np.float64).copy()
    lam_s[[0, s]] = lam_s[[s, 0]]
    return Ft[np.ix_(perm, perm)], Bt[:, perm][:, :, perm], lam_s


def _key(holes, parts):
    """int64 key of sorted hole / particle spin-orbitals (3 slots each, SENT
    for the missing third slot of a double)."""
    k = np.zeros(holes.shape[0], dtype=np.int64)
    for j in range(3):
        k |= holes[:, j].astype(np.int64) << (10 * j)
        k |= parts[:, j].astype(np.int64) << (30 + 10 * j)
    return k


class TopK:
    def __init__(self, Ft, Bt, lam, n_occ, n_top, spin=0):
        Ft = np.asarray(Ft, dtype=np.float64)
        self.Ft, self.Bt = Ft, Bt
        self.lam = np.asarray(lam, dtype=np.float64)
        self.no = no = n_occ
        self.n = n = Ft.shape[0]
        self.nv = n - no
        self.k = k = n_top
        self.sg = -1.0 if spin else 1.0
        self.spin = spin
        self.omega = float(np.sum(self.lam ** 2 * (np.diag(Ft)[no:2 * no] - np.diag(Ft)[:no])))
        self.E0 = float(2.0 * np.trace(Ft[:no, :no]) + self.omega)
        self.phi = sum(1 << p for p in range(no)) | sum(1 << (n + p) for p in range(no))
        holes, parts, sets, boxes, phase = [], [], [], [], []
        for s in range(k):
            for box, ops in enumerate_ops(no, self.nv):
                if s > 0 and box < 2:
                    continue                      # the doubles appear once, in set 0
                so = [(kind, sp, _relabel_orbital(o, no, s)) for kind, sp, o in ops]
                h = sorted(sp * n + o for kind, sp, o in so if kind == "a")
                p = sorted(sp * n + o for kind, sp, o in so if kind == "c")
                sign, _ = fm.apply_string(self.phi, [(kind, sp * n + o) for kind, sp, o in so])
                holes.append(h + [SENT] * (3 - len(h)))
                parts.append(p + [SENT] * (3 - len(p)))
                sets.append(s)
                boxes.append(box)
                phase.append(sign)
        self.holes = np.array(holes, dtype=np.int64)
        self.parts = np.array(parts, dtype=np.int64)
        self.set = np.array(sets)
        self.box = np.array(boxes)
        self.phase = np.array(phase, dtype=np.float64)   # canonical phase of the element's operator string
        self.dim = len(self.box)
        self.triple = self.holes[:, 2] != SENT
        # owner: smallest large TOP the triple contains; masked where it is not this set
        owner = np.full(self.dim, -1)
        for s in range(k - 1, -1, -1):
            has = np.zeros(self.dim, dtype=bool)
            sh = np.isin(self.holes % n, [s]).any(axis=1)
            sp = np.isin(self.parts % n, [no + s]).any(axis=1)
            has = sh & sp & self.triple
            owner[has] = s
        self.live = ~self.triple | (owner == self.set)
        self.w = np.where(self.box == 1, 1.0, 2.0)
        # lookup table: own determinants of live elements (factor 1), and the
        # spin-flip partners of live elements outside S2 (factor sg)
        own = _key(self.holes, self.parts)
        fh, fp = self._flip(self.holes), self._flip(self.parts)
        flip = _key(fh, fp)
        idx = np.arange(self.dim)
        live = self.live
        nons2 = live & (self.box != 1)
        keys = np.concatenate([own[live], flip[nons2]])
        elem = np.concatenate([idx[live], idx[nons2]])
        fac = np.concatenate([np.ones(live.sum()), np.full(nons2.sum(), self.sg)])
        isown = np.concatenate([np.ones(live.sum(), dtype=bool), np.zeros(nons2.sum(), dtype=bool)])
        order = np.argsort(keys, kind="stable")
        self.tkeys, self.telem, self.tfac, self.town = keys[order], elem[order], fac[order], isown[order]
        assert np.all(np.diff(self.tkeys) > 0), "every determinant of D + L appears once"
        # S2 partners (flip of the own determinant is another S2 element's own)
        self.s2 = np.where(self.box == 1)[0]
        pe, _ = self._lookup(fh[self.s2], fp[self.s2])
        self.s2_partner = pe
        self.eps = np.diag(Ft)

    # -- helpers ---------------------------------------------------------------
    def _flip(self, so):
        n = self.n
        out = np.where(so == SENT, SENT, np.where(so < n, so + n, so - n))
        return np.sort(out, axis=1)

    def _lookup(self, holes, parts):
        """(element, factor) of determinants, element -1 where not in D + L."""
        keys = _key(holes, parts)
        pos = np.searchsorted(self.tkeys, keys)
        pos = np.minimum(pos, len(self.tkeys) - 1)
        hit = self.tkeys[pos] == keys
        return np.where(hit, self.telem[pos], -1), np.where(hit, self.tfac[pos], 0.0)

    def _lookup_own(self, holes, parts):
        """(element, is its own determinant) of determinants, element -1 where
        not in D + L."""
        keys = _key(holes, parts)
        pos = np.searchsorted(self.tkeys, keys)
        pos = np.minimum(pos, len(self.tkeys) - 1)
        hit = self.tkeys[pos] == keys
        return np.where(hit, self.telem[pos], -1), hit & self.town[pos]

    def _coeff(self, x):
        """Coefficient of each element's own determinant (S2 flip-symmetrised)."""
        c = np.where(self.live, x, 0.0)
        c = c.copy()
        c[self.s2] = 0.5 * (x[self.s2] + self.sg * x[self.s2_partner])
        return c

    def _nbelow(self, v, holes, parts):
        """Occupied spin-orbitals of each determinant below spin-orbital v."""
        n, no = self.n, self.no
        base = np.where(v < n, np.minimum(v, no), no + np.minimum(v - n, no))
        return base - (holes < v[:, None]).sum(axis=1) + (parts < v[:, None]).sum(axis=1)

    # -- the operator ----------------------------------------------------------
    def sigma(self, x):
        n, no = self.n, self.no
        F = self.Ft
        c = self._coeff(x)
        H, P = self.holes, self.parts
        y = (self.diagonal_raw()) * c

        def add(rows, hn, pn, u, v):
            """y[rows] += f_uv eps c(D') for D' = (hn, pn), u removed, v added."""
            hs, ps = np.sort(hn, axis=1), np.sort(pn, axis=1)
            e, f = self._lookup(hs, ps)
            ok = e >= 0
            if not ok.any():
                return
            r, u, v, e, f = rows[ok], u[ok], v[ok], e[ok], f[ok]
            H0, P0 = H[r], P[r]
            eps = self._nbelow(v, H0, P0) - (u < v) + self._nbelow(u, H0, P0)
            sgn = np.where(eps % 2 == 0, 1.0, -1.0)
            val = F[u % n, v % n] * sgn * f * c[e]
            np.add.at(y, r, val)

        rows_all = np.where(self.live)[0]
        for j in range(3):
            # hole j refilled, occupied m (same spin, not a hole) emptied
            rows = rows_all[H[rows_all, j] != SENT]
            hj = H[rows, j]
            spin = hj // n
            for m in range(no):
                mm = spin * n + m
                ok = ~(H[rows] == mm[:, None]).any(axis=1)
                r = rows[ok]
                hn = H[r].copy()
                hn[:, j] = mm[ok]
                add(r, hn, P[r], mm[ok], hj[ok])
            # particle j replaced by virtual e (same spin, not a particle)
            rows = rows_all[P[rows_all, j] != SENT]
            pj = P[rows, j]
            spin = pj // n
            for a in range(self.nv):
                ee = spin * n + no + a
                ok = ~(P[rows] == ee[:, None]).any(axis=1)
                r = rows[ok]
                pn = P[r].copy()
                pn[:, j] = ee[ok]
                add(r, H[r], pn, pj[ok], ee[ok])
            # triples: particle j de-excited into a hole of the same spin
            for i in range(3):
                rows = rows_all[self.triple[rows_all]]
                pj, hi = P[rows, j], H[rows, i]
                ok = (pj // n) == (hi // n)
                r = rows[ok]
                hn, pn = H[r].copy(), P[r].copy()
                hn[:, i] = SENT
                pn[:, j] = SENT
                add(r, hn, pn, pj[ok], hi[ok])
        # doubles <- triples: the transpose of the de-excitations above (F is
        # symmetric), scattered from both determinants of every live triple
        # element onto the own determinants of the doubles
        rows_t = rows_all[self.triple[rows_all]]
        for flip in (False, True):
            Ht = self._flip(H[rows_t]) if flip else H[rows_t]
            Pt = self._flip(P[rows_t]) if flip else P[rows_t]
            ct = (self.sg if flip else 1.0) * c[rows_t]
            for j in range(3):
                for i in range(3):
                    pj, hi = Pt[:, j], Ht[:, i]
                    ok = (pj // n) == (hi // n)
                    hn, pn = Ht[ok].copy(), Pt[ok].copy()
                    hn[:, i] = SENT
                    pn[:, j] = SENT
                    e, own = self._lookup_own(np.sort(hn, axis=1), np.sort(pn, axis=1))
                    hit = (e >= 0) & own
                    u, v = pj[ok][hit], hi[ok][hit]
                    eps = self._nbelow(v, Ht[ok][hit], Pt[ok][hit]) - (u < v) + self._nbelow(u, Ht[ok][hit], Pt[ok][hit])
                    sgn = np.where(eps % 2 == 0, 1.0, -1.0)
                    np.add.at(y, e[hit], F[u % n, v % n] * sgn * ct[ok][hit])
        return np.where(self.live, y, 0.0)

    def diagonal_raw(self):
        """<D0|F|D0> - E0 = sum of particle orbital energies - holes - omega."""
        n = self.n
        eh = np.where(self.holes == SENT, 0.0, self.eps[np.minimum(self.holes, 2 * n - 1) % n])
        ep = np.where(self.parts == SENT, 0.0, self.eps[np.minimum(self.parts, 2 * n - 1) % n])
        return ep.sum(axis=1) - eh.sum(axis=1) - self.omega

    def diagonal(self):
        """Jacobi preconditioner (1 on masked slots, which stay zero)."""
        return np.where(self.live, self.diagonal_raw(), 1.0)

    def dot(self, x, y):
        return float(np.sum(self.w * x * y))

    # -- right-hand side and the S-triple energy --------------------------------
    def rhs(self):
        """b = <D0|H|Psi0> per element (canonical phase), from the one-TOP
        right-hand side of each relabelled problem (operator-string phase)."""
        b = np.zeros(self.dim)
        for s in range(self.k):
            Ft, Bt, lam = relabel_problem(self.Ft, self.Bt, self.lam, self.no, s) if s else (self.Ft, self.Bt, self.lam)
            bs = structured.RHS(Ft, Bt, lam, self.no, spin=self.spin).rhs()
            sel = np.where(self.set == s)[0]
            src = bs if s == 0 else bs[len(bs) - len(sel):]
            b[sel] = self.phase[sel] * src
        return np.where(self.live, b, 0.0)

    def e2_s(self, b=None):
        b = self.rhs() if b is None else b
        e = structured.RHS(self.Ft, self.Bt, self.lam, self.no, spin=self.spin).e2_s()
        extra = self.live & self.triple & (self.set > 0)
        return e + float(np.sum(2.0 * b[extra] ** 2 / self.diagonal_raw()[extra]))

    def solve(self, tol=1e-10, max_iter=400):
        b = self.rhs()
        x, r, it, rel = structured.pcg(self, b, tol=tol, max_iter=max_iter)
        e2_dl = self.dot(b, x) - self.dot(x, r)
        e2_s = self.e2_s(b)
        return dict(e2=e2_dl + e2_s, e2_dl=e2_dl, e2_s=e2_s, e0=self.E0, iters=it, rel=rel, x=x, b=b)

    def determinants(self):
        """Bit string of every element's own determinant (the oracle's fermion
        convention), for comparisons with the explicit construction."""
        out = []
        for h, p in zip(self.holes, self.parts):
            d = self.phi
            for v in h:
                if v != SENT:
                    d ^= 1 << int(v)
            for v in p:
                if v != SENT:
                    d |= 1 << int(v)
            out.append(d)
        return out
