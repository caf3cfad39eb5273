"""Tier 1 of the oracle: ESMP2 with the modified H0 built as an explicit matrix.

Test infrastructure (see the package docstring).  Everything here is the
definition written out on Slater determinants (tiny sizes only):

* reference (Sec. II.A, Eqs. for the ESMF ansatz and its TOP form):
  Psi0 = sum_l c_l (a+_{l' up} a_{l up} + a+_{l' dn} a_{l dn}) |Phi>,
  c_l = lambda_l / sqrt(2)  (singlet; the 1/sqrt(2) normalises Psi0 when
  ||C||_F = 1 -- the paper's equation omits it);
* first-order space (Sec. II.B, Eq. for Psi1): all M_s = 0 double and triple
  excitations of the closed shell Phi; no singles, no quadruples;
* triple classes (Sec. II.B triples matrix element, Sec. II.C): a triple
  "contains TOP l" when spatial occupied l is among its holes and spatial
  virtual l' among its particles (any spins).  L = contains a large TOP,
  S = contains some TOP but no large one, N = contains none;
* zeroth-order Hamiltonian (Sec. II.C, the original H0 and its modified
  Q F Q block): on D + L the full Fock operator, on S + N its diagonal.
  The Fock operator F is the given matrix (the Fock operator of the
  reference's one-body density), E0 = <Psi0|F|Psi0>;
* Hamiltonian: one-body part h = F - G[gamma] with gamma the spin-summed
  one-body density of Psi0 and G[g]_pq = sum_rs g_rs ((pq|rs) - (ps|rq)/2),
  two-body part (pq|rs);
* first-order equation Q(H0 - E0)Q Psi1 = -Q V Psi0 with Q V Psi0 = Q H Psi0,
  and E2 = <Psi0|V|Psi1> = sum_mu b_mu x_mu; S-triples are inverted
  directly (their block is diagonal), N-triples have b = 0.

``solve_original`` is the unmodified zeroth-order Hamiltonian of Sec. II.C
(Eq. for the original H0, the N^7 theory the paper starts from): the full
Fock operator on every double and triple, S and N triples included, so that
the E2 shift of the modification can be measured at tiny sizes.
"""
from __future__ import annotations

from itertools import combinations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fermion as fm


class ExplicitESMP2:
    def __init__(self, f, eri, lam, n_occ, n_top=1, rule="spatial", sign=+1):
        f = np.asarray(f, dtype=np.float64)
        self.f, self.eri = f, eri
        self.n = n = f.shape[0]
        self.n_occ = n_occ
        self.n_vir = n - n_occ
        self.lam = np.asarray(lam, dtype=np.float64)
        self.large = set(range(n_top))
        self.rule = rule
        self.c = self.lam / np.sqrt(2.0)
        # closed shell: alpha 0..n_occ-1 and beta n..n+n_occ-1
        self.phi = sum(1 << p for p in range(n_occ)) | sum(1 << (n + p) for p in range(n_occ))
        self.psi0 = {}
        for l in range(n_occ):
            for spin, sgn in ((0, 1.0), (1, float(sign))):
                r = fm.apply_string(self.phi, [("c", spin * n + n_occ + l), ("a", spin * n + l)])
                s, d = r
                self.psi0[d] = self.psi0.get(d, 0.0) + sgn * s * self.c[l]
        # spin-summed one-body density (diagonal in the TOP basis)
        gam = np.zeros((n, n))
        for l in range(n_occ):
            gam[l, l] = 2.0 - self.lam[l] ** 2 if l < len(self.lam) else 2.0
            gam[n_occ + l, n_occ + l] = self.lam[l] ** 2
        self.gamma = gam
        G = np.einsum("rs,pqrs->pq", gam, eri) - 0.5 * np.einsum("rs,psrq->pq", gam, eri)
        self.h = f - G
        fpsi = fm.apply_one_body(self.psi0, f, n)
        self.E0 = sum(c * fpsi.get(d, 0.0) for d, c in self.psi0.items())
        self._enumerate()

    # ----- space -------------------------------------------------------
    def spatial_class(self, det):
        n, no = self.n, self.n_occ
        holes = [p for p in range(2 * n) if ((self.phi >> p) & 1) and not ((det >> p) & 1)]
        parts = [p for p in range(2 * n) if ((det >> p) & 1) and not ((self.phi >> p) & 1)]
        if self.rule == "spatial":
            sh = {p % n for p in holes}
            sv = {p % n - no for p in parts}
            tops = sh & sv
        else:  # same-spin rule, kept only as an alternative reading
            tops = set()
            for p in holes:
                spin, i = divmod(p, n)
                if (spin * n + no + i) in parts:
                    tops.add(i)
        return tops

    def _enumerate(self):
        n, no = self.n, self.n_occ
        occ_a = list(range(no))
        occ_b = [n + i for i in range(no)]
        vir_a = list(range(no, n))
        vir_b = [n + a for a in range(no, n)]
        self.D, self.L, self.S, self.N = [], [], [], []
        for level in (2, 3):
            for nu in range(level + 1):
                nd = level - nu
                for ha in combinations(occ_a, nu):
                    for hb in combinations(occ_b, nd):
                        for pa in combinations(vir_a, nu):
                            for pb in combinations(vir_b, nd):
                                d = self.phi
                                for p in ha + hb:
                                    d ^= 1 << p
                                for p in pa + pb:
                                    d |= 1 << p
                                if level == 2:
                                    self.D.append(d)
                                    continue
                                tops = self.spatial_class(d)
                                if tops & self.large:
                                    self.L.append(d)
                                elif tops:
                                    self.S.append(d)
                                else:
                                    self.N.append(d)
        self.DL = self.D + self.L
        self.index = {d: k for k, d in enumerate(self.DL)}

    def diag_fock(self, det):
        n = self.n
        return sum(self.f[p % n, p % n] for p in range(2 * n) if (det >> p) & 1)

    # ----- operators ---------------------------------------------------
    def fock_matrix(self):
        """Sparse matrix <mu|F|nu> - E0 delta on D + L."""
        rows, cols, vals = [], [], []
        for k, d in enumerate(self.DL):
            out = fm.apply_one_body({d: 1.0}, self.f, self.n)
            for d2, v in out.items():
                j = self.index.get(d2)
                if j is not None and v != 0.0:
                    rows.append(j)
                    cols.append(k)
                    vals.append(v)
        m = len(self.DL)
        A = sp.csr_matrix((vals, (rows, cols)), shape=(m, m))
        return (A - self.E0 * sp.identity(m, format="csr")).tocsr()

    def h_psi0(self):
        """H|Psi0> as {det: coefficient}."""
        one = fm.apply_one_body(self.psi0, self.h, self.n)
        two = fm.apply_two_body(self.psi0, self.eri, self.n)
        for d, v in two.items():
            one[d] = one.get(d, 0.0) + v
        return one

    # ----- solve -------------------------------------------------------
    def solve(self, dense=None):
        hp = self.h_psi0()
        b = np.array([hp.get(d, 0.0) for d in self.DL])
        bS = np.array([hp.get(d, 0.0) for d in self.S])
        bN = np.array([hp.get(d, 0.0) for d in self.N])
        DS = np.array([self.diag_fock(d) - self.E0 for d in self.S])
        A = self.fock_matrix()
        if dense is None:
            dense = A.shape[0] <= 3000
        if dense:
            x = np.linalg.solve(A.toarray(), -b)
        else:
            # SciPy's conjugate gradient to round-off (a sparse LU fills in badly here)
            x, info = spla.cg(A, -b, rtol=1e-15, atol=0.0, maxiter=5000)
            res = np.linalg.norm(A @ x + b) / np.linalg.norm(b)
            if res > 1e-12:
                raise RuntimeError(f"explicit solve did not converge: {res}")
        e2_dl = float(b @ x)
        e2_s = float(-np.sum(bS * bS / DS)) if len(bS) else 0.0
        self.b, self.x, self.A = b, x, A
        self.bS, self.DS = bS, DS
        return dict(e2=e2_dl + e2_s, e2_dl=e2_dl, e2_s=e2_s, e0=self.E0,
                    max_bN=float(np.max(np.abs(bN))) if len(bN) else 0.0)

    def solve_original(self):
        """E2 with the original Q F Q: the full Fock operator coupling all
        doubles and triples (D, L, S, N), no diagonal blocks.  The first-order
        space stays doubles + triples (reading: the original theory is the
        modified one with the S/N diagonal approximation removed)."""
        space = self.D + self.L + self.S + self.N
        index = {d: k for k, d in enumerate(space)}
        rows, cols, vals = [], [], []
        for k, d in enumerate(space):
            out = fm.apply_one_body({d: 1.0}, self.f, self.n)
            for d2, v in out.items():
                j = index.get(d2)
                if j is not None and v != 0.0:
                    rows.append(j)
                    cols.append(k)
                    vals.append(v)
        m = len(space)
        A = (sp.csr_matrix((vals, (rows, cols)), shape=(m, m)) - self.E0 * sp.identity(m, format="csr")).toarray()
        hp = self.h_psi0()
        b = np.array([hp.get(d, 0.0) for d in space])
        x = np.linalg.solve(A, -b)
        return dict(e2=float(b @ x), e0=self.E0, dim=m)

    # ----- spin ---------------------------------------------------------
    def s_plus(self, vec):
        """S+ = sum_p a+_{p up} a_{p dn} applied to {det: c}."""
        n = self.n
        out = {}
        for d, c in vec.items():
            for p in range(n):
                r = fm.apply_string(d, [("c", p), ("a", n + p)])
                if r is None:
                    continue
                s, d2 = r
                out[d2] = out.get(d2, 0.0) + s * c
        return out


def from_problem(prob, n_top=1, rule="spatial"):
    """Rotate a synthetic problem to the TOP basis and build tier 1."""
    from .topbasis import top_rotation, rotate, eri_from_factor
    lam, R = top_rotation(prob.F, prob.C, prob.n_occ)
    Ft, Bt = rotate(prob.F, prob.B, R)
    return ExplicitESMP2(Ft, eri_from_factor(Bt), lam, prob.n_occ, n_top=n_top, rule=rule)
