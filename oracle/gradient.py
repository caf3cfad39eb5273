"""Derivatives of E2 with respect to the TOP-basis Fock matrix and DF factor.

Test infrastructure.  Plain FP64 numpy on top of ``structured``.

The orbital rotation is held fixed: E2 is taken as a function of the
TOP-basis Fock matrix F~ (symmetric, N x N) and factor B~ (n_aux x N x N,
symmetric in its orbital pair), with the singular values lambda fixed.

E2 = E2_DL + E2_S (paper Sec. II.C-II.D).  E2_DL = -<b, A^-1 b>_W is the
stationary value, at x = -A^-1 b, of the Hylleraas functional

    J(x) = 2 <b, x>_W + <x, A x>_W,        A = (H0 - E0) on D + L,

and E2_S = -sum_S b_S^2 / D_S is the stationary value of
sum_S (2 x_S b_S + x_S^2 D_S) at x_S = -b_S / D_S.  At a stationary point
the derivative of the value is the partial derivative of the functional with
the amplitudes held fixed, so the adjoint of the first-order equation is x
itself (A is symmetric) and no second solve is needed:

    dE2/dtheta = dL/dtheta |_(x, x_S fixed),
    L(theta) = 2 <b(theta), x>_W + <x, A(theta) x>_W
               + sum_S (2 x_S b_S(theta) + x_S^2 D_S(theta)).

With x and x_S fixed, L is linear in F~ (A, D_S, and b through f^Phi) and a
polynomial of degree two in any single entry of B~ (every integral is a
product of two factor entries), so a central difference of L along one
entry is its exact derivative up to rounding, whatever the step.  That is
how this module differentiates: the derivative written as a difference, no
hand-derived adjoint.

Convention for the symmetric arguments: G is the symmetric matrix with
dE2 = sum_pq G[p, q] dF[p, q] for every symmetric perturbation dF (likewise
per auxiliary index for B~).  A step h on the pair (p, q), p != q, moves
both F[p, q] and F[q, p], so G[p, q] = (L(+h) - L(-h)) / (4 h); on the
diagonal G[p, p] = (L(+h) - L(-h)) / (2 h).
"""
from __future__ import annotations

import numpy as np

from .structured import RHS, solve


class Lagrangian:
    """L(F~, B~) with the first-order amplitudes of the point (Ft, Bt) held fixed."""

    def __init__(self, Ft, Bt, lam, n_occ, tol=1e-13, max_iter=500, spin=0):
        self.spin = spin
        self.Ft = np.array(Ft, dtype=np.float64)
        self.Bt = np.array(Bt, dtype=np.float64)
        self.lam = np.asarray(lam, dtype=np.float64)
        self.no = n_occ
        out = solve(self.Ft, self.Bt, self.lam, n_occ, tol=tol, max_iter=max_iter, spin=spin)
        self.x = out["x"]
        self.e2 = out["e2"]
        self.e2_dl, self.e2_s = out["e2_dl"], out["e2_s"]
        rh = RHS(self.Ft, self.Bt, self.lam, n_occ, spin=spin)
        self.xs = [-b / D for b, D in rh.s_terms()]

    def value(self, Ft=None, Bt=None):
        Ft = self.Ft if Ft is None else Ft
        Bt = self.Bt if Bt is None else Bt
        rh = RHS(Ft, Bt, self.lam, self.no, spin=self.spin)
        op, x = rh.op, self.x
        b = rh.rhs()
        val = 2.0 * op.dot(b, x) + op.dot(x, op.sigma(x))
        for xs, (bs, D) in zip(self.xs, rh.s_terms()):
            val += 2.0 * np.sum(2.0 * xs * bs + xs * xs * D)      # x2: spin-flip partner
        return float(val)

    # -- entries of the gradient ---------------------------------------------
    def grad_F(self, p, q, h=1e-3):
        E = np.zeros_like(self.Ft)
        E[p, q] = E[q, p] = h
        d = self.value(Ft=self.Ft + E) - self.value(Ft=self.Ft - E)
        return d / (2.0 * h) / (1.0 if p == q else 2.0)

    def grad_B(self, Q, p, q, h=1e-3):
        E = np.zeros_like(self.Bt)
        E[Q, p, q] = E[Q, q, p] = h
        d = self.value(Bt=self.Bt + E) - self.value(Bt=self.Bt - E)
        return d / (2.0 * h) / (1.0 if p == q else 2.0)

    def full_gradient(self, h=1e-3):
        """Every entry (tiny sizes only): (G_F, G_B)."""
        n = self.Ft.shape[0]
        GF = np.zeros((n, n))
        GB = np.zeros_like(self.Bt)
        for p in range(n):
            for q in range(p, n):
                GF[p, q] = GF[q, p] = self.grad_F(p, q, h)
                for Q in range(self.Bt.shape[0]):
                    GB[Q, p, q] = GB[Q, q, p] = self.grad_B(Q, p, q, h)
        return GF, GB


def e2_of(Ft, Bt, lam, n_occ, tol=1e-13, max_iter=500, spin=0):
    """E2 by a full solve at (Ft, Bt): the function being differentiated."""
    return solve(Ft, Bt, lam, n_occ, tol=tol, max_iter=max_iter, spin=spin)["e2"]
