"""Seeded synthetic ESMF-shaped inputs.

This module only draws random numbers.  It holds none of the method's
arithmetic and is the one piece shared by the CPU oracle and the GPU path:
both read the same arrays, produced here from a seed.

Recipe (one dominant hole/particle transition, like the single-CSF-dominated
excited states the paper studies; see the paper's discussion of
single-configuration-dominated excitations):

  rng = numpy.random.default_rng(seed), drawing in this order
  1. occupied orbital energies  ~ U[-1.5, -0.3], sorted ascending
  2. virtual orbital energies   ~ U[ 0.1,  3.0], sorted ascending
  3. E ~ N(0, 1e-3^2) (N x N);  F = diag(eps) + triu(E,1) + triu(E,1)^T
  4. G ~ N(0, 1)     (n_aux x N x N);  B = 0.05 (G + G^T_pq) / 2
  5. C0 ~ N(0, 1)    (n_occ x n_vir);  C0[h, p] = 0;
     C = C0 * sqrt(0.05 / ||C0||^2);   C[h, p] = sqrt(0.95)
  with h = n_occ - 1 (HOMO) and p = 0 (LUMO), so ||C||_F = 1.

Two-electron integrals are (pq|rs) = sum_Q B[Q,p,q] B[Q,r,s].
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Problem:
    n_occ: int
    n_vir: int
    n_aux: int
    F: np.ndarray      # (N, N) symmetric, float64
    B: np.ndarray      # (n_aux, N, N), symmetric in the last two indices
    C: np.ndarray      # (n_occ, n_vir), Frobenius norm 1
    seed: object = None

    @property
    def n(self) -> int:
        return self.n_occ + self.n_vir


def make_problem(n_occ: int, n_vir: int, n_aux: int, seed, *, dominant=(None, 0),
                 fock_noise: float = 1e-3, b_scale: float = 0.05,
                 pair_weight: float = 0.95) -> Problem:
    """Draw one synthetic problem with the recipe in the module docstring."""
    if n_vir < n_occ:
        raise ValueError("the transition-orbital-pair basis needs n_vir >= n_occ")
    rng = np.random.default_rng(seed)
    n = n_occ + n_vir
    eps_o = np.sort(rng.uniform(-1.5, -0.3, n_occ))
    eps_v = np.sort(rng.uniform(0.1, 3.0, n_vir))
    E = rng.normal(0.0, fock_noise, (n, n))
    up = np.triu(E, 1)
    F = np.diag(np.concatenate([eps_o, eps_v])) + up + up.T
    G = rng.normal(0.0, 1.0, (n_aux, n, n))
    B = b_scale * (G + G.transpose(0, 2, 1)) / 2.0
    del G
    C0 = rng.normal(0.0, 1.0, (n_occ, n_vir))
    h = n_occ - 1 if dominant[0] is None else dominant[0]
    p = dominant[1]
    C0[h, p] = 0.0
    C = C0 * np.sqrt((1.0 - pair_weight) / np.sum(C0 * C0))
    C[h, p] = np.sqrt(pair_weight)
    return Problem(n_occ, n_vir, n_aux, F, B, C, seed)


# The five workloads: (n_occ, n_vir, n_aux, seed).
CONFIGS = {
    "c1": (4, 16, 48, 0),        # tiny: explicit determinant oracle in seconds
    "c2": (10, 100, 300, 1),     # FP64 Krylov solve
    "c3": (16, 160, 480, 2),     # FP64 vs mixed precision (the timed workload)
    "c5": (8, 80, 240, 4),       # differentiation workload
}


def config_problem(name: str) -> Problem:
    n_o, n_v, n_aux, seed = CONFIGS[name]
    return make_problem(n_o, n_v, n_aux, seed)


def batched_sizes():
    """The 32 uneven states of the batched workload: (n_occ, n_vir, n_aux, seed)."""
    rng = np.random.default_rng(3)
    out = []
    for s in range(32):
        n_o = int(rng.integers(6, 13))
        n_v = int(rng.integers(60, 121))
        out.append((n_o, n_v, 3 * n_v, [3, s]))
    return out


def random_amplitudes(n: int, seed) -> np.ndarray:
    """A seeded random vector (for operator-action parity tests)."""
    return np.random.default_rng(seed).standard_normal(n)


def make_canonical_problem(n_occ: int, n_vir: int, n_aux: int, seed, fock_noise: float = 1e-3,
                           b_scale: float = 0.05, pair_weight: float = 0.95) -> Problem:
    """A problem already expressed in its own TOP basis (random draws only).

    C = [diag(lambda), 0] with lambda descending (lambda_0^2 = pair_weight),
    and the Fock block of the virtuals beyond n_occ (the AVOs) diagonal and
    ascending, so the TOP rotation of this input is the identity.  Used to
    compare amplitude-level quantities element by element.
    """
    rng = np.random.default_rng(seed)
    n = n_occ + n_vir
    eps_o = np.sort(rng.uniform(-1.5, -0.3, n_occ))[::-1].copy()   # HOMO-like first
    eps_v = np.sort(rng.uniform(0.1, 3.0, n_vir))
    E = rng.normal(0.0, fock_noise, (n, n))
    up = np.triu(E, 1)
    F = np.diag(np.concatenate([eps_o, eps_v])) + up + up.T
    avo = np.arange(2 * n_occ, n)
    F[np.ix_(avo, avo)] = np.diag(eps_v[n_occ:])
    G = rng.normal(0.0, 1.0, (n_aux, n, n))
    B = b_scale * (G + G.transpose(0, 2, 1)) / 2.0
    rest = np.sort(rng.uniform(0.05, 1.0, n_occ - 1))[::-1]
    rest *= np.sqrt((1.0 - pair_weight) / np.sum(rest * rest))
    lam = np.concatenate([[np.sqrt(pair_weight)], rest])
    C = np.zeros((n_occ, n_vir))
    C[np.arange(n_occ), np.arange(n_occ)] = lam
    return Problem(n_occ, n_vir, n_aux, F, B, C, seed)
