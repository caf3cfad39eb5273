// Seven-box amplitudes -> determinant coefficients of the first-order wave
// function (paper Sec. II.B, the expansion of Psi1 over doubles and triples of
// the closed shell, the same-spin pairs and their spin-flip partners written
// out).  Every stored amplitude is the excitation-operator string listed with
// the layout in esmp2.h, acting on |Phi>; its determinant and the flip of
// every spin are written in the canonical phase: spin-orbitals ordered alpha
// string first, then beta, each ascending (alpha p -> p, beta p -> N + p,
// virtual a -> spatial n_occ + a).
#include "common.h"
#include "sigma.h"

namespace esmp2 {

struct Op {
  int create;   // 1: creation, 0: annihilation
  int spin;     // 0 alpha, 1 beta
  int orb;      // spatial orbital (virtuals shifted by n_occ)
};

// Phase of the operator string ops[0..n) (rightmost acts first) applied to the
// closed shell, and the excitation's holes and particles as spin-orbitals.
// Occupation below a spin-orbital p = closed-shell count below p, corrected
// by the toggles made so far.
__device__ inline int apply_ops(const Op* ops, int n, int no, int N, bool flip, int* holes, int& nh, int* parts,
                                int& np) {
  int sign = 1;
  int tog[6], ntog = 0, tsgn[6];   // toggled spin-orbitals: +1 added particle, -1 removed hole
  nh = 0; np = 0;
  for (int k = n - 1; k >= 0; --k) {
    const int sp = flip ? 1 - ops[k].spin : ops[k].spin;
    const int p = sp * N + ops[k].orb;
    int below = p < N ? min(p, no) : no + min(p - N, no);
    for (int t = 0; t < ntog; ++t)
      if (tog[t] < p) below += tsgn[t];
    if (below & 1) sign = -sign;
    tog[ntog] = p;
    tsgn[ntog] = ops[k].create ? 1 : -1;
    ++ntog;
    if (ops[k].create) parts[np++] = p;
    else holes[nh++] = p;
  }
  return sign;
}

__device__ inline void sort_small(int* v, int n) {
  for (int i = 1; i < n; ++i)
    for (int j = i; j > 0 && v[j - 1] > v[j]; --j) { const int t = v[j]; v[j] = v[j - 1]; v[j - 1] = t; }
}

// key: holes (ascending) in bits 0-29, particles in bits 30-59, 10 bits per
// spin-orbital, unused slots (doubles) 1023
__device__ inline int64_t det_key(int* holes, int nh, int* parts, int np) {
  sort_small(holes, nh);
  sort_small(parts, np);
  int64_t k = 0;
  for (int s = 0; s < 3; ++s) {
    k |= (int64_t)(s < nh ? holes[s] : 1023) << (10 * s);
    k |= (int64_t)(s < np ? parts[s] : 1023) << (30 + 10 * s);
  }
  return k;
}

// Operator string of stored amplitude g (layout of esmp2.h); returns its
// length.  *partner receives the S2 flip partner's index (S2 only).
__device__ inline int amp_ops(const Dims& d, int64_t g, int box, int loc, Op* ops, int64_t* partner) {
  const int no = d.no, nv = d.nv;
  auto V = [&](int a) { return no + a; };
  const int t = 0, tp = 0;
  switch (box) {
    case B_T2: {
      int i, j, a, b;
      tri_pq(loc / d.npv, no, i, j);
      tri_pq(loc % d.npv, nv, a, b);
      ops[0] = {1, 0, V(a)}; ops[1] = {1, 0, V(b)}; ops[2] = {0, 0, j}; ops[3] = {0, 0, i};
      return 4;
    }
    case B_S2: {
      int r = loc;
      const int b = r % nv; r /= nv;
      const int a = r % nv; r /= nv;
      const int j = r % no, i = r / no;
      ops[0] = {1, 0, V(a)}; ops[1] = {1, 1, V(b)}; ops[2] = {0, 1, j}; ops[3] = {0, 0, i};
      *partner = d.off[B_S2] + (((int64_t)j * no + i) * nv + b) * nv + a;
      return 4;
    }
    case B_T3: {
      int j, k, b, c;
      tri_pq(loc / d.npv1, no - 1, j, k);
      tri_pq(loc % d.npv1, nv - 1, b, c);
      ++j; ++k; ++b; ++c;
      ops[0] = {1, 0, V(tp)}; ops[1] = {1, 0, V(b)}; ops[2] = {1, 0, V(c)};
      ops[3] = {0, 0, k}; ops[4] = {0, 0, j}; ops[5] = {0, 0, t};
      return 6;
    }
    case B_H11: {
      int j, k, b, c;
      tri_pq(loc / d.npv, no, j, k);
      tri_pq(loc % d.npv, nv, b, c);
      ops[0] = {1, 0, V(tp)}; ops[1] = {1, 1, V(b)}; ops[2] = {1, 1, V(c)};
      ops[3] = {0, 1, k}; ops[4] = {0, 1, j}; ops[5] = {0, 0, t};
      return 6;
    }
    case B_H12: {
      const int m1 = nv - 1;
      int j, k;
      tri_pq(loc / (m1 * m1), no, j, k);
      const int a = (loc % (m1 * m1)) / m1 + 1, c = loc % m1 + 1;
      ops[0] = {1, 0, V(a)}; ops[1] = {1, 1, V(tp)}; ops[2] = {1, 1, V(c)};
      ops[3] = {0, 1, k}; ops[4] = {0, 1, j}; ops[5] = {0, 0, t};
      return 6;
    }
    case B_H21: {
      const int o = loc / d.npv;
      const int i = o / (no - 1) + 1, k = o % (no - 1) + 1;
      int b, c;
      tri_pq(loc % d.npv, nv, b, c);
      ops[0] = {1, 0, V(tp)}; ops[1] = {1, 1, V(b)}; ops[2] = {1, 1, V(c)};
      ops[3] = {0, 1, k}; ops[4] = {0, 1, t}; ops[5] = {0, 0, i};
      return 6;
    }
    default: {
      const int m1 = nv - 1;
      const int o = loc / (m1 * m1);
      const int i = o / (no - 1) + 1, k = o % (no - 1) + 1;
      const int a = (loc % (m1 * m1)) / m1 + 1, c = loc % m1 + 1;
      ops[0] = {1, 0, V(a)}; ops[1] = {1, 1, V(tp)}; ops[2] = {1, 1, V(c)};
      ops[3] = {0, 1, k}; ops[4] = {0, 1, t}; ops[5] = {0, 0, i};
      return 6;
    }
  }
}

// One thread per stored amplitude g.  Output order: the determinant of every
// stored amplitude in layout order (entries 0 .. n_amp-1), then the spin-flip
// partner of every amplitude outside S2 in layout order.  S2 holds both
// members of each flip pair, so its determinants appear once; its amplitudes
// enter flip-symmetrised, (x_g + sg x_partner) / 2.
__global__ __launch_bounds__(256) void k_export_dets(Dims d, const double* x, double* coeff, int64_t* key) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t namp = d.off[7];
  if (g >= namp) return;
  int k = 0;
  while (k < 6 && g >= d.off[k + 1]) ++k;
  const int box = k, loc = (int)(g - d.off[k]);
  Op ops[6];
  int64_t partner = g;
  const int n = amp_ops(d, g, box, loc, ops, &partner);
  const double sg = d.sg;
  int holes[3], parts[3], nh, np;
  const int s0 = apply_ops(ops, n, d.no, d.n, false, holes, nh, parts, np);
  key[g] = det_key(holes, nh, parts, np);
  if (box == B_S2) {
    coeff[g] = s0 * 0.5 * (x[g] + sg * x[partner]);
    return;
  }
  coeff[g] = s0 * x[g];
  const int s1 = apply_ops(ops, n, d.no, d.n, true, holes, nh, parts, np);
  const int64_t f = namp + (g < d.off[B_S2] ? g : g - (d.off[B_S2 + 1] - d.off[B_S2]));
  key[f] = det_key(holes, nh, parts, np);
  coeff[f] = sg * s1 * x[g];
}

}  // namespace esmp2
