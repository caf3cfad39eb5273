// Derivatives of E2 with respect to the TOP-basis Fock matrix F~ and DF factor
// B~, with the orbital rotation held fixed (paper Sec. II.C-II.D).
//
// E2_DL = -<b, A^-1 b>_W is the stationary value of the Hylleraas functional
// J(x) = 2 <b, x>_W + <x, A x>_W at x = -A^-1 b.  A = H0 - E0 is symmetric, so
// the adjoint of the first-order equation is the solution x itself and
//   dE2_DL = 2 <x, db>_W + <x, dA x>_W         (x held fixed).
// E2_S = -sum_S b_S^2 / D_S is explicit: per determinant (counted twice, with
// its spin-flip partner) dE2_S = -2 (b/D) db + (b/D)^2 dD.
//
// F~ enters A linearly (Fock blocks, omega, kappa), b through f^Phi_ov, and
// D_S through its diagonal and omega.  B~ enters b through the integral blocks
//   V[(ia),(jb)] = sum_Q Bov[Q][ia] Bov[Q][jb],  M[(ia),(jb)] = sum_Q X[Q][ia] Bov[Q][jb],
//   X[Q][ia] = c_i Bvt[Q][a][i] - c_a Boo[Q][a][i],   and through f^Phi,
// and E2_S through V.  The backward pass:
//   1. the first-order amplitudes as dense per-box tensors (S2 flip-symmetrised);
//   2. <x, dA x> / dF: Gram matrices of the batch matrices (matrix-core GEMMs)
//      for the Fock blocks acting on the free indices, strided contractions for
//      the pinned-row transfers and the f_ov couplings (doubles <-> L-triples,
//      counted twice: the de-excitation terms are their adjoint), squared norms
//      for omega and kappa;
//   3. the transpose of the right-hand-side assembly and of the S-triple energy,
//      scattered into dE/dV, dE/dM, dE/df^Phi (atomic FP64 adds);
//   4. the chain through the integral GEMMs, X and f^Phi to the factor blocks;
//   5. both gradients symmetrised: dE = sum_pq G[p][q] dF[p][q] for symmetric dF.
#include "common.h"
#include "reduce.h"

namespace esmp2 {

// out[o][d1][d0][r] = in[o][d0][d1][r]
__global__ void k_swap_mid(const double* in, double* out, int64_t outer, int d0, int d1, int64_t inner) {
  const int64_t n = outer * d0 * d1 * inner;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e % inner;
    int64_t t = e / inner;
    const int i1 = (int)(t % d1);
    t /= d1;
    const int i0 = (int)(t % d0);
    const int64_t o = t / d0;
    out[((o * d1 + i1) * d0 + i0) * inner + r] = in[e];
  }
}

// G[r * ld + c] += alpha * sum_b tmp[b][r][c]  (nb batches of m x n); the batches are
// split over gridDim.y workgroup rows, each adding its part atomically
__global__ void k_batch_sum_acc(const double* tmp, int nb, int m, int n, double alpha, double* G, int ld) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * n) return;
  const int b0 = (int)((int64_t)nb * blockIdx.y / gridDim.y), b1 = (int)((int64_t)nb * (blockIdx.y + 1) / gridDim.y);
  double s = 0.0;
  for (int b = b0; b < b1; ++b) s += tmp[(int64_t)b * m * n + e];
  unsafeAtomicAdd(&G[(int64_t)(e / n) * ld + e % n], alpha * s);
}

// Strided bilinear contraction:
//   out[e0, e1] = sum_{c0..c3} A[oA + e.aE + c.aC] * B[oB + e.bE + c.bC]
// grid (nE0 * nE1, nsplit): each block a share of the contraction, one partial per block.
struct Contr {
  const double* A;
  const double* B;
  int64_t oA, oB;
  int nE[2];
  int64_t aE[2], bE[2];
  int nC[4];
  int64_t aC[4], bC[4];
};

__global__ __launch_bounds__(256) void k_contract(Contr c, double* part) {
  const int e = blockIdx.x, e0 = e / c.nE[1], e1 = e % c.nE[1];
  const int64_t ncon = (int64_t)c.nC[0] * c.nC[1] * c.nC[2] * c.nC[3];
  const int64_t baseA = c.oA + e0 * c.aE[0] + e1 * c.aE[1];
  const int64_t baseB = c.oB + e0 * c.bE[0] + e1 * c.bE[1];
  double acc = 0.0;
  for (int64_t t = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; t < ncon; t += (int64_t)gridDim.y * blockDim.x) {
    int64_t r = t;
    const int i3 = (int)(r % c.nC[3]); r /= c.nC[3];
    const int i2 = (int)(r % c.nC[2]); r /= c.nC[2];
    const int i1 = (int)(r % c.nC[1]);
    const int i0 = (int)(r / c.nC[1]);
    acc += c.A[baseA + i0 * c.aC[0] + i1 * c.aC[1] + i2 * c.aC[2] + i3 * c.aC[3]] *
           c.B[baseB + i0 * c.bC[0] + i1 * c.bC[1] + i2 * c.bC[2] + i3 * c.bC[3]];
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) part[(int64_t)e * gridDim.y + blockIdx.y] = s;
}

// out[dst + e0 * so0 + e1 * so1] += alpha * sum of the partials of output (e0, e1)
__global__ void k_contract_fin(const double* part, int nE0, int nE1, int nsplit, double alpha, double* out,
                               int64_t dst, int64_t so0, int64_t so1) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nE0 * nE1) return;
  double s = 0.0;
  for (int k = 0; k < nsplit; ++k) s += part[(int64_t)e * nsplit + k];
  out[dst + (e / nE1) * so0 + (e % nE1) * so1] += alpha * s;
}

// partial sums of squares, one per block
__global__ __launch_bounds__(256) void k_sumsq(const double* v, int64_t n, double* part) {
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    acc += v[e] * v[e];
  const double s = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// scal[0] = coefficient of omega in <x, A x>_W (+ S-triples, scal[2]), scal[1] = coefficient of kappa
//   from the squared norms nrm[box] = s_box * |X_box|^2 (partials, nb per box)
// one wavefront
__global__ void k_norm_scalars(const double* part, int nb, const double* sbox, double* scal) {
  double nrm[7];
  for (int k = 0; k < 7; ++k) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += 64) s += part[k * nb + b];
    nrm[k] = sbox[k] * wave_sum(s);
  }
  if (threadIdx.x == 0) {
    scal[0] = -(nrm[B_T2] + nrm[B_S2]);
    scal[1] = nrm[B_T3] + nrm[B_H11] + nrm[B_H12] + nrm[B_H21] + nrm[B_H22];
  }
}

// ---------------------------------------------------------------------------
// Transpose of the right-hand-side assembly: for each amplitude mu, the
// factor 2 W_mu x_mu times each coefficient of b_mu goes to the integral or
// f^Phi element that coefficient multiplies.
// ---------------------------------------------------------------------------
struct RhsAdjArgs {
  Dims d;
  const double* x;
  const double* lam;
  double* GV;     // dE/dV[(ia),(jb)]
  double* GM;     // dE/dM[(ia),(jb)]
  double* Gf;     // dE/df^Phi[j][b]
};

__global__ void k_rhs_adj(RhsAdjArgs A) {
  const Dims& d = A.d;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= d.off[7]) return;
  int loc;
  const int box = box_of(d, g, loc);        // 32-bit local index (a box holds < 2^31 amplitudes)
  const int no = d.no, nv = d.nv, nov = no * nv;
  const double s2 = 0.70710678118654752440;
  auto c = [&](int l) -> double { return A.lam[l] * s2; };
  auto addV = [&](int i, int a, int j, int b, double v) {
    unsafeAtomicAdd(&A.GV[(int64_t)(i * nv + a) * nov + j * nv + b], v);
  };
  auto addm = [&](int i, int j, int a, int b, double v) {
    unsafeAtomicAdd(&A.GM[(int64_t)(i * nv + a) * nov + j * nv + b], v);
    if (a == i) unsafeAtomicAdd(&A.Gf[j * nv + b], c(i) * v);
  };
  auto addE = [&](int k, int x, double v) {      // E(k, x) = V(0,0,k,x) - V(k,0,0,x)
    addV(0, 0, k, x, v);
    addV(k, 0, 0, x, -v);
  };
  const double w = (box == B_S2) ? 1.0 : 2.0;
  const double cf = 2.0 * w * A.x[g];
  if (cf == 0.0) return;
  const double c0 = c(0);
  const double sg = (double)d.sg;        // beta singles' terms carry sg
  switch (box) {
    case B_T2: {
      int po = loc / d.npv, pv = loc % d.npv, i, j, a, b;
      tri_pq(po, no, i, j); tri_pq(pv, nv, a, b);
      addm(i, j, a, b, cf); addm(j, i, a, b, -cf); addm(i, j, b, a, -cf); addm(j, i, b, a, cf);
      break;
    }
    case B_S2: {
      int i = loc / (nov * nv), r = loc % (nov * nv);
      int j = r / (nv * nv); r %= nv * nv;
      int a = r / nv, b = r % nv;
      addm(i, j, a, b, cf); addm(j, i, b, a, sg * cf);
      break;
    }
    case B_T3: {
      int po = loc / d.npv1, pv = loc % d.npv1, j, k, b, cc;
      tri_pq(po, no - 1, j, k); tri_pq(pv, nv - 1, b, cc);
      ++j; ++k; ++b; ++cc;
      addV(j, b, k, cc, c0 * cf); addV(k, b, j, cc, -c0 * cf);
      if (b == j) addE(k, cc, c(j) * cf);
      if (b == k) addE(j, cc, -c(k) * cf);
      if (cc == j) addE(k, b, -c(j) * cf);
      if (cc == k) addE(j, b, c(k) * cf);
      break;
    }
    case B_H11: {
      int po = loc / d.npv, pv = loc % d.npv, j, k, b, cc;
      tri_pq(po, no, j, k); tri_pq(pv, nv, b, cc);
      addV(j, b, k, cc, c0 * cf); addV(k, b, j, cc, -c0 * cf);
      if (b == j) addV(0, 0, k, cc, sg * c(j) * cf);
      if (b == k) addV(0, 0, j, cc, -sg * c(k) * cf);
      if (cc == j) addV(0, 0, k, b, -sg * c(j) * cf);
      if (cc == k) addV(0, 0, j, b, sg * c(k) * cf);
      break;
    }
    case B_H12: {
      const int m1 = nv - 1;
      int po = loc / (m1 * m1), r = loc % (m1 * m1), j, k;
      tri_pq(po, no, j, k);
      const int a = r / m1 + 1, cc = r % m1 + 1;
      const double sf = sg * cf;
      if (j == 0) addV(0, a, k, cc, c0 * sf);
      if (cc == j) addV(0, a, k, 0, -c(j) * sf);
      if (k == 0) addV(0, a, j, cc, -c0 * sf);
      if (cc == k) addV(0, a, j, 0, c(k) * sf);
      break;
    }
    case B_H21: {
      int o = loc / d.npv, pv = loc % d.npv, b, cc;
      const int i = o / (no - 1) + 1, k = o % (no - 1) + 1;
      tri_pq(pv, nv, b, cc);
      const double sf = sg * cf;
      if (b == 0) addV(i, 0, k, cc, c0 * sf);
      if (b == k) addV(i, 0, 0, cc, -c(k) * sf);
      if (cc == 0) addV(i, 0, k, b, -c0 * sf);
      if (cc == k) addV(i, 0, 0, b, c(k) * sf);
      break;
    }
    default: {  // B_H22
      const int m1 = nv - 1;
      const int o = loc / (m1 * m1), r = loc % (m1 * m1);
      const int i = o / (no - 1) + 1, k = o % (no - 1) + 1;
      const int a = r / m1 + 1, cc = r % m1 + 1;
      if (a == i) addE(k, cc, c(i) * cf);
      addV(i, a, k, cc, sg * c0 * cf);
      if (cc == k) addV(i, a, 0, 0, sg * c(k) * cf);
      break;
    }
  }
}

// ---------------------------------------------------------------------------
// Transpose of the S-triple energy: per determinant (counted twice) with
// b = sum_t coef_t V_t and D = sum particle - sum hole energies - omega,
//   dE/dV_t += -4 (b/D) coef_t,   dE/dev[p] += 2 (b/D)^2, dE/deo[h] -= 2 (b/D)^2, dE/domega -= 2 (b/D)^2.
// The orbital-energy and omega parts are summed in LDS per block first.
// ---------------------------------------------------------------------------
struct E2sAdjArgs {
  Dims d;
  const double* V; const double* lam; const double* eo; const double* ev;
  double omega;
  const int *pv, *pv1, *po, *po1;
  double* GV;
  double* Gev;      // nv
  double* Geo;      // no
  double* Gom;      // 1
};

// Orbital-energy parts of the S-triple gradient, summed in LDS per workgroup.
// The loops below keep every lane of a wavefront in step (an out-of-range lane
// carries gd = 0), so that wavefront-wide reductions can replace atomics on
// keys that many lanes share:
//   * a key fixed for a whole row of the grid: per-thread registers, one
//     workgroup sum per row;
//   * a key that changes slowly along the lanes: wave_keyed_add (one LDS atomic
//     per distinct key in the wavefront);
//   * a key that differs from lane to lane: a plain LDS atomic.
struct SAcc {
  double* ev;     // LDS, 192
  double* eo;     // LDS, 64
  double* om;     // LDS, 1
};

// acc1[key] += v (and acc2[key] += v2 when acc2 is given) summed over the
// wavefront, one LDS atomic per distinct key.  Every lane of the wavefront
// calls it; a lane with nothing to add passes v = 0 and any valid key.
__device__ inline void wave_keyed_add(double* acc1, double* acc2, int key, double v, double v2) {
  const int lane = threadIdx.x & 63;
  unsigned long long pending = ~0ull;
  while (pending) {
    const int src = __ffsll((long long)pending) - 1;
    const int k0 = __shfl(key, src);
    const bool mine = (key == k0);
    const double s1 = wave_sum(mine ? v : 0.0);
    const double s2 = acc2 ? wave_sum(mine ? v2 : 0.0) : 0.0;
    if (lane == src) {
      atomicAdd(&acc1[k0], s1);
      if (acc2) atomicAdd(&acc2[k0], s2);
    }
    pending &= ~__ballot(mine);
  }
}

// adds the row-fixed registers (particle pf, hole hf, omega) of the workgroup
__device__ inline void s_row_flush(const SAcc& s, int pf, int hf, double& rp, double& rh, double& ro) {
  const double a = block_sum(rp);
  const double b = block_sum(rh);
  const double c = block_sum(ro);
  if (threadIdx.x == 0) {
    s.ev[pf] += a;
    s.eo[hf] += b;
    s.om[0] += c;
  }
  rp = rh = ro = 0.0;
  __syncthreads();
}

__device__ inline void s_flush(const E2sAdjArgs& A, const SAcc& s) {
  __syncthreads();
  for (int e = threadIdx.x; e < A.d.nv; e += blockDim.x) if (s.ev[e] != 0.0) unsafeAtomicAdd(&A.Gev[e], s.ev[e]);
  for (int e = threadIdx.x; e < A.d.no; e += blockDim.x) if (s.eo[e] != 0.0) unsafeAtomicAdd(&A.Geo[e], s.eo[e]);
  if (threadIdx.x == 0 && s.om[0] != 0.0) unsafeAtomicAdd(A.Gom, s.om[0]);
}

#define ESMP2_SACC_DECL                                                   \
  __shared__ double sev[192], seo[64], som[1];                            \
  for (int e = threadIdx.x; e < 192; e += blockDim.x) sev[e] = 0.0;       \
  for (int e = threadIdx.x; e < 64; e += blockDim.x) seo[e] = 0.0;        \
  if (threadIdx.x == 0) som[0] = 0.0;                                     \
  __syncthreads();                                                        \
  const SAcc sacc{sev, seo, som};

__device__ inline void sort3_adj(int& x, int& y, int& z) {
  if (x > y) { int t = x; x = y; y = t; }
  if (y > z) { int t = y; y = z; z = t; }
  if (x > y) { int t = x; x = y; y = t; }
}

// same-spin sector (enumeration of the energy kernel): triples {l, j, k; l', b, c},
// l fixed per grid row
__global__ __launch_bounds__(256) void k_e2s_same_adj(E2sAdjArgs A) {
  ESMP2_SACC_DECL
  const Dims& d = A.d;
  const int no = d.no, nv = d.nv, nov = no * nv;
  const int per_l = d.npo1 * d.npv1;
  const double s2 = 0.70710678118654752440;
  double rp = 0.0, rh = 0.0, ro = 0.0;
  for (int l = 1 + blockIdx.y; l < no; l += gridDim.y) {
    for (int base = blockIdx.x * blockDim.x; base < per_l; base += gridDim.x * blockDim.x) {
      const int r = base + threadIdx.x;
      int j = 0, k = 0, b = 0, c = 0;
      double gd = 0.0;
      if (r < per_l) {
        const int to = A.po1[r / d.npv1], tv = A.pv1[r % d.npv1];
        const int jr = to >> 16, kr = to & 0xffff, br = tv >> 16, cr = tv & 0xffff;
        j = jr + (jr >= l); k = kr + (kr >= l); b = br + (br >= l); c = cr + (cr >= l);
        if (!((j < l && (j == b || j == c)) || (k < l && (k == b || k == c)))) {
          int I[3] = {l, j, k}, P[3] = {l, b, c};
          sort3_adj(I[0], I[1], I[2]);
          sort3_adj(P[0], P[1], P[2]);
          double bv = 0.0;
          for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q) {
              if (P[p] != I[q]) continue;
              const int a1 = P[p == 0 ? 1 : 0], a2 = P[p == 2 ? 1 : 2];
              const int i1 = I[q == 0 ? 1 : 0], i2 = I[q == 2 ? 1 : 2];
              const double anti = A.V[(int64_t)(i1 * nv + a1) * nov + i2 * nv + a2] -
                                  A.V[(int64_t)(i2 * nv + a1) * nov + i1 * nv + a2];
              const double sg = ((p + q) & 1) ? -1.0 : 1.0;
              bv += sg * A.lam[I[q]] * s2 * anti;
            }
          const double D = A.ev[P[0]] + A.ev[P[1]] + A.ev[P[2]] - A.eo[I[0]] - A.eo[I[1]] - A.eo[I[2]] - A.omega;
          const double gb = -4.0 * bv / D;
          gd = 2.0 * (bv / D) * (bv / D);
          for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q) {
              if (P[p] != I[q]) continue;
              const int a1 = P[p == 0 ? 1 : 0], a2 = P[p == 2 ? 1 : 2];
              const int i1 = I[q == 0 ? 1 : 0], i2 = I[q == 2 ? 1 : 2];
              const double sg = ((p + q) & 1) ? -1.0 : 1.0;
              const double v = gb * sg * A.lam[I[q]] * s2;
              unsafeAtomicAdd(&A.GV[(int64_t)(i1 * nv + a1) * nov + i2 * nv + a2], v);
              unsafeAtomicAdd(&A.GV[(int64_t)(i2 * nv + a1) * nov + i1 * nv + a2], -v);
            }
          atomicAdd(&sacc.ev[c], gd);
        }
      }
      // particles {l, b, c}, holes {l, j, k}, omega
      rp += gd; rh -= gd; ro -= gd;
      wave_keyed_add(sacc.ev, nullptr, b, gd, 0.0);
      wave_keyed_add(sacc.eo, nullptr, j, -gd, 0.0);
      wave_keyed_add(sacc.eo, nullptr, k, -gd, 0.0);
    }
    s_row_flush(sacc, l, l, rp, rh, ro);
  }
  s_flush(A, sacc);
}

// mixed sector: b of the energy kernel and the scatter of g * db/dV
__device__ inline double b_mixed_adj(const E2sAdjArgs& A, int i, int a, int j, int k, int b, int c) {
  const int nv = A.d.nv, nov = A.d.no * nv;
  const double s2 = 0.70710678118654752440;
  auto V = [&](int p, int x, int q, int y) { return A.V[(int64_t)(p * nv + x) * nov + q * nv + y]; };
  double bd = 0.0;
  if (b == j) bd += A.lam[j] * s2 * V(i, a, k, c);
  if (b == k) bd -= A.lam[k] * s2 * V(i, a, j, c);
  if (c == j) bd -= A.lam[j] * s2 * V(i, a, k, b);
  if (c == k) bd += A.lam[k] * s2 * V(i, a, j, b);
  double bv = (double)A.d.sg * bd;
  if (a == i) bv += A.lam[i] * s2 * (V(j, b, k, c) - V(k, b, j, c));
  return bv;
}

__device__ inline void scatter_mixed(const E2sAdjArgs& A, int i, int a, int j, int k, int b, int c, double g) {
  const int nv = A.d.nv, nov = A.d.no * nv;
  const double s2 = 0.70710678118654752440;
  auto add = [&](int p, int x, int q, int y, double v) {
    unsafeAtomicAdd(&A.GV[(int64_t)(p * nv + x) * nov + q * nv + y], v);
  };
  if (a == i) { add(j, b, k, c, g * A.lam[i] * s2); add(k, b, j, c, -g * A.lam[i] * s2); }
  g *= (double)A.d.sg;                    // the remaining terms come from the beta singles
  if (b == j) add(i, a, k, c, g * A.lam[j] * s2);
  if (b == k) add(i, a, j, c, -g * A.lam[k] * s2);
  if (c == j) add(i, a, k, b, -g * A.lam[j] * s2);
  if (c == k) add(i, a, j, b, g * A.lam[k] * s2);
}

// mixed sector, case A (a = i >= 1 fixed per grid row)
__global__ __launch_bounds__(256) void k_e2s_mixed_a_adj(E2sAdjArgs A) {
  ESMP2_SACC_DECL
  const Dims& d = A.d;
  const int no = d.no;
  const int per_i = d.npo * d.npv;
  double rp = 0.0, rh = 0.0, ro = 0.0;
  for (int i = 1 + blockIdx.y; i < no; i += gridDim.y) {
    for (int base = blockIdx.x * blockDim.x; base < per_i; base += gridDim.x * blockDim.x) {
      const int r = base + threadIdx.x;
      int j = 0, k = 0, b = 0;
      double gd = 0.0;
      if (r < per_i) {
        const int to = A.po[r / d.npv], tv = A.pv[r % d.npv];
        j = to >> 16; k = to & 0xffff; b = tv >> 16;
        const int c = tv & 0xffff;
        if (!((j == 0 || k == 0) && (b == 0 || c == 0))) {
          const double bv = b_mixed_adj(A, i, i, j, k, b, c);
          const double D = A.ev[i] + A.ev[b] + A.ev[c] - A.eo[i] - A.eo[j] - A.eo[k] - A.omega;
          scatter_mixed(A, i, i, j, k, b, c, -4.0 * bv / D);
          gd = 2.0 * (bv / D) * (bv / D);
          atomicAdd(&sacc.ev[c], gd);
        }
      }
      // particles {i, b, c}, holes {i, j, k}, omega
      rp += gd; rh -= gd; ro -= gd;
      wave_keyed_add(sacc.ev, nullptr, b, gd, 0.0);
      wave_keyed_add(sacc.eo, nullptr, j, -gd, 0.0);
      wave_keyed_add(sacc.eo, nullptr, k, -gd, 0.0);
    }
    s_row_flush(sacc, i, i, rp, rh, ro);
  }
  s_flush(A, sacc);
}

// mixed sector, case B (up excitation i -> a, a != i, fixed per grid row; down pair
// holes {l, m}, particles {l', e})
__global__ __launch_bounds__(256) void k_e2s_mixed_b_adj(E2sAdjArgs A) {
  ESMP2_SACC_DECL
  const Dims& d = A.d;
  const int no = d.no, nv = d.nv;
  const int inner = no * (no - 1) * (nv - 1);
  double rp = 0.0, rh = 0.0, ro = 0.0;
  for (int ia = blockIdx.y; ia < no * nv; ia += gridDim.y) {
    const int i = ia / nv, a = ia - i * nv;
    if (a == i) continue;                                  // uniform over the workgroup
    for (int base = blockIdx.x * blockDim.x; base < inner; base += gridDim.x * blockDim.x) {
      const int r = base + threadIdx.x;
      int l = 0, m = 0;
      double gd = 0.0;
      if (r < inner) {
        const int er = r % (nv - 1), q = r / (nv - 1);
        const int mr = q % (no - 1);
        l = q / (no - 1);
        m = mr + (mr >= l);
        const int e = er + (er >= l);
        if (!(m < l && e == m) && !((i == 0 || l == 0 || m == 0) && (a == 0 || l == 0 || e == 0))) {
          const int j = l < m ? l : m, k = l < m ? m : l;
          const int b = l < e ? l : e, c = l < e ? e : l;
          const double bv = b_mixed_adj(A, i, a, j, k, b, c);
          const double D = A.ev[a] + A.ev[b] + A.ev[c] - A.eo[i] - A.eo[j] - A.eo[k] - A.omega;
          scatter_mixed(A, i, a, j, k, b, c, -4.0 * bv / D);
          gd = 2.0 * (bv / D) * (bv / D);
          atomicAdd(&sacc.ev[e], gd);
        }
      }
      // particles {a, l, e}, holes {i, l, m}, omega
      rp += gd; rh -= gd; ro -= gd;
      wave_keyed_add(sacc.ev, sacc.eo, l, gd, -gd);
      wave_keyed_add(sacc.eo, nullptr, m, -gd, 0.0);
    }
    s_row_flush(sacc, a, i, rp, rh, ro);
  }
  s_flush(A, sacc);
}

// ---------------------------------------------------------------------------
// Chain to the factor blocks
// ---------------------------------------------------------------------------
// X[Q][(i,a)] = c_i Bvt[Q][a][i] - c_a Boo[Q][a][i] (a < n_occ):  dBvt, dBoo from dX
__global__ void k_make_x_adj(const double* dX, const double* lam, int no, int nv, int naux, double* dBvt,
                             double* dBoo) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)naux * no * nv) return;
  const int Q = (int)(e / (no * nv)), r = (int)(e % (no * nv));
  const int i = r / nv, a = r % nv;
  const double s2 = 0.70710678118654752440;
  dBvt[((int64_t)Q * nv + a) * no + i] += lam[i] * s2 * dX[e];       // one (Q, a, i) per thread
  if (a < no) unsafeAtomicAdd(&dBoo[((int64_t)Q * no + a) * no + i], -lam[a] * s2 * dX[e]);
}

// f^Phi_ia = F~_ia - sum_Q [dq_Q Bov_Q[i][a] - 1/2 sum_k w_k Bov_Q[i][k] Bvt_Q[a][k]
//                          + 1/2 sum_k w_k Boo_Q[i][k] Bov_Q[k][a]],
// dq_Q = sum_k w_k (Bvt_Q[k][k] - Boo_Q[k][k]), w_k = lam_k^2.  One block per Q;
// Gf = dE/df^Phi.
__global__ __launch_bounds__(256) void k_fphi_adj(const double* Bov, const double* Bvt, const double* Boo,
                                                  const double* lam, const double* Gf, int no, int nv,
                                                  double* dBov, double* dBvt, double* dBoo) {
  const int Q = blockIdx.x, tid = threadIdx.x;
  const double* bov = Bov + (int64_t)Q * no * nv;
  const double* bvt = Bvt + (int64_t)Q * nv * no;
  const double* boo = Boo + (int64_t)Q * no * no;
  double* gov = dBov + (int64_t)Q * no * nv;
  double* gvt = dBvt + (int64_t)Q * nv * no;
  double* goo = dBoo + (int64_t)Q * no * no;
  __shared__ double sh[2];
  // dq_Q and ddq = dE/ddq_Q = -sum_ia Gf[i][a] Bov_Q[i][a]
  double t = 0.0;
  for (int e = tid; e < no * nv; e += blockDim.x) t += Gf[e] * bov[e];
  t = block_sum(t);
  if (tid == 0) {
    double dq = 0.0;
    for (int k = 0; k < no; ++k) dq += lam[k] * lam[k] * (bvt[k * no + k] - boo[k * no + k]);
    sh[0] = dq;
    sh[1] = -t;
  }
  __syncthreads();
  const double dq = sh[0], ddq = sh[1];
  // dBov[i][a]: -Gf dq; + 1/2 w_a sum_a' Gf[i][a'] Bvt[a'][a] (a < no); - 1/2 w_i sum_i' Gf[i'][a] Boo[i'][i]
  for (int e = tid; e < no * nv; e += blockDim.x) {
    const int i = e / nv, a = e % nv;
    double v = -Gf[e] * dq;
    if (a < no) {
      double s = 0.0;
      for (int ap = 0; ap < nv; ++ap) s += Gf[i * nv + ap] * bvt[ap * no + a];
      v += 0.5 * lam[a] * lam[a] * s;
    }
    double s = 0.0;
    for (int ip = 0; ip < no; ++ip) s += Gf[ip * nv + a] * boo[ip * no + i];
    v -= 0.5 * lam[i] * lam[i] * s;
    gov[e] += v;
  }
  // dBvt[a][k]: + w_k ddq (a == k); + 1/2 w_k sum_i Gf[i][a] Bov[i][k]
  for (int e = tid; e < nv * no; e += blockDim.x) {
    const int a = e / no, k = e % no;
    const double w = lam[k] * lam[k];
    double s = 0.0;
    for (int i = 0; i < no; ++i) s += Gf[i * nv + a] * bov[i * nv + k];
    gvt[e] += 0.5 * w * s + (a == k ? w * ddq : 0.0);
  }
  // dBoo[i][k]: - w_k ddq (i == k); - 1/2 w_k sum_a Gf[i][a] Bov[k][a]
  for (int e = tid; e < no * no; e += blockDim.x) {
    const int i = e / no, k = e % no;
    const double w = lam[k] * lam[k];
    double s = 0.0;
    for (int a = 0; a < nv; ++a) s += Gf[i * nv + a] * bov[k * nv + a];
    goo[e] += -0.5 * w * s - (i == k ? w * ddq : 0.0);
  }
}

// The Fock gradient: the f^Phi part, omega / kappa through the diagonal, the
// S-triple denominators, then symmetrised.  G (n x n, read positions) is
// complete on entry except for these diagonal / ov terms.
//   scal[0] coefficient of omega in <x, A x>, scal[1] of kappa, scal[2] of omega in E2_S
__global__ void k_grad_f_finish(double* G, const double* lam, const double* Gf, const double* Gev,
                                const double* Geo, const double* scal, int no, int nv, double* dF) {
  const int n = no + nv;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int p = e / n, q = e % n;
  auto read = [&](int r, int c) -> double {
    double v = G[r * n + c];
    if (r < no && c >= no) v += Gf[r * nv + (c - no)];
    if (r == c) {
      const double gom = scal[0] + scal[2] - scal[1];        // kappa = f_t't' - f_tt - omega
      if (r < no) v += Geo[r] - lam[r] * lam[r] * gom - (r == 0 ? scal[1] : 0.0);
      else {
        const int a = r - no;
        v += Gev[a] + (a < no ? lam[a] * lam[a] * gom : 0.0) + (a == 0 ? scal[1] : 0.0);
      }
    }
    return v;
  };
  dF[e] = 0.5 * (read(p, q) + read(q, p));
}

// dB[Q] = (R + R^T) / 2, R the read-position gradient: Bov at (i, n_occ + a), Bvt at
// (n_occ + a, n_occ + l), Boo at (i, j), zero elsewhere
__global__ void k_grad_b_assemble(const double* dBov, const double* dBvt, const double* dBoo, int no, int nv,
                                  int naux, double* dB) {
  const int n = no + nv;
  const int64_t tot = (int64_t)naux * n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int Q = (int)(e / ((int64_t)n * n)), r = (int)(e % ((int64_t)n * n));
    const int p = r / n, q = r % n;
    auto read = [&](int r0, int c0) -> double {
      if (r0 < no && c0 >= no) return dBov[((int64_t)Q * no + r0) * nv + (c0 - no)];
      if (r0 >= no && c0 >= no && c0 - no < no) return dBvt[((int64_t)Q * nv + (r0 - no)) * no + (c0 - no)];
      if (r0 < no && c0 < no) return dBoo[((int64_t)Q * no + r0) * no + c0];
      return 0.0;
    };
    dB[e] = 0.5 * (read(p, q) + read(q, p));
  }
}

// TOP-basis factor blocks of a problem given in the TOP basis
__global__ void k_extract_blocks(const double* B, int no, int nv, int naux, double* Bov, double* Bvt, double* Boo) {
  const int n = no + nv;
  const int64_t per = (int64_t)no * nv * 2 + (int64_t)no * no;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)naux * per;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int Q = (int)(e / per);
    int r = (int)(e % per);
    const double* b = B + (int64_t)Q * n * n;
    if (r < no * nv) {
      Bov[(int64_t)Q * no * nv + r] = b[(r / nv) * n + no + r % nv];
    } else if ((r -= no * nv) < nv * no) {
      Bvt[(int64_t)Q * nv * no + r] = b[(no + r / no) * n + no + r % no];
    } else {
      r -= nv * no;
      Boo[(int64_t)Q * no * no + r] = b[(r / no) * n + r % no];
    }
  }
}

__global__ void k_identity(double* R, int n) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n * n; e += gridDim.x * blockDim.x)
    R[e] = (e / n == e % n) ? 1.0 : 0.0;
}

}  // namespace esmp2
