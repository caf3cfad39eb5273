// Right-hand side b_mu = <mu|H|Psi0> on doubles + L-triples, the diagonal
// denominators D_mu = <mu|F|mu> - E0, and the directly inverted S-triple
// energy E2_S = -sum_S b^2/D (paper Sec. II.B-II.D).
//
// Reference Psi0 = sum_l c_l (a+_{l' u} a_{l u} + sg a+_{l' d} a_{l d})|Phi>,
// c_l = lambda_l / sqrt(2), TOP basis (t = occupied 0, t' = virtual 0);
// sg = +1 for the singlet, -1 for the M_s = 0 triplet.  A stored amplitude
// receives the alpha singles' terms as they are and the beta singles' terms
// times sg (the flip partner of a stored determinant carries sg times its
// amplitude).
// Singles -> doubles couple through f^Phi (Fock matrix of the closed shell)
// and the integrals with one TOP index; singles -> triples through the
// antisymmetrised (ov|ov) integrals.  Integral blocks (DF form):
//   V[(i,a),(j,b)] = (ia|jb)
//   M[(i,a),(j,b)] = c_i (a i'|b j) - c_a (a_o i|b j)   (a_o: occupied a, a < n_occ)
#include "common.h"
#include "sigma.h"
#include "reduce.h"
#include <math.h>

namespace esmp2 {

// f^Phi_ov = F~_ov - G[gamma - gamma_Phi]_ov, G[g]_pq = sum_rs g_rs((pq|rs) - (ps|rq)/2),
// gamma - gamma_Phi = diag(-lam_l^2 on l, +lam_l^2 on l'):
//   G_ia = sum_Q [ dq_Q Bov_Q[i][a] - (1/2) sum_k w_k Bov_Q[i][k] Bvt_Q[a][k]
//                  + (1/2) sum_k w_k Boo_Q[i][k] Bov_Q[k][a] ],
//   dq_Q = sum_k w_k (Bvt_Q[k][k] - Boo_Q[k][k]),  w_k = lam_k^2.
constexpr int FPHI_QCHUNKS = 64;   // 64 x n_occ workgroups: enough to spread the n_aux sum over the chip

__global__ void k_fphi_dq(const double* Bvt, const double* Boo, const double* lam, int no, int nv, int naux,
                          double* dq) {
  const int Q = blockIdx.x * blockDim.x + threadIdx.x;
  if (Q >= naux) return;
  const double* bvt = Bvt + (int64_t)Q * nv * no;
  const double* boo = Boo + (int64_t)Q * no * no;
  double t = 0.0;
  for (int k = 0; k < no; ++k) t += lam[k] * lam[k] * (bvt[k * no + k] - boo[k * no + k]);
  dq[Q] = t;
}

// partial G_ia over one chunk of the auxiliary index: grid (FPHI_QCHUNKS, no), thread = a
__global__ __launch_bounds__(256) void k_fphi_part(const double* Bov, const double* Bvt, const double* Boo,
                                                   const double* lam, const double* dq, int no, int nv, int naux,
                                                   double* part) {
  const int i = blockIdx.y, a = threadIdx.x;
  if (a >= nv) return;
  const int q0 = (int)((int64_t)naux * blockIdx.x / gridDim.x), q1 = (int)((int64_t)naux * (blockIdx.x + 1) / gridDim.x);
  double g = 0.0;
  for (int Q = q0; Q < q1; ++Q) {
    const double* bov = Bov + (int64_t)Q * no * nv;
    const double* bvt = Bvt + (int64_t)Q * nv * no;
    const double* boo = Boo + (int64_t)Q * no * no;
    double kv = 0.0, ko = 0.0;
    for (int k = 0; k < no; ++k) {
      const double w = lam[k] * lam[k];
      kv += w * bov[i * nv + k] * bvt[a * no + k];
      ko += w * boo[i * no + k] * bov[k * nv + a];
    }
    g += dq[Q] * bov[i * nv + a] - 0.5 * kv + 0.5 * ko;
  }
  part[((int64_t)blockIdx.x * no + i) * nv + a] = g;
}

__global__ void k_fphi_sum(const double* Ft, const double* part, int no, int nv, int nchunks, double* fphi) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= no * nv) return;
  const int i = e / nv, a = e % nv, n = no + nv;
  double g = 0.0;
  for (int c = 0; c < nchunks; ++c) g += part[(int64_t)c * no * nv + e];
  fphi[e] = Ft[i * n + no + a] - g;
}

// X[Q][(i,a)] = c_i Bvt[Q][a][i] - c_a Boo[Q][a][i]  (second term only for a < n_occ)
__global__ void k_make_x(const double* Bvt, const double* Boo, const double* lam, int no, int nv,
                         int naux, double* X) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)naux * no * nv) return;
  int Q = e / (no * nv);
  int r = e % (no * nv);
  int i = r / nv, a = r % nv;
  const double s2 = 0.70710678118654752440;
  double v = lam[i] * s2 * Bvt[((int64_t)Q * nv + a) * no + i];
  if (a < no) v -= lam[a] * s2 * Boo[((int64_t)Q * no + a) * no + i];
  X[e] = v;
}

struct RhsArgs {
  Dims d;
  const double* V;      // (ia|jb)
  const double* M;      // sum_Q X[Q][(i,a)] Bov[Q][(j,b)] (c_i (a i'|b j) - c_a (a_o i|b j) in the TOP basis)
  const double* fphi;   // no x nv
  const double* lam;
  double* b;
  const double* Cs;     // GEN: singles amplitudes C[i][a] of Psi0 in the orbital basis of V, M, fphi (no x nv)
  // the Jacobi diagonal and the start of a conjugate gradient from x = 0 in the
  // same pass (chunk kernel, when p is set): dinv = 1/D from the orbital
  // energies eo, ev of this basis (as k_diag_chunks), r = -b, p = dinv r, and
  // per workgroup the parts of <r, dinv r>_W into part[blk] and of <r, r>_W
  // into part[nblocks + blk]
  float* dinv = nullptr;
  double* p = nullptr;
  double* part = nullptr;
  const double* eo = nullptr;
  const double* ev = nullptr;
  double omega = 0.0;
};

// Box and local index of a flat amplitude index.  A box holds fewer than 2^31
// amplitudes (at most 64^2 x 192^2), so the local index and the index
// arithmetic on it are 32-bit (a 64-bit division is a long software sequence).
__device__ inline int box_of(const Dims& d, int64_t g, int& loc) {
  int k = 0;
  while (k < 6 && g >= d.off[k + 1]) ++k;
  loc = (int)(g - d.off[k]);
  return k;
}

// GEN = false: the TOP basis, where Psi0's singles amplitudes are diagonal,
// C[l][l'] = c_l, and a term c_l [x = l'] is kept only where the indices meet.
// GEN = true: any orbital basis that leaves t and t' in place (the
// pinned-semicanonical one): every such term reads C[l][x].  The terms with a
// pinned index (C[t][x] = c_0 [x = t'], C[l][t'] = c_0 [l = t]) keep their TOP
// form in both.  V, M and fphi are tensors in (i, a): given in the new basis.
// b of one amplitude of box `box` with occupied indices (P, Q) and virtual
// indices (X, Y) in the box's own naming (actual orbitals): T2 and S2 (i, j,
// a, b); T3 and H1P1 (j, k, b, c); H1P2 (j, k, a, c); H2P1 (i, k, b, c);
// H2P2 (i, k, a, c).
template <bool GEN>
__device__ __attribute__((always_inline)) inline double rhs_element(const RhsArgs& A, int box, int P, int Q, int X,
                                                                    int Y) {
  const Dims& d = A.d;
  const int nv = d.nv, nov = d.no * nv;
  const double s2 = 0.70710678118654752440;
  auto c = [&](int l) -> double { return A.lam[l] * s2; };
  // c_l [x = l'] (TOP) or C[l][x] (GEN); occupied l, virtual x
  auto cx = [&](int l, int x) -> double { return GEN ? A.Cs[l * nv + x] : (x == l ? c(l) : 0.0); };
  auto V = [&](int i, int a, int j, int b) -> double { return A.V[(int64_t)(i * nv + a) * nov + j * nv + b]; };
  // m[i,j,a,b] = c_i d(a,i) fphi[j][b] + M[(i,a),(j,b)]
  auto m = [&](int i, int j, int a, int b) -> double {
    double v = A.M[(int64_t)(i * nv + a) * nov + j * nv + b];
    if (GEN) v += cx(i, a) * A.fphi[j * nv + b];
    else if (a == i) v += c(i) * A.fphi[j * nv + b];
    return v;
  };
  double out = 0.0;
  const double c0 = c(0);
  const double sg = (double)d.sg;
  switch (box) {
    case B_T2: {
      const int i = P, j = Q, a = X, b = Y;
      out = m(i, j, a, b) - m(j, i, a, b) - m(i, j, b, a) + m(j, i, b, a);
      break;
    }
    case B_S2: {
      const int i = P, j = Q, a = X, b = Y;
      out = m(i, j, a, b) + sg * m(j, i, b, a);        // second term: the beta singles
      break;
    }
    case B_T3: {
      const int j = P, k = Q, b = X, cc = Y;
      auto E = [&](int kk, int x) { return V(0, 0, kk, x) - V(kk, 0, 0, x); };
      out = c0 * (V(j, b, k, cc) - V(k, b, j, cc));
      if (GEN) {
        out += cx(j, b) * E(k, cc) - cx(k, b) * E(j, cc) - cx(j, cc) * E(k, b) + cx(k, cc) * E(j, b);
      } else {
        if (b == j) out += c(j) * E(k, cc);
        if (b == k) out -= c(k) * E(j, cc);
        if (cc == j) out -= c(j) * E(k, b);
        if (cc == k) out += c(k) * E(j, b);
      }
      break;
    }
    case B_H11: {
      const int j = P, k = Q, b = X, cc = Y;
      double o2 = 0.0;                                    // beta singles (down TOP pairs)
      if (GEN) {
        o2 = cx(j, b) * V(0, 0, k, cc) - cx(k, b) * V(0, 0, j, cc) - cx(j, cc) * V(0, 0, k, b)
           + cx(k, cc) * V(0, 0, j, b);
      } else {
        if (b == j) o2 += c(j) * V(0, 0, k, cc);
        if (b == k) o2 -= c(k) * V(0, 0, j, cc);
        if (cc == j) o2 -= c(j) * V(0, 0, k, b);
        if (cc == k) o2 += c(k) * V(0, 0, j, b);
      }
      out = c0 * (V(j, b, k, cc) - V(k, b, j, cc)) + sg * o2;
      break;
    }
    case B_H12: {
      const int j = P, k = Q, a = X, cc = Y;
      if (j == 0) out += c0 * V(0, a, k, cc);            // all from the beta singles
      if (k == 0) out -= c0 * V(0, a, j, cc);
      if (GEN) {
        out += cx(k, cc) * V(0, a, j, 0) - cx(j, cc) * V(0, a, k, 0);
      } else {
        if (cc == j) out -= c(j) * V(0, a, k, 0);
        if (cc == k) out += c(k) * V(0, a, j, 0);
      }
      out *= sg;
      break;
    }
    case B_H21: {
      const int i = P, k = Q, b = X, cc = Y;
      if (b == 0) out += c0 * V(i, 0, k, cc);            // all from the beta singles
      if (cc == 0) out -= c0 * V(i, 0, k, b);
      if (GEN) {
        out += cx(k, cc) * V(i, 0, 0, b) - cx(k, b) * V(i, 0, 0, cc);
      } else {
        if (b == k) out -= c(k) * V(i, 0, 0, cc);
        if (cc == k) out += c(k) * V(i, 0, 0, b);
      }
      out *= sg;
      break;
    }
    default: {  // B_H22
      const int i = P, k = Q, a = X, cc = Y;
      double o2 = c0 * V(i, a, k, cc);                   // beta singles
      if (GEN) o2 += cx(k, cc) * V(i, a, 0, 0);
      else if (cc == k) o2 += c(k) * V(i, a, 0, 0);
      out = sg * o2;
      if (GEN) out += cx(i, a) * (V(0, 0, k, cc) - V(k, 0, 0, cc));
      else if (a == i) out += c(i) * (V(0, 0, k, cc) - V(k, 0, 0, cc));    // the alpha single i -> i'
      break;
    }
  }
  return out;
}

// one thread per amplitude, the indices decoded from the flat position
template <bool GEN>
__global__ void k_rhs(RhsArgs A) {
  const Dims& d = A.d;
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= d.off[7]) return;
  int loc;
  const int box = box_of(d, g, loc);
  const int no = d.no, nv = d.nv, m1 = nv - 1;
  int P, Q, X, Y;
  switch (box) {
    case B_T2: tri_pq(loc / d.npv, no, P, Q); tri_pq(loc % d.npv, nv, X, Y); break;
    case B_S2: P = loc / (no * nv * nv); Q = (loc / (nv * nv)) % no; X = (loc / nv) % nv; Y = loc % nv; break;
    case B_T3:
      tri_pq(loc / d.npv1, no - 1, P, Q); tri_pq(loc % d.npv1, nv - 1, X, Y);
      ++P; ++Q; ++X; ++Y;
      break;
    case B_H11: tri_pq(loc / d.npv, no, P, Q); tri_pq(loc % d.npv, nv, X, Y); break;
    case B_H12: {
      tri_pq(loc / (m1 * m1), no, P, Q);
      const int r = loc % (m1 * m1);
      X = r / m1 + 1; Y = r % m1 + 1;
      break;
    }
    case B_H21: {
      const int o = loc / d.npv;
      P = o / (no - 1) + 1; Q = o % (no - 1) + 1;
      tri_pq(loc % d.npv, nv, X, Y);
      break;
    }
    default: {
      const int o = loc / (m1 * m1), r = loc % (m1 * m1);
      P = o / (no - 1) + 1; Q = o % (no - 1) + 1;
      X = r / m1 + 1; Y = r % m1 + 1;
      break;
    }
  }
  A.b[g] = rhs_element<GEN>(A, box, P, Q, X, Y);
}

// The same by the coupling chunks (box, batch, inner range; 16 x 16 tiles of
// (a, b) in S2, so that the transposed integral reads M[(j,b),(i,a)] come in
// 128-byte runs): the occupied indices come with the chunk, the virtual pair
// from the pair tables, no square roots.
template <bool GEN>
__global__ __launch_bounds__(256) void k_rhs_chunks(RhsArgs A, PairTables T, const int4* chunks) {
  const Dims& d = A.d;
  const int4 ch = chunks[blockIdx.x];
  const int box = ch.x, batch = ch.y, P = ch.w >> 16, Q = ch.w & 0xffff;
  const int nv = d.nv, m1 = nv - 1;
  int inner;
  switch (box) {
    case B_T2: case B_H11: case B_H21: inner = d.npv; break;
    case B_S2: inner = nv * nv; break;
    case B_T3: inner = d.npv1; break;
    default: inner = m1 * m1; break;
  }
  const int v = chunk_inner(box, ch.z, (int)threadIdx.x, nv, inner);
  const bool in = v < inner;
  const int64_t g = d.off[box] + (int64_t)batch * inner + v;
  double rz = 0.0, rr = 0.0;
  if (in) {
    int X, Y;
    switch (box) {
      case B_T2: case B_H11: case B_H21: { const int t = T.pv[v]; X = t >> 16; Y = t & 0xffff; break; }
      case B_S2: X = v / nv; Y = v - X * nv; break;
      case B_T3: { const int t = T.pv1[v]; X = (t >> 16) + 1; Y = (t & 0xffff) + 1; break; }
      default: X = v / m1 + 1; Y = v - (X - 1) * m1 + 1; break;
    }
    float dv = 0.0f;
    if (A.p) {
      const double D = box >= B_T3 ? (A.ev[0] - A.eo[0] - A.omega) + A.ev[X] + A.ev[Y] - A.eo[P] - A.eo[Q]
                                   : A.ev[X] + A.ev[Y] - A.eo[P] - A.eo[Q] - A.omega;
      dv = (float)(1.0 / D);
      __builtin_nontemporal_store(dv, A.dinv + g);
    }
    const double bv = rhs_element<GEN>(A, box, P, Q, X, Y);
    __builtin_nontemporal_store(bv, A.b + g);
    if (A.p) {
      const double rg = -bv, w = box == B_S2 ? 1.0 : 2.0;
      __builtin_nontemporal_store((double)dv * rg, A.p + g);
      rz = w * rg * rg * (double)dv;
      rr = w * rg * rg;
    }
  }
  if (A.p) {               // the same for every workgroup of the launch
    const double a = block_sum(rz);
    const double c = block_sum(rr);
    if (threadIdx.x == 0) { A.part[blockIdx.x] = a; A.part[gridDim.x + blockIdx.x] = c; }
  }
}

// Singles amplitudes of Psi0 in a basis reached from the TOP one by the
// orbital rotations To (occupied) and Tv (virtual): C[I][A] = sum_l To[l][I]
// c_l Tv[l][A], c_l = lambda_l / sqrt(2) on the pair (l, l').
__global__ void k_singles_sc(const double* To, const double* Tv, const double* lam, int no, int nv, double* C) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= no * nv) return;
  const int I = e / nv, A = e % nv;
  const double s2 = 0.70710678118654752440;
  double v = 0.0;
  for (int l = 0; l < no; ++l) v += To[l * no + I] * (lam[l] * s2) * Tv[l * nv + A];
  C[e] = v;
}

template __global__ void k_rhs<false>(RhsArgs);
template __global__ void k_rhs<true>(RhsArgs);
template __global__ void k_rhs_chunks<false>(RhsArgs, PairTables, const int4*);
template __global__ void k_rhs_chunks<true>(RhsArgs, PairTables, const int4*);

// Diagonal D_mu = (sum of particle minus hole orbital energies) - omega and its
// inverse; also records the minimum (for the NOT_SPD check) per block.
struct DiagArgs {
  Dims d;
  const double* eo;     // TOP-basis occupied orbital energies F~_ii
  const double* ev;     // TOP-basis virtual orbital energies F~_aa
  double omega;
  float* dinv;          // the Jacobi preconditioner 1/D, rounded once to FP32
  double* blockmin;
};

__device__ inline double diag_of(const Dims& d, int box, int loc, const double* eo, const double* ev,
                                 double om) {
  const int no = d.no, nv = d.nv;
  const double base = ev[0] - eo[0] - om;
  switch (box) {
    case B_T2: {
      int po = loc / d.npv, pv = loc % d.npv, i, j, a, b;
      tri_pq(po, no, i, j); tri_pq(pv, nv, a, b);
      return ev[a] + ev[b] - eo[i] - eo[j] - om;
    }
    case B_S2: {
      int nov = no * nv;
      int i = loc / (nov * nv), r = loc % (nov * nv);
      int j = r / (nv * nv); r %= nv * nv;
      return ev[r / nv] + ev[r % nv] - eo[i] - eo[j] - om;
    }
    case B_T3: {
      int po = loc / d.npv1, pv = loc % d.npv1, j, k, b, c;
      tri_pq(po, no - 1, j, k); tri_pq(pv, nv - 1, b, c);
      return base + ev[b + 1] + ev[c + 1] - eo[j + 1] - eo[k + 1];
    }
    case B_H11: {
      int po = loc / d.npv, pv = loc % d.npv, j, k, b, c;
      tri_pq(po, no, j, k); tri_pq(pv, nv, b, c);
      return base + ev[b] + ev[c] - eo[j] - eo[k];
    }
    case B_H12: {
      int m1 = nv - 1, po = loc / (m1 * m1), r = loc % (m1 * m1), j, k;
      tri_pq(po, no, j, k);
      return base + ev[r / m1 + 1] + ev[r % m1 + 1] - eo[j] - eo[k];
    }
    case B_H21: {
      int o = loc / d.npv, pv = loc % d.npv, b, c;
      tri_pq(pv, nv, b, c);
      return base + ev[b] + ev[c] - eo[o / (no - 1) + 1] - eo[o % (no - 1) + 1];
    }
    default: {
      int m1 = nv - 1, o = loc / (m1 * m1), r = loc % (m1 * m1);
      return base + ev[r / m1 + 1] + ev[r % m1 + 1] - eo[o / (no - 1) + 1] - eo[o % (no - 1) + 1];
    }
  }
}

// grid-stride over the amplitudes (a grid of at most DIAG_BLOCKS workgroups)
constexpr int DIAG_BLOCKS = 2048;

__global__ __launch_bounds__(256) void k_diag(DiagArgs A) {
  double mn = 1e300;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < A.d.off[7];
       g += (int64_t)gridDim.x * blockDim.x) {
    int loc;
    int box = box_of(A.d, g, loc);
    double D = diag_of(A.d, box, loc, A.eo, A.ev, A.omega);
    A.dinv[g] = (float)(1.0 / D);
    mn = fmin(mn, D);
  }
  // block minimum
  for (int o = 32; o > 0; o >>= 1) mn = fmin(mn, __shfl_xor(mn, o));
  __shared__ double ws[4];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = mn;
  __syncthreads();
  if (threadIdx.x == 0) A.blockmin[blockIdx.x] = fmin(fmin(ws[0], ws[1]), fmin(ws[2], ws[3]));
}

// The same diagonal walked by coupling chunks (box, batch, inner range; the
// table of the coupling kernels): the occupied indices come with the chunk and
// the virtual pair from the pair tables, so no element decodes its position by
// square roots.  Each workgroup takes DIAG_UNROLL consecutive chunks per pass,
// their table reads issued together (the walk is bound by the latency of the
// chunk -> pair -> orbital-energy reads, not by the 4-byte stores), grid-stride
// over the passes; blockmin[blockIdx.x] as k_diag.
constexpr int DIAG_UNROLL = 4;

__device__ inline int chunk_inner_count(const Dims& d, int box) {
  switch (box) {
    case B_T2: case B_H11: case B_H21: return d.npv;
    case B_S2: return d.nv * d.nv;
    case B_T3: return d.npv1;
    default: return (d.nv - 1) * (d.nv - 1);
  }
}

__global__ __launch_bounds__(256) void k_diag_chunks(DiagArgs A, PairTables P, const int4* chunks, int nchunks) {
  const Dims& d = A.d;
  const int nv = d.nv, m1 = nv - 1;
  const double base = A.ev[0] - A.eo[0] - A.omega;   // the pinned pair of the L-triples
  double mn = 1e300;
  for (int c0 = blockIdx.x * DIAG_UNROLL; c0 < nchunks; c0 += gridDim.x * DIAG_UNROLL) {
    int4 ch[DIAG_UNROLL];
    int v[DIAG_UNROLL], inner[DIAG_UNROLL], t[DIAG_UNROLL];
#pragma unroll
    for (int u = 0; u < DIAG_UNROLL; ++u) ch[u] = chunks[min(c0 + u, nchunks - 1)];
#pragma unroll
    for (int u = 0; u < DIAG_UNROLL; ++u) {
      inner[u] = chunk_inner_count(d, ch[u].x);
      v[u] = c0 + u < nchunks ? chunk_inner(ch[u].x, ch[u].z, (int)threadIdx.x, nv, inner[u]) : inner[u];
      const int box = ch[u].x;
      t[u] = 0;
      if (v[u] < inner[u]) {
        if (box == B_T2 || box == B_H11 || box == B_H21) t[u] = P.pv[v[u]];
        else if (box == B_T3) t[u] = P.pv1[v[u]];
      }
    }
#pragma unroll
    for (int u = 0; u < DIAG_UNROLL; ++u) {
      if (v[u] >= inner[u]) continue;
      const int box = ch[u].x, i = ch[u].w >> 16, j = ch[u].w & 0xffff;
      int a, b;
      switch (box) {
        case B_T2: case B_H11: case B_H21: a = t[u] >> 16; b = t[u] & 0xffff; break;
        case B_S2: a = v[u] / nv; b = v[u] - a * nv; break;
        case B_T3: a = (t[u] >> 16) + 1; b = (t[u] & 0xffff) + 1; break;
        default: a = v[u] / m1 + 1; b = v[u] - (a - 1) * m1 + 1; break;
      }
      const double D = box >= B_T3 ? base + A.ev[a] + A.ev[b] - A.eo[i] - A.eo[j]
                                   : A.ev[a] + A.ev[b] - A.eo[i] - A.eo[j] - A.omega;
      A.dinv[d.off[box] + (int64_t)ch[u].y * inner[u] + v[u]] = (float)(1.0 / D);
      mn = fmin(mn, D);
    }
  }
  for (int o = 32; o > 0; o >>= 1) mn = fmin(mn, __shfl_xor(mn, o));
  __shared__ double ws[4];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = mn;
  __syncthreads();
  if (threadIdx.x == 0) A.blockmin[blockIdx.x] = fmin(fmin(ws[0], ws[1]), fmin(ws[2], ws[3]));
}

// The smallest diagonal denominator D of the one-TOP space, from the orbital
// energies alone: D separates into particle minus hole energies, so the
// minimum over a box is its smallest particle sum minus its largest hole sum
// (two distinct indices for a packed pair, any two for a free pair; virtual
// and occupied index 0 excluded where the box excludes t' or t).  One
// wavefront: per-lane two smallest (largest) values, merged by shuffles.
__device__ inline void merge_two_small(double& s1, double& s2) {
  for (int o = 32; o > 0; o >>= 1) {
    const double t1 = __shfl_xor(s1, o), t2 = __shfl_xor(s2, o);
    const double n1 = fmin(s1, t1), n2 = fmin(fmax(s1, t1), fmin(s2, t2));
    s1 = n1; s2 = n2;
  }
}

__global__ __launch_bounds__(64) void k_diag_min(Dims d, const double* eo, const double* ev, double omega,
                                                 double* out) {
  const int no = d.no, nv = d.nv, l = threadIdx.x;
  // two smallest virtual energies over [lo, nv) and two largest occupied ones
  // over [lo, no) (the largest as the smallest of -eo)
  double va1 = 1e300, va2 = 1e300, vb1 = 1e300, vb2 = 1e300;
  double oa1 = 1e300, oa2 = 1e300, ob1 = 1e300, ob2 = 1e300;
  auto ins = [](double e, double& s1, double& s2) {
    if (e < s1) { s2 = s1; s1 = e; } else if (e < s2) s2 = e;
  };
  for (int a = l; a < nv; a += 64) {
    ins(ev[a], va1, va2);
    if (a >= 1) ins(ev[a], vb1, vb2);
  }
  for (int i = l; i < no; i += 64) {
    ins(-eo[i], oa1, oa2);
    if (i >= 1) ins(-eo[i], ob1, ob2);
  }
  merge_two_small(va1, va2);
  merge_two_small(vb1, vb2);
  merge_two_small(oa1, oa2);
  merge_two_small(ob1, ob2);
  if (l != 0) return;
  const double base = ev[0] - eo[0] - omega;
  double mn = 1e300;
  auto take = [&](int box, double v) { if (d.off[box + 1] > d.off[box]) mn = fmin(mn, v); };
  take(B_T2, (va1 + va2) + (oa1 + oa2) - omega);
  take(B_S2, 2.0 * va1 + 2.0 * oa1 - omega);
  take(B_T3, base + (vb1 + vb2) + (ob1 + ob2));
  take(B_H11, base + (va1 + va2) + (oa1 + oa2));
  take(B_H12, base + 2.0 * vb1 + (oa1 + oa2));
  take(B_H21, base + (va1 + va2) + 2.0 * ob1);
  take(B_H22, base + 2.0 * vb1 + 2.0 * ob1);
  out[0] = mn;
}

__global__ void k_min_reduce(const double* v, int64_t n, double* out) {
  double mn = 1e300;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) mn = fmin(mn, v[i]);
  for (int o = 32; o > 0; o >>= 1) mn = fmin(mn, __shfl_xor(mn, o));
  __shared__ double ws[16];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = mn;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 1e300;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) r = fmin(r, ws[k]);
    out[0] = r;
  }
}

// ---------------------------------------------------------------------------
// E2_S.  Same-spin sector (up up up; doubled for down down down): triples
// {l, j, k; l', b, c} enumerated by the smallest TOP l >= 1 they contain, with
// no smaller TOP m (m in {j,k} and m' in {b,c}); t = 0 is therefore excluded.
// b = sum over contained TOP pairs (A_p = I_q') of (-1)^{p+q} c_{I_q} <A..||I..>.
// ---------------------------------------------------------------------------
struct E2sArgs {
  Dims d;
  const double* V; const double* lam; const double* eo; const double* ev;
  double omega;
  double* partial;      // one per block (blockIdx.y * gridDim.x + blockIdx.x)
  const int *pv, *pv1, *po, *po1;   // pair tables ((p << 16) | q, p < q) of nv, nv-1, no, no-1
};

// 1/D for the S-triple sums: the hardware reciprocal estimate refined by two
// Newton steps (relative error at the FP64 rounding level; D > 0 here)
__device__ inline double recip_fast(double D) {
  double r = __builtin_amdgcn_rcp(D);
  r = fma(fma(-D, r, 1.0), r, r);
  r = fma(fma(-D, r, 1.0), r, r);
  return r;
}

__device__ inline void sort3(int& x, int& y, int& z) {
  if (x > y) { int t = x; x = y; y = t; }
  if (y > z) { int t = y; y = z; z = t; }
  if (x > y) { int t = x; x = y; y = t; }
}

// b of the same-spin triple {l, j, k; l', b, c} from every contained TOP pair
__device__ inline double b_same(const E2sArgs& A, int l, int j, int k, int b, int c) {
  const int nv = A.d.nv, nov = A.d.no * nv;
  const double s2 = 0.70710678118654752440;
  int I[3] = {l, j, k}, P[3] = {l, b, c};
  sort3(I[0], I[1], I[2]);
  sort3(P[0], P[1], P[2]);
  double bv = 0.0;
  for (int p = 0; p < 3; ++p)
    for (int q = 0; q < 3; ++q) {
      if (P[p] != I[q]) continue;
      int a1 = P[p == 0 ? 1 : 0], a2 = P[p == 2 ? 1 : 2];
      int i1 = I[q == 0 ? 1 : 0], i2 = I[q == 2 ? 1 : 2];
      double anti = A.V[(int64_t)(i1 * nv + a1) * nov + i2 * nv + a2] -
                    A.V[(int64_t)(i2 * nv + a1) * nov + i1 * nv + a2];
      double sg = ((p + q) & 1) ? -1.0 : 1.0;
      bv += sg * A.lam[I[q]] * s2 * anti;
    }
  return bv;
}

// The grid's workgroups stride over the chunks of 256 (b<c) pairs of one (j<k)
// pair (all orbitals); a lane runs over the smallest TOP l >= 1 outside both
// pairs.  Unless b or c is one of j, k, the one contained TOP pair is (l, l'),
// whose integral <j b||k c> does not depend on l: loaded once, then only the
// sign (positions of l among the sorted holes and particles), lam_l and the
// denominator change with l.
__global__ __launch_bounds__(256) void k_e2s_same(E2sArgs A) {
  const Dims& d = A.d;
  const int no = d.no, nv = d.nv, nov = no * nv;
  const int nch = (d.npv + 255) / 256, nt = d.npo * nch;
  const int bid = blockIdx.y * gridDim.x + blockIdx.x, nb = gridDim.x * gridDim.y;
  const double s2 = 0.70710678118654752440;
  double acc = 0.0;
  for (int t = bid; t < nt; t += nb) {
    const int pi = t / nch, vi = (t - pi * nch) * 256 + (int)threadIdx.x;
    if (vi >= d.npv) continue;
    const int to = A.po[pi], tv = A.pv[vi];
    const int j = to >> 16, k = to & 0xffff, b = tv >> 16, c = tv & 0xffff;
    const bool kron = b == j || b == k || c == j || c == k;
    const double anti = kron ? 0.0
                             : A.V[(int64_t)(j * nv + b) * nov + k * nv + c] -
                               A.V[(int64_t)(k * nv + b) * nov + j * nv + c];
    for (int l = 1; l < no; ++l) {
      if (l == j || l == k || l == b || l == c) continue;
      if ((j < l && (j == b || j == c)) || (k < l && (k == b || k == c))) continue;   // a smaller TOP
      int I[3] = {l, j, k}, P[3] = {l, b, c};
      sort3(I[0], I[1], I[2]);
      sort3(P[0], P[1], P[2]);
      double bv;
      if (kron) {
        bv = b_same(A, l, j, k, b, c);
      } else {
        const int pp = (l > b) + (l > c), qq = (l > j) + (l > k);    // positions of l
        bv = (((pp + qq) & 1) ? -1.0 : 1.0) * A.lam[l] * s2 * anti;
      }
      double D = A.ev[P[0]] + A.ev[P[1]] + A.ev[P[2]] - A.eo[I[0]] - A.eo[I[1]] - A.eo[I[2]] - A.omega;
      acc += bv * bv * recip_fast(D);
    }
  }
  double s = block_sum(2.0 * acc);
  if (threadIdx.x == 0) A.partial[blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// Mixed sector (up; down down), doubled for its spin flip.  Case A: the up pair
// is a TOP (a = i >= 1), down pairs arbitrary.  Case B: a != i, the down pairs
// share a TOP l (smallest such l), holes {l, m}, particles {l', e}.  Triples
// containing t (0 among the holes and 0 among the particles) are L, skipped.
__device__ inline double b_mixed(const E2sArgs& A, int i, int a, int j, int k, int b, int c) {
  const int nv = A.d.nv, nov = A.d.no * nv;
  const double s2 = 0.70710678118654752440;
  auto V = [&](int p, int x, int q, int y) { return A.V[(int64_t)(p * nv + x) * nov + q * nv + y]; };
  double bd = 0.0;                                 // beta singles (down TOP pairs)
  if (b == j) bd += A.lam[j] * s2 * V(i, a, k, c);
  if (b == k) bd -= A.lam[k] * s2 * V(i, a, j, c);
  if (c == j) bd -= A.lam[j] * s2 * V(i, a, k, b);
  if (c == k) bd += A.lam[k] * s2 * V(i, a, j, b);
  double bv = (double)A.d.sg * bd;
  if (a == i) bv += A.lam[i] * s2 * (V(j, b, k, c) - V(k, b, j, c));     // the alpha single i -> i'
  return bv;
}

// The grid's workgroups stride over the chunks of 256 (b<c) pairs of one (j<k)
// pair; a lane loads the pair's antisymmetrised integral once and runs over the
// up hole i >= 1 of the up TOP pair (a = i), which enters only through lam_i,
// the denominator and the rare Kronecker terms of b_mixed.
__global__ __launch_bounds__(256) void k_e2s_mixed_a(E2sArgs A) {
  const Dims& d = A.d;
  const int no = d.no, nv = d.nv, nov = no * nv;
  const int nch = (d.npv + 255) / 256, nt = d.npo * nch;
  const int bid = blockIdx.y * gridDim.x + blockIdx.x, nb = gridDim.x * gridDim.y;
  const double s2 = 0.70710678118654752440;
  auto V = [&](int p, int x, int q, int y) { return A.V[(int64_t)(p * nv + x) * nov + q * nv + y]; };
  double acc = 0.0;
  for (int t = bid; t < nt; t += nb) {
    const int pi = t / nch, vi = (t - pi * nch) * 256 + (int)threadIdx.x;
    if (vi >= d.npv) continue;
    const int to = A.po[pi], tv = A.pv[vi];
    const int j = to >> 16, k = to & 0xffff, b = tv >> 16, c = tv & 0xffff;
    if ((j == 0 || k == 0) && (b == 0 || c == 0)) continue;     // contains t
    const double vd = V(j, b, k, c) - V(k, b, j, c);
    const bool kron = b == j || b == k || c == j || c == k;
    for (int i = 1; i < no; ++i) {
      const double bv = kron ? b_mixed(A, i, i, j, k, b, c) : A.lam[i] * s2 * vd;
      const double D = A.ev[i] + A.ev[b] + A.ev[c] - A.eo[i] - A.eo[j] - A.eo[k] - A.omega;
      acc += bv * bv * recip_fast(D);
    }
  }
  double s = block_sum(2.0 * acc);
  if (threadIdx.x == 0) A.partial[blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// A wavefront per (up excitation (i, a), a != i; down hole m), the grid's
// wavefronts striding over these pairs; its lanes take the down particles e
// (64 at a time), whose integrals V(i a|m e) it loads once for every other
// down hole l (holes {l, m}, particles {l', e}, e != l).  With a != i only the
// beta singles of b_mixed enter, and with the holes and particles sharing l
// their four Kronecker terms reduce to
//   bd = s lam_l V(i a|m e) + [l < m, e = m] lam_m V(i a|l l),
//   s = +1 if (l < m) == (l < e), else -1
// (the case m < l, e = m belongs to the smaller TOP m and is skipped; l = 0
// with t' among the particles is an L-triple).
__global__ __launch_bounds__(256) void k_e2s_mixed_b(E2sArgs A) {
  const Dims& d = A.d;
  const int no = d.no, nv = d.nv, nov = no * nv;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  const int64_t nitem = (int64_t)nov * no;             // item = (i a) * no + m
  const int64_t gw = ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * nw + wave;
  const int64_t NW = (int64_t)gridDim.x * gridDim.y * nw;
  const double s2 = 0.70710678118654752440, sg = (double)d.sg;
  constexpr int EU = 3;                                // particles per lane in registers (64 EU per pass)
  double acc = 0.0;
  for (int64_t it = gw; it < nitem; it += NW) {
    const int ia = (int)(it / no), m = (int)(it - (int64_t)ia * no);
    const int i = ia / nv, a = ia - i * nv;
    if (a == i) continue;
    const double* Vr = A.V + (int64_t)ia * nov;        // row (i, a) of V
    const bool t_hole = i == 0 || m == 0;              // with l >= 1
    const double cm = A.lam[m] * s2;
    // V(i a|l l) of every l, one per lane, loaded together (read back per l by
    // a lane broadcast: a load per l would wait once per iteration)
    const double vll_lane = lane < no ? Vr[lane * nv + lane] : 0.0;
    for (int e0 = 0; e0 < nv; e0 += 64 * EU) {
      double vme[EU], eve[EU];
#pragma unroll
      for (int u = 0; u < EU; ++u) {
        const int e = e0 + lane + 64 * u;
        vme[u] = e < nv ? Vr[m * nv + e] : 0.0;
        eve[u] = e < nv ? A.ev[e] : 0.0;
      }
      for (int l = 1; l < no; ++l) {
        if (l == m) continue;
        const int j = l < m ? l : m, k = l < m ? m : l;
        const double cl = A.lam[l] * s2;
        const long long vb = __double_as_longlong(vll_lane);
        const double vll = __longlong_as_double(
            ((long long)__builtin_amdgcn_readlane((int)(vb >> 32), l) << 32) |
            (unsigned)__builtin_amdgcn_readlane((int)(vb & 0xffffffff), l));
        // D = dq + ev[e]: the particles are {a, l', e}, the holes {i, l, m}
        const double dq = A.ev[a] + A.ev[l] - A.eo[i] - A.eo[j] - A.eo[k] - A.omega;
#pragma unroll
        for (int u = 0; u < EU; ++u) {
          const int e = e0 + lane + 64 * u;
          if (e >= nv || e == l) continue;
          if (m < l && e == m) continue;                              // smaller down TOP m
          if (t_hole && (a == 0 || e == 0)) continue;                 // contains t
          const double t = cl * vme[u];
          double bd = ((l < m) == (l < e)) ? t : -t;
          if (l < m && e == m) bd += cm * vll;
          const double bv = sg * bd;
          acc += bv * bv * recip_fast(dq + eve[u]);
        }
      }
    }
  }
  double s = block_sum(2.0 * acc);
  if (threadIdx.x == 0) A.partial[blockIdx.y * gridDim.x + blockIdx.x] = s;
}

__global__ void k_sum_partials(const double* v, int n, double* out, double scale) {
  Acc2 acc;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc.add(v[i]);
  double s = block_sum2(acc);
  if (threadIdx.x == 0) out[0] = scale * s;
}

}  // namespace esmp2
