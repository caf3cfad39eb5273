// sigma = (H0 - E0) x in the pinned-semicanonical basis.
//
// There F_oo[1:,1:] and F_vv[1:,1:] are diagonal: the Fock blocks are "arrow"
// matrices, dense only in the row and column of the pinned orbital (t for the
// occupied block, t' for the virtual one).  The Sylvester product of a batch,
// Y = F'X + XF', reduces to
//   Y[a][b] = (F'_aa + F'_bb) X[a][b] + u_a X[0][b] + X[a][0] u_b       (a, b >= 1 parts)
//           + [a = 0] g_b + [b = 0] h_a,   g_b = sum_{c>=1} u_c X[c][b],  h_a = sum_{c>=1} X[a][c] u_c,
// with u_c = F'[0][c]; boxes whose virtual indices exclude t' see only the
// diagonal term, and their row-0 product is the transfer row.  The occupied
// action is the same with w_m = F[t][m].  Per amplitude the work is O(1), plus
// O(n_occ) for the batches that hold t, and O(n_vir) per batch for g and h:
// the operator costs O(N_o^2 N_v^2) instead of O(N_o^2 N_v^3).
#include "common.h"
#include "sigma.h"
#include "reduce.h"

namespace esmp2 {

template <class T>
struct ArrowArgs {
  GatherArgs<T> ga;      // x, S~, y, Fock blocks, side contractions, transfer rows
  const T* Fd;           // F'_vv of the doubles boxes (padded mv x mv)
  const T* Fl;           // F'_vv of the L boxes
  T* tr;                 // transfer rows (the same buffer as ga.side_tr)
  T* gv;                 // row/column GEMVs: T2 [npo][nv], S2 g [no^2][nv], S2 h [no^2][nv],
                         // H1P1 [npo][nv], H2P1 [(no-1)^2][nv]
};

template <class T>
__device__ inline void arrow_offsets(const Dims& d, int64_t off[5]) {
  const int64_t nv = d.nv;
  off[0] = 0;                                        // T2
  off[1] = off[0] + (int64_t)d.npo * nv;             // S2 g
  off[2] = off[1] + (int64_t)d.no * d.no * nv;       // S2 h
  off[3] = off[2] + (int64_t)d.no * d.no * nv;       // H1P1
  off[4] = off[3] + (int64_t)d.npo * nv;             // H2P1
}

// Per-batch GEMVs with the t' row of F'.  Jobs: T2 (npo), S2 (no^2), H1P1 (npo),
// H2P1 ((no-1)^2), H1P2 (npo, transfer rows), H2P2 ((no-1)^2, transfer rows).
template <class T>
__global__ __launch_bounds__(256) void k_arrow_side(ArrowArgs<T> A) {
  const GatherArgs<T>& G = A.ga;
  const Dims& d = G.d;
  const int no = d.no, nv = d.nv, n2 = (no - 1) * (no - 1);
  Look<T> L{d, G.x, G.S};
  const T* u = G.fv;                   // u_c = fv[0*nv + c]
  int64_t off[5];
  arrow_offsets<T>(d, off);
  int job = blockIdx.x, box;
  if (job < d.npo) box = B_T2;
  else if ((job -= d.npo) < no * no) box = B_S2;
  else if ((job -= no * no) < d.npo) box = B_H11;
  else if ((job -= d.npo) < n2) box = B_H21;
  else if ((job -= n2) < d.npo) box = B_H12;
  else { job -= d.npo; box = B_H22; }
  // lane -> output column b (64 per workgroup along y), wavefront -> a quarter
  // of the contracted range 1..nv-1; partial sums meet in LDS
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int b = blockIdx.y * 64 + lane;
  const bool col = b < nv;
  const int lo = 1 + (nv - 1) * wave / 4, hi = 1 + (nv - 1) * (wave + 1) / 4;
  int p, q;
  if (box == B_S2) { p = job / no; q = job % no; }
  else if (box == B_H21 || box == B_H22) { p = job / (no - 1) + 1; q = job % (no - 1) + 1; }
  else tri_pq(job, no, p, q);
  T g = 0, hh = 0;
  if (col) {
    switch (box) {
      case B_T2: for (int c = lo; c < hi; ++c) g += u[c] * L.T2(p, q, c, b); break;
      case B_S2:
        for (int c = lo; c < hi; ++c) {
          g += u[c] * L.St(p, q, c, b);
          hh += L.St(p, q, b, c) * u[c];
        }
        break;
      case B_H11: for (int c = lo; c < hi; ++c) g += u[c] * L.H11(p, q, c, b); break;
      case B_H21: for (int c = lo; c < hi; ++c) g += u[c] * L.H21(p, q, c, b); break;
      case B_H12: if (b >= 1) for (int c = lo; c < hi; ++c) g += u[c] * L.H12(p, q, c, b); break;
      default: if (b >= 1) for (int c = lo; c < hi; ++c) g += u[c] * L.H22(p, q, c, b); break;
    }
  }
  __shared__ T part[2][4][64];
  part[0][wave][lane] = g; part[1][wave][lane] = hh;
  __syncthreads();
  if (wave != 0 || !col) return;
  g = part[0][0][lane] + part[0][1][lane] + part[0][2][lane] + part[0][3][lane];
  hh = part[1][0][lane] + part[1][1][lane] + part[1][2][lane] + part[1][3][lane];
  switch (box) {
    case B_T2: A.gv[off[0] + (int64_t)job * nv + b] = g; break;
    case B_S2: A.gv[off[1] + (int64_t)job * nv + b] = g; A.gv[off[2] + (int64_t)job * nv + b] = hh; break;
    case B_H11: A.gv[off[3] + (int64_t)job * nv + b] = g; break;
    case B_H21: A.gv[off[4] + (int64_t)job * nv + b] = g; break;
    case B_H12: A.tr[(int64_t)job * nv + b] = g; break;              // transfer row into H1P1
    default: A.tr[((int64_t)d.npo + job) * nv + b] = g; break;      // transfer row into H2P1
  }
}

// y = sigma for every amplitude: diagonal, arrow terms of both Fock blocks,
// transfer rows, couplings.  One workgroup per chunk of 256 inner indices of
// one batch matrix, 16 x 16 tiles of (a, b) in S2 (the coupling kernel's chunk
// table).
// With pq != nullptr each workgroup also writes its part of <x, y>_W (the CG
// denominator p.Ap) to pq[blockIdx.x].
template <class T>
__device__ __attribute__((always_inline)) inline double arrow_element(const ArrowArgs<T>& A, const PairTables& P,
                                                                      int box, int batch, int i, int j, int v,
                                                                      int inner);

template <class T>
__device__ __attribute__((always_inline)) inline void arrow_body(const ArrowArgs<T>& A, const PairTables& P, const int4* chunks, double* pq, int bid_, int nb_) {
  const Dims& d = A.ga.d;
  const int4 ch = chunks[xcd_remap<32>(bid_, nb_)];
  const int box = ch.x, batch = ch.y;
  const int i = ch.w >> 16, j = ch.w & 0xffff;      // occupied indices of the batch (actual orbitals)
  const int nv = d.nv, m1 = nv - 1;
  int inner;
  switch (box) {
    case B_T2: case B_H11: case B_H21: inner = d.npv; break;
    case B_S2: inner = nv * nv; break;
    case B_T3: inner = d.npv1; break;
    default: inner = m1 * m1; break;
  }
  const int v = chunk_inner(box, ch.z, (int)threadIdx.x, nv, inner);
  double part = 0.0;
  if (v < inner) part = arrow_element(A, P, box, batch, i, j, v, inner);
  if (pq) {
    const double s = block_sum(part);
    if (threadIdx.x == 0) pq[bid_] = s;
  }
}

template <class T>
__global__ __launch_bounds__(256) void k_arrow(ArrowArgs<T> A, PairTables P, const int4* chunks, double* pq) {
  arrow_body<T>(A, P, chunks, pq, blockIdx.x, gridDim.x);
}

template <class T>
__device__ __attribute__((always_inline)) inline double arrow_element(const ArrowArgs<T>& A, const PairTables& P,
                                                                      int box, int batch, int i, int j, int v,
                                                                      int inner) {
  const GatherArgs<T>& G = A.ga;
  const Dims& d = G.d;
  const int no = d.no, nv = d.nv, m1 = nv - 1, mv = d.mv;
  int a, b;                                         // virtual indices (actual orbitals)
  switch (box) {
    case B_T2: case B_H11: case B_H21: { const int t = P.pv[v]; a = t >> 16; b = t & 0xffff; break; }
    case B_S2: a = v / nv; b = v - a * nv; break;
    case B_T3: { const int t = P.pv1[v]; a = (t >> 16) + 1; b = (t & 0xffff) + 1; break; }
    default: a = v / m1 + 1; b = v - (a - 1) * m1 + 1; break;
  }
  Look<T> L{d, G.x, G.S};
  auto X = [&](int p, int q, int r, int c) -> T {   // amplitude of this box (S~ for S2)
    switch (box) {
      case B_T2: return L.T2(p, q, r, c);
      case B_S2: return L.St(p, q, r, c);
      case B_T3: return L.T3(p, q, r, c);
      case B_H11: return L.H11(p, q, r, c);
      case B_H12: return L.H12(p, q, r, c);
      case B_H21: return L.H21(p, q, r, c);
      default: return L.H22(p, q, r, c);
    }
  };
  const T* Fp = (box == B_T2 || box == B_S2) ? A.Fd : A.Fl;
  const T* fo = G.fo;
  const T* u = G.fv;          // u_c = F'[t'][c] (c >= 1)
  const T* w = G.fo;          // w_m = F[t][m] (m >= 1)
  int64_t off[5];
  arrow_offsets<T>(d, off);
  const T xs = X(i, j, a, b);
  T y = (Fp[a * mv + a] + Fp[b * mv + b] - fo[i * no + i] - fo[j * no + j]) * xs;
  // virtual arrow (boxes whose two virtual indices run over all virtuals)
  if (box == B_T2 || box == B_S2 || box == B_H11 || box == B_H21) {
    if (a >= 1) y += u[a] * X(i, j, 0, b);
    if (b >= 1) y += X(i, j, a, 0) * u[b];
    if (a == 0) {
      const int64_t row = box == B_T2 ? off[0] : box == B_S2 ? off[1] : box == B_H11 ? off[3] : off[4];
      y += A.gv[row + (int64_t)batch * nv + b];
    }
    if (b == 0) {            // only S2 has b = 0 (the packed boxes keep a < b)
      y += A.gv[off[2] + (int64_t)batch * nv + a];
    }
  }
  // occupied arrow (boxes whose two occupied indices run over all occupied orbitals)
  if (box == B_T2 || box == B_S2 || box == B_H11 || box == B_H12) {
    T z = 0;
    if (i >= 1) z += w[i] * X(0, j, a, b);
    if (j >= 1) z += X(i, 0, a, b) * w[j];
    if (i == 0)
      for (int m = 1; m < no; ++m) z += w[m] * X(m, j, a, b);
    if (j == 0)
      for (int m = 1; m < no; ++m) z += X(i, m, a, b) * w[m];
    y -= z;
  }
  // transfer rows of the embedded H1P2 / H2P2 products, into (t', c) of H1P1 / H2P1
  if ((box == B_H11 || box == B_H21) && a == 0)
    y += G.side_tr[((box == B_H11 ? 0 : (int64_t)d.npo) + batch) * nv + b];
  y += couple_terms(G, P, box, batch, i, j, v);
  const int64_t g = d.off[box] + (int64_t)batch * inner + v;
  __builtin_nontemporal_store(y, G.y + g);
  return (box == B_S2 ? 1.0 : 2.0) * (double)G.x[g] * (double)y;     // weighted product for <x, y>_W
}

#define ESMP2_ARROW_INSTANCES(T)                                                        \
  template __global__ void k_arrow_side<T>(ArrowArgs<T>);                               \
  template __global__ void k_arrow<T>(ArrowArgs<T>, PairTables, const int4*, double*);
ESMP2_ARROW_INSTANCES(double)
ESMP2_ARROW_INSTANCES(float)
#undef ESMP2_ARROW_INSTANCES

}  // namespace esmp2
