// Per-batch matrix-vector products of the sigma kernels, one pass over each
// batch matrix X (the two virtual indices of one occupied batch of one box):
//   column sums  v[c] = sum_r w[r] X[r][c],   row sums  u[r] = sum_c X[r][c] w[c],
// with w a column of f_ov (the doubles <-> L-triples couplings) or, in the
// pinned-semicanonical basis, the t' row of the Fock block (the arrow terms
// and the transfer rows of the boxes without t').  Rows of X are staged
// through LDS 16 at a time with coalesced loads; a thread owns one column of
// the column sums, 16 lanes reduce a row for the row sums.  For a packed
// antisymmetric X only the upper triangle is read: its column sums minus its
// row sums give the column sums of the whole matrix.
#include "common.h"
#include "sigma.h"
#include "reduce.h"

namespace esmp2 {

template <class T>
struct GemvArgs {
  SideArgs<T> sd;        // x, f_ov, side-contraction outputs
  const T* S;            // flip-symmetrised S2
  const T* fv;           // F_vv (row 0: the t' row)
  T* gv;                 // arrow GEMVs (layout of ArrowArgs::gv)
  T* tr;                 // transfer rows
  int arrow;             // 0: side contractions only (TOP basis); 1: also the arrow GEMVs
};

constexpr int GV_MAXW = 3;     // weight vectors per pass

// MV: the largest virtual dimension the LDS arrays hold (160 or 192); with
// MV = 160 the FP64 kernel's LDS (32.1 KB) lets five workgroups share a CU.
template <class T, int MV>
__device__ __attribute__((always_inline)) inline void gemv_body(GemvArgs<T> A, int bid_, int nb_) {
  const SideArgs<T>& sd = A.sd;
  const Dims& d = sd.d;
  const int no = d.no, nv = d.nv, n2 = (no - 1) * (no - 1);
  __shared__ T tile[16][MV + 1];
  __shared__ T rowres[GV_MAXW][MV];
  // ---- job -> box, batch, occupied indices
  int job = bid_, box;
  if (job < d.npo1) box = B_T3;
  else if ((job -= d.npo1) < d.npo) box = B_H11;
  else if ((job -= d.npo) < d.npo) box = B_H12;
  else if ((job -= d.npo) < n2) box = B_H21;
  else if ((job -= n2) < n2) box = B_H22;
  else if ((job -= n2) < d.npo) box = B_T2;
  else { job -= d.npo; box = B_S2; }
  const int batch = job;
  int p, q;
  if (box == B_T3) { tri_pq(batch, no - 1, p, q); ++p; ++q; }
  else if (box == B_H11 || box == B_H12 || box == B_T2) tri_pq(batch, no, p, q);
  else if (box == B_S2) { p = batch / no; q = batch % no; }
  else { p = batch / (no - 1) + 1; q = batch % (no - 1) + 1; }
  // ---- storage of the batch matrix: m x m (packed upper or dense), virtual offset lo
  const bool anti = (box == B_T2 || box == B_T3 || box == B_H11 || box == B_H21);
  const int lo = (box == B_T3 || box == B_H12 || box == B_H22) ? 1 : 0;
  const int m = nv - lo;
  const T* X;
  switch (box) {
    case B_T2: X = sd.x + d.off[B_T2] + (int64_t)batch * d.npv; break;
    case B_S2: X = A.S + (int64_t)batch * nv * nv; break;
    case B_T3: X = sd.x + d.off[B_T3] + (int64_t)batch * d.npv1; break;
    case B_H11: X = sd.x + d.off[B_H11] + (int64_t)batch * d.npv; break;
    case B_H12: X = sd.x + d.off[B_H12] + (int64_t)batch * m * m; break;
    case B_H21: X = sd.x + d.off[B_H21] + (int64_t)batch * d.npv; break;
    default: X = sd.x + d.off[B_H22] + (int64_t)batch * m * m; break;
  }
  // ---- weight vectors (indexed by the actual virtual index) and outputs
  const T* fov = sd.fov;
  const T* u = A.fv;                   // u[c] = F[t'][c]; only c >= 1 enters
  const int64_t o = (int64_t)batch * nv;
  const T* wc[GV_MAXW] = {nullptr, nullptr, nullptr};   // column-sum weights (over the row index)
  T* oc[GV_MAXW] = {nullptr, nullptr, nullptr};
  const T* wr[GV_MAXW] = {nullptr, nullptr, nullptr};   // row-sum weights (over the column index)
  T* orow[GV_MAXW] = {nullptr, nullptr, nullptr};
  bool uc = false;                     // the column weight of slot 2 is u (zero at index 0)
  switch (box) {
    case B_T3:
      wc[0] = fov; oc[0] = sd.t3_t + o;
      wc[1] = fov + p * nv; oc[1] = sd.t3_p1 + o;
      wc[2] = fov + q * nv; oc[2] = sd.t3_p2 + o;
      break;
    case B_H11:
      wc[0] = fov + p * nv; oc[0] = sd.h11_p1 + o;
      wc[1] = fov + q * nv; oc[1] = sd.h11_p2 + o;
      if (A.arrow) { wc[2] = u; oc[2] = A.gv + ((int64_t)d.npo + 2 * no * no) * nv + o; uc = true; }
      break;
    case B_H12:
      wc[0] = fov; oc[0] = sd.h12_t + o;
      wr[0] = fov + p * nv; orow[0] = sd.h12_u1 + o;
      wr[1] = fov + q * nv; orow[1] = sd.h12_u2 + o;
      if (A.arrow) { wc[2] = u; oc[2] = A.tr + o; uc = true; }
      break;
    case B_H21:
      wc[0] = fov; oc[0] = sd.h21_t + o;
      wc[1] = fov + q * nv; oc[1] = sd.h21_k + o;
      if (A.arrow) { wc[2] = u; oc[2] = A.gv + (2 * (int64_t)d.npo + 2 * no * no) * nv + o; uc = true; }
      break;
    case B_H22:
      wr[0] = fov; orow[0] = sd.h22_ut + o;
      wr[1] = fov + q * nv; orow[1] = sd.h22_uk + o;
      wc[0] = fov + p * nv; oc[0] = sd.h22_i + o;
      if (A.arrow) { wc[2] = u; oc[2] = A.tr + ((int64_t)d.npo + batch) * nv; uc = true; }
      break;
    case B_T2:
      wc[2] = u; oc[2] = A.gv + o; uc = true;
      break;
    default:      // S2 (S~): g and h
      wc[2] = u; oc[2] = A.gv + (int64_t)d.npo * nv + o; uc = true;
      wr[2] = u; orow[2] = A.gv + ((int64_t)d.npo + no * no) * nv + o;
      break;
  }
  // weights in LDS (zero where a weight vector is absent or u at index 0)
  __shared__ T swc[GV_MAXW][MV], swr[GV_MAXW][MV];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int e = tid; e < GV_MAXW * MV; e += blockDim.x) {
    const int k = e / MV, i = e % MV;
    T vc = 0, vr = 0;
    if (i < nv) {
      if (wc[k] && !(uc && k == 2 && i == 0)) vc = wc[k][i];
      if (wr[k] && !(k == 2 && i == 0)) vr = wr[k][i];
    }
    swc[k][i] = vc;
    swr[k][i] = vr;
    rowres[k][i] = 0;
  }
  // an antisymmetric batch needs the row sums of its column weights as well
  const bool hasc[GV_MAXW] = {wc[0] != nullptr, wc[1] != nullptr, wc[2] != nullptr};
  const bool hasr[GV_MAXW] = {anti ? hasc[0] : wr[0] != nullptr, anti ? hasc[1] : wr[1] != nullptr,
                              anti ? hasc[2] : wr[2] != nullptr};
  const int c = tid;                   // column owned (storage index)
  T cacc[GV_MAXW] = {0, 0, 0};
  // rows r0..r0+15 of this thread's column (zeros below the diagonal of a packed batch)
  auto load_slab = [&](int r0, T* v) {
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
      const int r = r0 + rr;
      const bool ok = c < m && r < m && (!anti || c > r);
      const int64_t idx = !ok ? 0 : (anti ? (int64_t)(r * m - r * (r + 1) / 2 + (c - r - 1)) : (int64_t)r * m + c);
      const T x = X[idx];
      v[rr] = ok ? x : T(0);
    }
  };
  T v[16], vn[16];
  load_slab(0, v);
  for (int r0 = 0; r0 < m; r0 += 16) {
    __syncthreads();
    // the next slab's loads are in flight during the column and row sums of this one
    if (r0 + 16 < m) load_slab(r0 + 16, vn);
    // stage the slab; the thread of each column accumulates the column sums on the way
    if (c < m) {
#pragma unroll
      for (int rr = 0; rr < 16; ++rr) {
        const int r = r0 + rr;
        tile[rr][c] = v[rr];
        if (r < m) {
#pragma unroll
          for (int k = 0; k < GV_MAXW; ++k)
            if (hasc[k]) cacc[k] += swc[k][r + lo] * v[rr];
        }
      }
    }
    __syncthreads();
    // row sums: 16 lanes per staged row, each over every 16th column, then a
    // 4-step reduction inside the 16-lane group
    {
      const int rr = tid >> 4, seg = tid & 15;
#pragma unroll
      for (int k = 0; k < GV_MAXW; ++k) {
        if (!hasr[k]) continue;
        const T* w = anti ? swc[k] : swr[k];
        T sacc = 0;
#pragma unroll
        for (int i = 0; i < MV / 16; ++i) {       // m <= MV
          const int cc = seg + 16 * i;
          if (cc < m) sacc += tile[rr][cc] * w[cc + lo];
        }
        // sum over the 16-lane group (DPP: quads, then the mirrored quad and half)
        sacc += dpp_move<0xb1, 0xf>(sacc);
        sacc += dpp_move<0x4e, 0xf>(sacc);
        sacc += dpp_move<0x141, 0xf>(sacc);
        sacc += dpp_move<0x140, 0xf>(sacc);
        if (seg == 0 && r0 + rr < m) rowres[k][r0 + rr] = sacc;
      }
    }
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) v[rr] = vn[rr];
  }
  // column sums move from the thread of each storage column to the output threads through LDS
  __syncthreads();
  T* colres = &tile[0][0];               // reuse: [GV_MAXW][MV] fits in 16 x (MV + 1)
  if (c < m) {
#pragma unroll
    for (int k = 0; k < GV_MAXW; ++k) colres[k * MV + c] = cacc[k];
  }
  __syncthreads();
  if (c >= nv) return;
  // outputs over the actual virtual index c; storage index cs = c - lo (index 0 of a
  // batch without t' is zero)
  const int cs = c - lo;
  const bool in = cs >= 0 && cs < m;
#pragma unroll
  for (int k = 0; k < GV_MAXW; ++k) {
    if (oc[k]) oc[k][c] = in ? colres[k * MV + cs] - (anti ? rowres[k][cs] : T(0)) : T(0);
    if (orow[k] && !anti) orow[k][c] = in ? rowres[k][cs] : T(0);
  }
}

// five workgroups of 256 per CU where the LDS allows it (MV = 160): the whole
// grid of a c3-sized operator in one round
template <class T, int MV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MV <= 160 ? 5 : 4))) void k_gemv(GemvArgs<T> A) {
  gemv_body<T, MV>(A, blockIdx.x, gridDim.x);
}

template __global__ void k_gemv<double, 160>(GemvArgs<double>);
template __global__ void k_gemv<double, 192>(GemvArgs<double>);
template __global__ void k_gemv<float, 160>(GemvArgs<float>);
template __global__ void k_gemv<float, 192>(GemvArgs<float>);

}  // namespace esmp2
