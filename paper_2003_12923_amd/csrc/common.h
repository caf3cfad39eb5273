// Internal definitions shared by the HIP sources of libesmp2 (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include "esmp2.h"

namespace esmp2 {

// Sizes of one problem and the offsets of the seven amplitude boxes.
struct Dims {
  int no, nv, naux, n;   // occupied, virtual, auxiliary, total orbitals
  int npo;               // C(no,2)   occupied pairs
  int npo1;              // C(no-1,2) occupied pairs excluding t
  int npv;               // C(nv,2)   virtual pairs
  int npv1;              // C(nv-1,2) virtual pairs excluding t'
  int mv;                // nv rounded up to a multiple of 16 (padded virtual dimension)
  int sg;                // spin-flip sign of the first-order amplitudes: +1 singlet, -1 M_s = 0 triplet
  int64_t off[8];        // box offsets, off[7] = total amplitudes
};

enum Box { B_T2 = 0, B_S2 = 1, B_T3 = 2, B_H11 = 3, B_H12 = 4, B_H21 = 5, B_H22 = 6 };

inline Dims make_dims(int no, int nv, int naux) {
  Dims d;
  d.no = no; d.nv = nv; d.naux = naux; d.n = no + nv;
  d.npo = no * (no - 1) / 2;
  d.npo1 = (no - 1) * (no - 2) / 2;
  d.npv = nv * (nv - 1) / 2;
  d.npv1 = (nv - 1) * (nv - 2) / 2;
  d.mv = (nv + 15) / 16 * 16;
  d.sg = 1;
  int64_t s[7];
  s[0] = (int64_t)d.npo * d.npv;
  s[1] = (int64_t)no * no * nv * nv;
  s[2] = (int64_t)d.npo1 * d.npv1;
  s[3] = (int64_t)d.npo * d.npv;
  s[4] = (int64_t)d.npo * (nv - 1) * (nv - 1);
  s[5] = (int64_t)(no - 1) * (no - 1) * d.npv;
  s[6] = (int64_t)(no - 1) * (no - 1) * (nv - 1) * (nv - 1);
  d.off[0] = 0;
  for (int k = 0; k < 7; ++k) d.off[k + 1] = d.off[k] + s[k];
  return d;
}

// XCD-aware workgroup order.  The workgroups of one launch are dealt to the
// 8 XCDs round-robin (b -> XCD b % 8) and each XCD has its own L2.  Renumber
// them so that each XCD walks runs of C consecutive logical blocks (data
// shared by neighbouring blocks is fetched into one L2 once) while the runs
// still rotate over the XCDs (work of uneven cost stays balanced).  A
// bijection of [0, nblocks); the tail that does not fill 8 C blocks keeps
// its order.
template <unsigned C>
__device__ inline unsigned xcd_remap(unsigned b, unsigned nblocks) {
  const unsigned full = nblocks / (8u * C) * (8u * C);
  if (b >= full) return b;
  const unsigned x = b & 7u, r = b >> 3;
  return ((r / C) * 8u + x) * C + (r % C);
}

// Packed strict-upper-triangle index of (p,q), p<q, in an m x m matrix.
__host__ __device__ inline int tri_idx(int p, int q, int m) {
  return p * m - p * (p + 1) / 2 + (q - p - 1);
}

// Inverse of tri_idx: packed index -> (p,q).
__device__ inline void tri_pq(int idx, int m, int& p, int& q) {
  // p is the largest row with start(p) <= idx, start(p) = p*m - p(p+1)/2; a
  // single-precision estimate from the quadratic, made exact by the two loops
  const float mm = 2.0f * m - 1.0f;
  int pp = (int)floorf((mm - sqrtf(fmaxf(mm * mm - 8.0f * (float)idx, 0.0f))) * 0.5f);
  if (pp < 0) pp = 0;
  while (pp > 0 && pp * m - pp * (pp + 1) / 2 > idx) --pp;
  while ((pp + 1) * m - (pp + 1) * (pp + 2) / 2 <= idx) ++pp;
  p = pp;
  q = idx - (pp * m - pp * (pp + 1) / 2) + pp + 1;
}

}  // namespace esmp2

// Error helpers for host code.
#define ESMP2_HIP(call)                                                        \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) {                                                    \
      return fail(h, ESMP2_HIP_ERROR, std::string(#call) + ": " + hipGetErrorString(e_)); \
    }                                                                          \
  } while (0)
