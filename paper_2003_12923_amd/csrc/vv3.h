// Definitions shared by the Sylvester kernels (FP64 / FP32 operands in
// vv3.hip, BF16 operands in vv3b.hip): the per-job view of a batch matrix,
// element offsets with their factor codes, the output stores and the
// per-wavefront tile lists.
#pragma once
#include "common.h"
#include "mfma.h"
#include "sigma.h"

namespace esmp2 {

enum { K3_PACK = 0, K3_PACKRED = 1, K3_DENSERED = 2, K3_S2PAIR = 3, K3_S2DIAG = 4 };

template <class T>
struct V3Ctx {
  const T* src;          // batch storage (S~ for S2)
  T* dst;
  T* dstT;               // S2 pair: transposed destination
  T* tr;                 // H1P2/H2P2: transfer row
  const T* F;            // F' (mv x mv)
  int m;                 // storage dimension (nv or nv-1)
  T sg;                  // S2: the flip partner of batch (i, j) is sg times the transpose of (j, i)
};

// Element (r, c) of the embedded batch matrix as an in-bounds offset into c.src
// and a factor code f: 0 (outside the matrix or on the diagonal of a packed
// antisymmetric one: the element is zero), 1 (as stored), 2 (negated).  The
// load is issued at once and the factor applied only when the value is
// stashed in LDS, so that the load stays in flight across the matrix-core work.
template <int FMT, class T>
__device__ inline int x3_off(const V3Ctx<T>& c, int r, int col, int& f) {
  if (FMT == K3_PACK || FMT == K3_PACKRED) {
    const int off = (FMT == K3_PACKRED) ? 1 : 0;
    const int rr = r - off, cc = col - off;
    const bool ok = rr >= 0 && cc >= 0 && rr < c.m && cc < c.m && rr != cc;
    const int lo = min(rr, cc), hi = max(rr, cc);
    f = ok ? (rr < cc ? 1 : 2) : 0;
    return ok ? lo * c.m - lo * (lo + 1) / 2 + (hi - lo - 1) : 0;
  } else if (FMT == K3_DENSERED) {
    const int rr = r - 1, cc = col - 1;
    const bool ok = rr >= 0 && cc >= 0 && rr < c.m && cc < c.m;
    f = ok ? 1 : 0;
    return ok ? rr * c.m + cc : 0;
  } else {
    const bool ok = r < c.m && col < c.m;
    f = ok ? 1 : 0;
    return ok ? r * c.m + col : 0;
  }
}

template <class T>
__device__ inline T apply_code(T v, int f) {
  return f == 1 ? v : (f == 2 ? -v : T(0));
}

template <int FMT, class T>
__device__ inline void y3(const V3Ctx<T>& c, int r, int col, T val, bool diag_tile) {
  if (FMT == K3_PACK) {
    if (r < col && col < c.m) {
      c.dst[r * c.m - r * (r + 1) / 2 + (col - r - 1)] = val;
    }
  } else if (FMT == K3_PACKRED) {
    int rr = r - 1, cc = col - 1;
    if (rr >= 0 && rr < cc && cc < c.m) {
      c.dst[rr * c.m - rr * (rr + 1) / 2 + (cc - rr - 1)] = val;
    }
  } else if (FMT == K3_DENSERED) {
    if (col >= 1 && col <= c.m && r <= c.m) {
      if (r >= 1) {
        c.dst[(r - 1) * c.m + (col - 1)] = val;
      } else {
        c.tr[col] = val;
      }
    }
  } else if (FMT == K3_S2PAIR) {
    if (r < c.m && col < c.m) {
      c.dst[r * c.m + col] = val;
      c.dstT[col * c.m + r] = c.sg * val;
    }
  } else {
    if (r < c.m && col < c.m) {
      c.dst[r * c.m + col] = val;
      if (!diag_tile) c.dst[col * c.m + r] = c.sg * val;
    }
  }
}

// Output tiles of one batch matrix dealt to the 8 wavefronts (wavefront w runs
// on SIMD w % 4).  A single wavefront keeps the FP64 matrix core busy only
// about 40 % of the time, two interleaved ones about 90 %, so both
// wavefronts of a SIMD get the same number of tiles (within one) and keep the
// core fed together to the end of every K step.  Dense output: SIMD s takes a
// quadrant, its tiles in column-major order split in two halves.  Upper
// triangle (diagonal tiles included): all its tiles in column-major order cut
// into 8 consecutive runs, SIMD s taking runs 2s and 2s + 1.  A wavefront
// reads the A operands of its distinct tile rows and the B operands of its
// distinct tile columns.
template <int NT, bool TRI, int WAVE>
struct TileSet {
  int n = 0, nr = 0, nc = 0;                        // tiles, distinct tile rows, distinct tile columns
  int ti[32] = {}, tj[32] = {};                     // tile n = (ti[n], tj[n])
  int ri[32] = {}, ci[32] = {};                     // its row / column among rows[] / cols[]
  int rows[16] = {}, cols[16] = {};
  constexpr void add(int i, int j) {
    int a = -1, b = -1;
    for (int k = 0; k < nr; ++k)
      if (rows[k] == i) a = k;
    if (a < 0) { rows[nr] = i; a = nr++; }
    for (int k = 0; k < nc; ++k)
      if (cols[k] == j) b = k;
    if (b < 0) { cols[nc] = j; b = nc++; }
    ti[n] = i; tj[n] = j; ri[n] = a; ci[n] = b; ++n;
  }
  constexpr TileSet() {
    const int S = WAVE & 3, PART = WAVE >> 2;
    if (!TRI) {
      const int H = (NT + 1) / 2;
      const int r0 = (S >> 1) * H, r1 = (S >> 1) ? NT : H, c0 = (S & 1) * H, c1 = (S & 1) ? NT : H;
      const int half = ((r1 - r0) * (c1 - c0) + 1) / 2;
      int k = 0;
      for (int j = c0; j < c1; ++j)
        for (int i = r0; i < r1; ++i) {
          if ((k < half) == (PART == 0)) add(i, j);
          ++k;
        }
    } else {
      const int tot = NT * (NT + 1) / 2, g = 2 * S + PART;
      const int b0 = g * tot / 8, b1 = (g + 1) * tot / 8;
      int k = 0;
      for (int j = 0; j < NT; ++j)
        for (int i = 0; i <= j; ++i) {
          if (k >= b0 && k < b1) add(i, j);
          ++k;
        }
    }
  }
};

// job (box, batch or i, storage format code, j) -> its batch matrix in the operand buffers
template <class T>
__device__ inline V3Ctx<T> v3_ctx(const VVArgs<T>& A, int4 jb) {
  const Dims& d = A.d;
  const int box = jb.x;
  V3Ctx<T> c;
  c.F = (box == B_T2 || box == B_S2) ? A.Fd : A.Fl;
  c.dstT = nullptr;
  c.tr = nullptr;
  c.sg = T(d.sg);
  if (box == B_S2) {
    const int si = jb.y, sj = jb.w;
    c.m = d.nv;
    c.src = A.S + ((int64_t)si * d.no + sj) * d.nv * d.nv;
    c.dst = A.y + d.off[B_S2] + ((int64_t)si * d.no + sj) * d.nv * d.nv;
    c.dstT = A.y + d.off[B_S2] + ((int64_t)sj * d.no + si) * d.nv * d.nv;
  } else {
    int64_t o = d.off[box];
    const int batch = jb.y;
    if (box == B_T3) { c.m = d.nv - 1; o += (int64_t)batch * d.npv1; }
    else if (box == B_H12 || box == B_H22) {
      c.m = d.nv - 1;
      o += (int64_t)batch * (d.nv - 1) * (d.nv - 1);
      c.tr = A.side_tr + ((box == B_H12 ? 0 : d.npo) + (int64_t)batch) * d.nv;
    } else { c.m = d.nv; o += (int64_t)batch * d.npv; }
    c.src = A.x + o;
    c.dst = A.y + o;
  }
  return c;
}

}  // namespace esmp2
