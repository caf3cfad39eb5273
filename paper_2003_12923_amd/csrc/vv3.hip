// Specialised Sylvester kernel Y = F' X + X F' on FP64 matrix cores for the
// padded virtual dimension mv = 16 * NT (NT <= 10 tiles), one batch matrix per
// workgroup of 4 wavefronts.  Everything that varies per job -- the storage
// format of X, the output symmetry, and the block of 16x16 output tiles a
// wavefront owns -- is a template parameter, so the matrix-core loop is
// straight-line code.  K runs over 2*mv (k < mv: A = F', B = X; k >= mv:
// A = X, B = F') in 16-wide chunks staged through double-buffered LDS; the
// next chunk is loaded into registers while the current one is multiplied.
#include "common.h"
#include "mfma.h"
#include "sigma.h"

namespace esmp2 {

enum { K3_PACK = 0, K3_PACKRED = 1, K3_DENSERED = 2, K3_S2PAIR = 3, K3_S2DIAG = 4 };

struct V3Ctx {
  int box, bi, bj;       // box and the occupied indices of this batch (actual orbital indices)
  int o;                 // batch index within the box
  const GatherArgs* g;   // coupling terms (null: Sylvester part only)
  const double* src;     // batch storage (S~ for S2)
  double* dst;
  double* dstT;          // S2 pair: transposed destination
  double* tr;            // H1P2/H2P2: transfer row
  const double* F;       // F' (mv x mv)
  int m;                 // storage dimension (nv or nv-1)
  int nv;
};

// element (r, c) of the embedded batch matrix; branch-free select, in-bounds address
template <int FMT>
__device__ inline double x3(const V3Ctx& c, int r, int col) {
  if (FMT == K3_PACK || FMT == K3_PACKRED) {
    const int off = (FMT == K3_PACKRED) ? 1 : 0;
    int rr = r - off, cc = col - off;
    bool ok = rr >= 0 && cc >= 0 && rr < c.m && cc < c.m && rr != cc;
    int lo = min(rr, cc), hi = max(rr, cc);
    int idx = ok ? lo * c.m - lo * (lo + 1) / 2 + (hi - lo - 1) : 0;
    double v = c.src[idx];
    return ok ? (rr < cc ? v : -v) : 0.0;
  } else if (FMT == K3_DENSERED) {
    int rr = r - 1, cc = col - 1;
    bool ok = rr >= 0 && cc >= 0 && rr < c.m && cc < c.m;
    double v = c.src[ok ? rr * c.m + cc : 0];
    return ok ? v : 0.0;
  } else {
    bool ok = r < c.m && col < c.m;
    double v = c.src[ok ? r * c.m + col : 0];
    return ok ? v : 0.0;
  }
}

__device__ inline double special(const V3Ctx& c, int r, int col);

template <int FMT>
__device__ inline void y3(const V3Ctx& c, int r, int col, double val, bool diag_tile) {
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
      c.dstT[col * c.m + r] = val;
    }
  } else {
    if (r < c.m && col < c.m) {
            c.dst[r * c.m + col] = val;
      if (!diag_tile) c.dst[col * c.m + r] = val;
    }
  }
}

// Per-element couplings other than the occupied-index Fock action: pinned
// TOP-index transfers, doubles <-> L-triples through f_ov and the side
// contractions.  (r, col) are the actual virtual indices of the output.
__device__ inline double special(const V3Ctx& c, int r, int col) {
  const GatherArgs& A = *c.g;
  const Dims& d = A.d;
  const int no = d.no, nv = d.nv;
  Look L{d, A.x, A.S};
  const double* fo = A.fo;
  const double* fv = A.fv;
  auto FOV = [&](int i, int a) { return A.fov[i * nv + a]; };
  const double ftt = FOV(0, 0);
  double acc = 0.0;
  switch (c.box) {
    case B_T2: {
      const int i = c.bi, j = c.bj, a = r, b = col;
      if (i >= 1 && a >= 1) acc += ftt * L.T3(i, j, a, b);
      acc += ftt * L.H11(i, j, a, b);
      if (i == 0) {
        if (a >= 1)
          for (int m = 1; m < no; ++m) acc -= FOV(m, 0) * L.T3(m, j, a, b);
        for (int m = 1; m < no; ++m) acc += FOV(m, 0) * L.H21(m, j, a, b);
      }
      if (a == 0) {
        if (i >= 1) acc -= A.t3_t[tri_idx(i - 1, j - 1, no - 1) * nv + b];
        acc += A.h12_t[c.o * nv + b];
        if (i == 0)
          for (int m = 1; m < no; ++m) {
            if (m < j) acc += A.t3_p1[tri_idx(m - 1, j - 1, no - 1) * nv + b];
            else if (m > j) acc -= A.t3_p2[tri_idx(j - 1, m - 1, no - 1) * nv + b];
            acc += A.h22_i[((m - 1) * (no - 1) + (j - 1)) * nv + b];
          }
      }
      break;
    }
    case B_S2: {
      const int i = c.bi, j = c.bj, a = r, b = col;
      for (int rep = 0; rep < 2; ++rep) {
        int p = rep ? j : i, q = rep ? i : j, xx = rep ? b : a, z = rep ? a : b;
        if (p == 0 && xx == 0)
          for (int m = 0; m < no; ++m) {
            if (m < q) acc += A.h11_p1[tri_idx(m, q, no) * nv + z];
            else if (m > q) acc -= A.h11_p2[tri_idx(q, m, no) * nv + z];
          }
        if (p == 0 && xx >= 1 && z >= 1)
          for (int m = 0; m < no; ++m) acc += FOV(m, 0) * L.H12(m, q, xx, z);
        if (p == 0 && xx >= 1 && z == 0)
          for (int m = 0; m < no; ++m) {
            if (m < q) acc -= A.h12_u1[tri_idx(m, q, no) * nv + xx];
            else if (m > q) acc += A.h12_u2[tri_idx(q, m, no) * nv + xx];
          }
        if (p >= 1 && q >= 1 && xx == 0) acc += A.h21_t[((p - 1) * (no - 1) + (q - 1)) * nv + z];
        if (p >= 1 && q == 0 && xx == 0)
          for (int m = 1; m < no; ++m) acc -= A.h21_k[((p - 1) * (no - 1) + (m - 1)) * nv + z];
        if (p >= 1 && q >= 1 && xx >= 1 && z >= 1) acc += ftt * L.H22(p, q, xx, z);
        if (p >= 1 && q == 0 && xx >= 1 && z >= 1)
          for (int m = 1; m < no; ++m) acc -= FOV(m, 0) * L.H22(p, m, xx, z);
        if (p >= 1 && q >= 1 && xx >= 1 && z == 0) acc -= A.h22_ut[((p - 1) * (no - 1) + (q - 1)) * nv + xx];
        if (p >= 1 && q == 0 && xx >= 1 && z == 0)
          for (int m = 1; m < no; ++m) acc += A.h22_uk[((p - 1) * (no - 1) + (m - 1)) * nv + xx];
      }
      break;
    }
    case B_T3: {
      const int j = c.bi, k = c.bj, b = r, cc = col;
      acc += ftt * L.T2(j, k, b, cc) - FOV(j, 0) * L.T2(0, k, b, cc) + FOV(k, 0) * L.T2(0, j, b, cc)
           - FOV(0, b) * L.T2(j, k, 0, cc) + FOV(j, b) * L.T2(0, k, 0, cc) - FOV(k, b) * L.T2(0, j, 0, cc)
           + FOV(0, cc) * L.T2(j, k, 0, b) - FOV(j, cc) * L.T2(0, k, 0, b) + FOV(k, cc) * L.T2(0, j, 0, b);
      break;
    }
    case B_H11: {
      const int j = c.bi, k = c.bj, b = r, cc = col;
      if (j == 0)
        for (int m = 1; m < no; ++m) acc -= fo[m * no + 0] * L.H21(m, k, b, cc);
      acc += ftt * L.T2(j, k, b, cc);
      acc += FOV(j, b) * L.St(0, k, 0, cc) - FOV(k, b) * L.St(0, j, 0, cc)
           - FOV(j, cc) * L.St(0, k, 0, b) + FOV(k, cc) * L.St(0, j, 0, b);
      break;
    }
    case B_H12: {
      const int j = c.bi, k = c.bj, a = r, cc = col;
      acc += fv[a * nv + 0] * L.H11(j, k, 0, cc);
      if (j == 0)
        for (int m = 1; m < no; ++m) acc -= fo[m * no + 0] * L.H22(m, k, a, cc);
      acc += FOV(0, a) * L.T2(j, k, 0, cc);
      acc += FOV(j, 0) * L.St(0, k, a, cc) - FOV(k, 0) * L.St(0, j, a, cc)
           - FOV(j, cc) * L.St(0, k, a, 0) + FOV(k, cc) * L.St(0, j, a, 0);
      break;
    }
    case B_H21: {
      const int i = c.bi, k = c.bj, b = r, cc = col;
      acc -= fo[0 * no + i] * L.H11(0, k, b, cc);
      acc += FOV(i, 0) * L.T2(0, k, b, cc);
      acc += FOV(0, b) * L.St(i, k, 0, cc) - FOV(k, b) * L.St(i, 0, 0, cc)
           - FOV(0, cc) * L.St(i, k, 0, b) + FOV(k, cc) * L.St(i, 0, 0, b);
      break;
    }
    default: {
      const int i = c.bi, k = c.bj, a = r, cc = col;
      acc -= fo[0 * no + i] * L.H12(0, k, a, cc);
      acc += fv[a * nv + 0] * L.H21(i, k, 0, cc);
      acc += FOV(i, a) * L.T2(0, k, 0, cc);
      acc += ftt * L.St(i, k, a, cc) - FOV(k, 0) * L.St(i, 0, a, cc)
           - FOV(0, cc) * L.St(i, k, a, 0) + FOV(k, cc) * L.St(i, 0, a, 0);
      break;
    }
  }
  return acc;
}

// tile block owned by a wavefront
template <int NT, bool TRIKIND, int WAVE>
struct WRect {
  static constexpr int H = (NT + 1) / 2;
  static constexpr int SPLIT = H + (NT - H) / 2;
  static constexpr int R0 = TRIKIND ? (WAVE == 3 ? H : 0) : ((WAVE >> 1) * H);
  static constexpr int R1 = TRIKIND ? (WAVE == 3 ? NT : H) : ((WAVE >> 1) ? NT : H);
  static constexpr int C0 = TRIKIND ? (WAVE == 0 ? 0 : WAVE == 1 ? SPLIT : H) : ((WAVE & 1) * H);
  static constexpr int C1 = TRIKIND ? (WAVE == 0 ? H : WAVE == 1 ? NT : WAVE == 2 ? SPLIT : NT)
                                    : ((WAVE & 1) ? NT : H);
  static constexpr bool TRI = TRIKIND && (WAVE == 0 || WAVE == 3);
  static constexpr int NR = R1 - R0 > 0 ? R1 - R0 : 1;
  static constexpr int NC = C1 - C0 > 0 ? C1 - C0 : 1;
  static constexpr bool EMPTY = (R1 <= R0) || (C1 <= C0);
};

template <int FMT, int NT, int WAVE>
__device__ __attribute__((always_inline)) inline void vv3_body(const V3Ctx& c, double (*As)[16][16 * NT + 1],
                                                               double (*Bs)[16][16 * NT + 1]) {
  constexpr int MV = 16 * NT;
  constexpr bool TRIKIND = (FMT == K3_PACK || FMT == K3_PACKRED || FMT == K3_S2DIAG);
  using Rc = WRect<NT, TRIKIND, WAVE>;
  const int tid = threadIdx.x, l = tid & 63;
  f64x4 acc[Rc::NR][Rc::NC];
#pragma unroll
  for (int i = 0; i < Rc::NR; ++i)
#pragma unroll
    for (int j = 0; j < Rc::NC; ++j) acc[i][j] = (f64x4){0.0, 0.0, 0.0, 0.0};
  // staging map: A chunk (MV rows x 16 k): thread -> k = tid & 15, rows (tid >> 4) + 16 t;
  //              B chunk (16 k x MV cols): thread -> k = tid >> 4, cols (tid & 15) + 16 t
  double pa[NT], pb[NT];
  const int lo4 = tid & 15, hi4 = tid >> 4;
  auto fetch = [&](int k0) {
    const bool second = k0 >= MV;
    const int kb = second ? k0 - MV : k0;
    if (second) {
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        pa[t] = x3<FMT>(c, hi4 + 16 * t, kb + lo4);
        pb[t] = c.F[(kb + hi4) * MV + lo4 + 16 * t];
      }
    } else {
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        pa[t] = c.F[(hi4 + 16 * t) * MV + kb + lo4];
        pb[t] = x3<FMT>(c, kb + hi4, lo4 + 16 * t);
      }
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      As[buf][lo4][hi4 + 16 * t] = pa[t];
      Bs[buf][hi4][lo4 + 16 * t] = pb[t];
    }
  };
  constexpr int NCH = 2 * MV / 16;
  fetch(0);
  stash(0);
  fetch(16);
  __syncthreads();
  for (int q = 0; q < NCH; ++q) {
    const int buf = q & 1;
    if (!Rc::EMPTY) {
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        double a[Rc::NR], b[Rc::NC];
#pragma unroll
        for (int t = 0; t < Rc::NR; ++t) a[t] = As[buf][ks * 4 + (l >> 4)][(Rc::R0 + t) * 16 + (l & 15)];
#pragma unroll
        for (int t = 0; t < Rc::NC; ++t) b[t] = Bs[buf][ks * 4 + (l >> 4)][(Rc::C0 + t) * 16 + (l & 15)];
#pragma unroll
        for (int i = 0; i < Rc::NR; ++i)
#pragma unroll
          for (int j = 0; j < Rc::NC; ++j)
            if (!Rc::TRI || Rc::C0 + j >= Rc::R0 + i) acc[i][j] = mfma16x16x4(a[i], b[j], acc[i][j]);
      }
    }
    if (q + 1 < NCH) {
      stash(buf ^ 1);                       // chunk q+1 (loaded during the previous iteration)
      if (q + 2 < NCH) fetch((q + 2) * 16);
    }
    __syncthreads();
  }
  if (Rc::EMPTY) return;
#pragma unroll
  for (int i = 0; i < Rc::NR; ++i)
#pragma unroll
    for (int j = 0; j < Rc::NC; ++j) {
      if (Rc::TRI && Rc::C0 + j < Rc::R0 + i) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = (Rc::R0 + i) * 16 + mfma_row(l, q), col = (Rc::C0 + j) * 16 + (l & 15);
        y3<FMT>(c, r, col, acc[i][j][q], Rc::R0 + i == Rc::C0 + j);
      }
    }
}

// y += couplings for every output of this batch; rows by wavefront, columns by lane.
__device__ __attribute__((noinline)) void couplings_pass(V3Ctx c, int fmt) {
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int m = c.m;
  if (fmt == K3_PACK || fmt == K3_PACKRED) {
    const int off = (fmt == K3_PACKRED) ? 1 : 0;
    for (int r = wave; r < m; r += 4) {
      const int base = r * m - r * (r + 1) / 2 - r - 1;
      for (int col = r + 1 + l; col < m; col += 64) c.dst[base + col] += special(c, r + off, col + off);
    }
  } else if (fmt == K3_DENSERED) {
    for (int r = wave; r < m; r += 4)
      for (int col = l; col < m; col += 64) c.dst[r * m + col] += special(c, r + 1, col + 1);
  } else {
    for (int r = wave; r < m; r += 4)
      for (int col = l; col < m; col += 64) c.dst[r * m + col] += special(c, r, col);
    if (fmt == K3_S2PAIR) {
      V3Ctx t = c;
      t.bi = c.bj; t.bj = c.bi;
      for (int r = wave; r < m; r += 4)
        for (int col = l; col < m; col += 64) c.dstT[r * m + col] += special(t, r, col);
    }
  }
}

template <int FMT, int NT>
__device__ inline void vv3_dispatch(const V3Ctx& c, double (*As)[16][16 * NT + 1], double (*Bs)[16][16 * NT + 1]) {
  switch (threadIdx.x >> 6) {
    case 0: vv3_body<FMT, NT, 0>(c, As, Bs); break;
    case 1: vv3_body<FMT, NT, 1>(c, As, Bs); break;
    case 2: vv3_body<FMT, NT, 2>(c, As, Bs); break;
    default: vv3_body<FMT, NT, 3>(c, As, Bs); break;
  }
}

// jobs4: (box, batch or i, format code, j)
template <int NT>
__global__ __launch_bounds__(256) void k_vv3(VVArgs A) {
  __shared__ double As[2][16][16 * NT + 1];
  __shared__ double Bs[2][16][16 * NT + 1];
  const int4 jb = A.jobs4[blockIdx.x];
  const Dims& d = A.d;
  const int box = jb.x, fmt = jb.z;
  V3Ctx c;
  c.nv = d.nv;
  c.box = box;
  c.g = A.use_ga ? &A.ga : nullptr;
  c.o = jb.y;
  c.F = (box == B_T2 || box == B_S2) ? A.Fd : A.Fl;
  c.dstT = nullptr;
  c.tr = nullptr;
  if (box == B_S2) {
    const int si = jb.y, sj = jb.w;
    c.bi = si; c.bj = sj;
    c.m = d.nv;
    c.src = A.S + ((int64_t)si * d.no + sj) * d.nv * d.nv;
    c.dst = A.y + d.off[B_S2] + ((int64_t)si * d.no + sj) * d.nv * d.nv;
    c.dstT = A.y + d.off[B_S2] + ((int64_t)sj * d.no + si) * d.nv * d.nv;
  } else {
    int64_t o = d.off[box];
    const int batch = jb.y;
    if (box == B_T2 || box == B_H11 || box == B_H12) { tri_pq(batch, d.no, c.bi, c.bj); }
    else if (box == B_T3) { tri_pq(batch, d.no - 1, c.bi, c.bj); c.bi += 1; c.bj += 1; }
    else { c.bi = batch / (d.no - 1) + 1; c.bj = batch % (d.no - 1) + 1; }
    if (box == B_T3) { c.m = d.nv - 1; o += (int64_t)batch * d.npv1; }
    else if (box == B_H12 || box == B_H22) {
      c.m = d.nv - 1;
      o += (int64_t)batch * (d.nv - 1) * (d.nv - 1);
      c.tr = A.side_tr + ((box == B_H12 ? 0 : d.npo) + (int64_t)batch) * d.nv;
    } else { c.m = d.nv; o += (int64_t)batch * d.npv; }
    c.src = A.x + o;
    c.dst = A.y + o;
  }
  switch (fmt) {
    case K3_PACK: vv3_dispatch<K3_PACK, NT>(c, As, Bs); break;
    case K3_PACKRED: vv3_dispatch<K3_PACKRED, NT>(c, As, Bs); break;
    case K3_DENSERED: vv3_dispatch<K3_DENSERED, NT>(c, As, Bs); break;
    case K3_S2PAIR: vv3_dispatch<K3_S2PAIR, NT>(c, As, Bs); break;
    default: vv3_dispatch<K3_S2DIAG, NT>(c, As, Bs); break;
  }
}

// Coupling terms (everything except the two Fock contractions over the free
// index pairs) for every output: one workgroup per batch matrix; y += ...
// jobs: (box, batch) for every batch of every box; S2 batches are (i, j).
__global__ __launch_bounds__(256) void k_couple(GatherArgs G, const int2* jobs) {
  const int2 jb = jobs[blockIdx.x];
  const Dims& d = G.d;
  const int box = jb.x, batch = jb.y;
  V3Ctx c;
  c.box = box;
  c.g = &G;
  c.o = batch;
  c.nv = d.nv;
  c.tr = nullptr;
  c.dstT = nullptr;
  int fmt;
  int64_t o = d.off[box];
  switch (box) {
    case B_T2: case B_H11: tri_pq(batch, d.no, c.bi, c.bj); c.m = d.nv; o += (int64_t)batch * d.npv; fmt = K3_PACK; break;
    case B_T3: tri_pq(batch, d.no - 1, c.bi, c.bj); c.bi += 1; c.bj += 1; c.m = d.nv - 1;
               o += (int64_t)batch * d.npv1; fmt = K3_PACKRED; break;
    case B_H12: tri_pq(batch, d.no, c.bi, c.bj); c.m = d.nv - 1; o += (int64_t)batch * (d.nv - 1) * (d.nv - 1);
                fmt = K3_DENSERED; break;
    case B_S2: c.bi = batch / d.no; c.bj = batch % d.no; c.m = d.nv; o += (int64_t)batch * d.nv * d.nv;
               fmt = K3_S2DIAG; break;
    default: c.bi = batch / (d.no - 1) + 1; c.bj = batch % (d.no - 1) + 1; c.m = d.nv - 1;
             o += (int64_t)batch * (box == B_H21 ? d.npv : (d.nv - 1) * (d.nv - 1));
             fmt = (box == B_H21) ? K3_PACK : K3_DENSERED;
             if (box == B_H21) c.m = d.nv;
             break;
  }
  c.dst = G.y + o;
  couplings_pass(c, fmt);
}

template __global__ void k_vv3<10>(VVArgs);
template __global__ void k_vv3<7>(VVArgs);
template __global__ void k_vv3<5>(VVArgs);

}  // namespace esmp2
