// Specialised Sylvester kernel Y = F' X + X F' on FP64 matrix cores for the
// padded virtual dimension mv = 16 * NT (NT <= 10 tiles), one batch matrix per
// workgroup of 8 wavefronts, two per SIMD: the output tiles are dealt to the
// four SIMDs in blocks and each block is split between the SIMD's two
// wavefronts, so that one wavefront's LDS waits and staging overlap the
// other's matrix-core work (and each holds half the accumulators).
// Everything that varies per job -- the storage format of X, the output
// symmetry, and the block of 16x16 output tiles a wavefront owns -- is a
// template parameter, so the matrix-core loop is straight-line code.  K runs
// over 2*mv (k < mv: A = F', B = X; k >= mv: A = X, B = F') in 16-wide chunks
// staged through double-buffered LDS; the next chunk is loaded into registers
// while the current one is multiplied.
#include <type_traits>
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

constexpr int V3_THREADS = 512;

// rows of the first part when the upper triangle (diagonal included) of an
// n x n tile block is split by rows into two parts of nearly equal tile counts
constexpr int tri_split_rows(int n) {
  int acc = 0, r = 0;
  while (r < n && 2 * (acc + (n - r)) <= n * (n + 1) / 2 + (n - r)) { acc += n - r; ++r; }
  return r;
}

// tile block owned by a wavefront.  SIMD s = WAVE % 4 owns a block (one of the
// four quadrants of a dense output; for an upper-triangular output: the two
// diagonal triangles and two rectangles above them); wavefront WAVE / 4 of
// that SIMD takes the first or the second part of it (triangles split by rows,
// rectangles by columns).
template <int NT, bool TRIKIND, int WAVE>
struct WRect {
  static constexpr int S = WAVE & 3, PART = WAVE >> 2;
  static constexpr int H = (NT + 1) / 2;
  static constexpr int SPLIT = H + (NT - H) / 2;
  static constexpr int BR0 = TRIKIND ? (S == 3 ? H : 0) : ((S >> 1) * H);
  static constexpr int BR1 = TRIKIND ? (S == 3 ? NT : H) : ((S >> 1) ? NT : H);
  static constexpr int BC0 = TRIKIND ? (S == 0 ? 0 : S == 1 ? SPLIT : H) : ((S & 1) * H);
  static constexpr int BC1 = TRIKIND ? (S == 0 ? H : S == 1 ? NT : S == 2 ? SPLIT : NT) : ((S & 1) ? NT : H);
  static constexpr bool TRI = TRIKIND && (S == 0 || S == 3);
  static constexpr int RS = tri_split_rows(BR1 - BR0);        // triangle: rows of the first part
  static constexpr int CS = (BC1 - BC0 + 1) / 2;              // rectangle: columns of the first part
  static constexpr int R0 = TRI ? (PART ? BR0 + RS : BR0) : BR0;
  static constexpr int R1 = TRI ? (PART ? BR1 : BR0 + RS) : BR1;
  static constexpr int C0 = TRI ? (PART ? BC0 + RS : BC0) : (PART ? BC0 + CS : BC0);
  static constexpr int C1 = TRI ? BC1 : (PART ? BC1 : BC0 + CS);
  static constexpr int NR = R1 - R0 > 0 ? R1 - R0 : 1;
  static constexpr int NC = C1 - C0 > 0 ? C1 - C0 : 1;
  static constexpr bool EMPTY = (R1 <= R0) || (C1 <= C0);
};

template <class T, int FMT, int NT, int WAVE>
__device__ __attribute__((always_inline)) inline void vv3_body(const V3Ctx<T>& c, T (*As)[16][16 * NT + 1],
                                                               T (*Bs)[16][16 * NT + 1]) {
  constexpr int MV = 16 * NT;
  constexpr bool TRIKIND = (FMT == K3_PACK || FMT == K3_PACKRED || FMT == K3_S2DIAG);
  using Rc = WRect<NT, TRIKIND, WAVE>;
  const int tid = threadIdx.x, l = tid & 63;
  typedef typename MfmaAcc<T>::type AccT;
  AccT acc[Rc::NR][Rc::NC];
#pragma unroll
  for (int i = 0; i < Rc::NR; ++i)
#pragma unroll
    for (int j = 0; j < Rc::NC; ++j) acc[i][j] = AccT{0, 0, 0, 0};
  // staging map (512 threads): A chunk (MV rows x 16 k): thread -> k = tid & 15,
  //   rows (tid >> 4) + 32 t;  B chunk (16 k x MV cols): thread -> k = tid >> 5,
  //   cols (tid & 31) + 32 t;  t < ceil(NT / 2), rows / cols < MV
  // Raw values are loaded in fetch and their factor codes (2 bits per value in
  // fa / fb) applied in stash.  Rows / columns beyond MV (odd NT) load element 0
  // of F and are not stashed.
  constexpr int NS = (NT + 1) / 2;
  T pa[NS], pb[NS];
  int fa = 0, fb = 0;
  const int ka = tid & 15, ra = tid >> 4, kb4 = tid >> 5, cb = tid & 31;
  auto fetch = [&](int k0) {
    const bool second = k0 >= MV;
    const int kb = second ? k0 - MV : k0;
    fa = 0;
    fb = 0;
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      const int r = ra + 32 * t, col = cb + 32 * t;
      const bool okr = (2 * NS == NT) || r < MV, okc = (2 * NS == NT) || col < MV;
      int f;
      if (second) {
        const int o = x3_off<FMT, T>(c, r, kb + ka, f);
        pa[t] = c.src[o];
        fa |= (okr ? f : 0) << (2 * t);
        pb[t] = c.F[okc ? (kb + kb4) * MV + col : 0];
        fb |= (okc ? 1 : 0) << (2 * t);
      } else {
        pa[t] = c.F[okr ? r * MV + kb + ka : 0];
        fa |= (okr ? 1 : 0) << (2 * t);
        const int o = x3_off<FMT, T>(c, kb + kb4, col, f);
        pb[t] = c.src[o];
        fb |= (okc ? f : 0) << (2 * t);
      }
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      const int r = ra + 32 * t, col = cb + 32 * t;
      if ((2 * NS == NT) || r < MV) As[buf][ka][r] = apply_code(pa[t], (fa >> (2 * t)) & 3);
      if ((2 * NS == NT) || col < MV) Bs[buf][kb4][col] = apply_code(pb[t], (fb >> (2 * t)) & 3);
    }
  };
  constexpr int NCH = 2 * MV / 16;                 // even for every instantiated NT
  // One K chunk from LDS buffer BUF; with STASH / FETCH the staging of chunks
  // q+1 and q+2 is placed between the matrix-core groups, so that its loads
  // and LDS stores issue while the matrix cores are busy.  The buffer and the
  // staging switches are compile-time, so the loop body has no branches and
  // the accumulators stay in place across iterations.
  auto chunk = [&](int q, auto buf_c, auto stash_c, auto fetch_c) {
    constexpr int BUF = decltype(buf_c)::value;
    constexpr bool STASH = decltype(stash_c)::value, FETCH = decltype(fetch_c)::value;
    if constexpr (!Rc::EMPTY) {
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        T a[Rc::NR], b[Rc::NC];
#pragma unroll
        for (int t = 0; t < Rc::NR; ++t) a[t] = As[BUF][ks * 4 + (l >> 4)][(Rc::R0 + t) * 16 + (l & 15)];
#pragma unroll
        for (int t = 0; t < Rc::NC; ++t) b[t] = Bs[BUF][ks * 4 + (l >> 4)][(Rc::C0 + t) * 16 + (l & 15)];
#pragma unroll
        for (int i = 0; i < Rc::NR; ++i)
#pragma unroll
          for (int j = 0; j < Rc::NC; ++j)
            if (!Rc::TRI || Rc::C0 + j >= Rc::R0 + i) acc[i][j] = mfma16x16x4(a[i], b[j], acc[i][j]);
        if constexpr (STASH) { if (ks == 0) stash(BUF ^ 1); }     // chunk q+1 (loaded one chunk ago)
        if constexpr (FETCH) { if (ks == 1) fetch((q + 2) * 16); }
      }
    } else {
      if constexpr (STASH) stash(BUF ^ 1);
      if constexpr (FETCH) fetch((q + 2) * 16);
    }
    __syncthreads();
  };
  using B0 = std::integral_constant<int, 0>;
  using B1 = std::integral_constant<int, 1>;
  using Yes = std::true_type;
  using No = std::false_type;
  fetch(0);
  stash(0);
  fetch(16);
  __syncthreads();
  // the first pair of chunks outside the loop: the accumulators enter the loop
  // as matrix-core results rather than as the zero initialisation
  chunk(0, B0{}, Yes{}, Yes{});
  chunk(1, B1{}, Yes{}, Yes{});
  for (int q = 2; q < NCH - 2; q += 2) {
    chunk(q, B0{}, Yes{}, Yes{});
    chunk(q + 1, B1{}, Yes{}, Yes{});
  }
  chunk(NCH - 2, B0{}, Yes{}, No{});
  chunk(NCH - 1, B1{}, No{}, No{});
  if (Rc::EMPTY) return;
#pragma unroll
  for (int i = 0; i < Rc::NR; ++i)
#pragma unroll
    for (int j = 0; j < Rc::NC; ++j) {
      if (Rc::TRI && Rc::C0 + j < Rc::R0 + i) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = (Rc::R0 + i) * 16 + mfma_row_t<T>(l, q), col = (Rc::C0 + j) * 16 + (l & 15);
        y3<FMT, T>(c, r, col, acc[i][j][q], Rc::R0 + i == Rc::C0 + j);
      }
    }
}

template <class T, int FMT, int NT>
__device__ inline void vv3_dispatch(const V3Ctx<T>& c, T (*As)[16][16 * NT + 1], T (*Bs)[16][16 * NT + 1]) {
  switch (threadIdx.x >> 6) {
    case 0: vv3_body<T, FMT, NT, 0>(c, As, Bs); break;
    case 1: vv3_body<T, FMT, NT, 1>(c, As, Bs); break;
    case 2: vv3_body<T, FMT, NT, 2>(c, As, Bs); break;
    case 3: vv3_body<T, FMT, NT, 3>(c, As, Bs); break;
    case 4: vv3_body<T, FMT, NT, 4>(c, As, Bs); break;
    case 5: vv3_body<T, FMT, NT, 5>(c, As, Bs); break;
    case 6: vv3_body<T, FMT, NT, 6>(c, As, Bs); break;
    default: vv3_body<T, FMT, NT, 7>(c, As, Bs); break;
  }
}

// jobs4: (box, batch or i, format code, j)
template <class T, int NT>
__global__ __launch_bounds__(V3_THREADS, 1) void k_vv3(VVArgs<T> A) {
  __shared__ T As[2][16][16 * NT + 1];
  __shared__ T Bs[2][16][16 * NT + 1];
  const int4 jb = A.jobs4[blockIdx.x];
  const Dims& d = A.d;
  const int box = jb.x, fmt = jb.z;
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
  switch (fmt) {
    case K3_PACK: vv3_dispatch<T, K3_PACK, NT>(c, As, Bs); break;
    case K3_PACKRED: vv3_dispatch<T, K3_PACKRED, NT>(c, As, Bs); break;
    case K3_DENSERED: vv3_dispatch<T, K3_DENSERED, NT>(c, As, Bs); break;
    case K3_S2PAIR: vv3_dispatch<T, K3_S2PAIR, NT>(c, As, Bs); break;
    default: vv3_dispatch<T, K3_S2DIAG, NT>(c, As, Bs); break;
  }
}

template __global__ void k_vv3<double, 10>(VVArgs<double>);
template __global__ void k_vv3<double, 7>(VVArgs<double>);
template __global__ void k_vv3<double, 5>(VVArgs<double>);
template __global__ void k_vv3<float, 10>(VVArgs<float>);
template __global__ void k_vv3<float, 7>(VVArgs<float>);
template __global__ void k_vv3<float, 5>(VVArgs<float>);

}  // namespace esmp2
