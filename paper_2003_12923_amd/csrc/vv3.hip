// Specialised Sylvester kernel Y = F' X + X F' on the matrix cores for the
// padded virtual dimension mv = 16 * NT (NT <= 10 tiles), one batch matrix per
// workgroup of 8 wavefronts, two per SIMD, each with its own list of 16x16
// output tiles (balanced within every SIMD).  Everything that varies per job
// -- the storage format of X, the output symmetry, the tiles a wavefront owns
// -- is a template parameter, so the matrix-core loop is straight-line code.
// K runs over 2*mv (k < mv: A = F', B = X; k >= mv: A = X, B = F') in 16-wide
// chunks staged through double-buffered LDS, the loads of later chunks in
// flight while the current one is multiplied.
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

// One batch matrix, one wavefront's tiles.  K runs over 2*mv in chunks of 16
// (k < mv: A = F', B = X; k >= mv: A = X, B = F'), each chunk staged in one of
// two LDS buffers while the other is multiplied.  The X operand (an HBM
// stream, long load latency) is loaded three chunks ahead into two register
// sets that alternate; the F' operand (the same for every job, so L2
// resident) two chunks ahead.  F' is symmetric, so its A slab (first half)
// and B slab (second half) are both read as rows of F'.
template <class T, int FMT, int NT, int WAVE>
__device__ __attribute__((always_inline)) inline void vv3_body(const V3Ctx<T>& c, T (*As)[16][16 * NT + 1],
                                                               T (*Bs)[16][16 * NT + 1]) {
  constexpr int MV = 16 * NT;
  constexpr bool TRIKIND = (FMT == K3_PACK || FMT == K3_PACKRED || FMT == K3_S2DIAG);
  constexpr TileSet<NT, TRIKIND, WAVE> TS{};
  static_assert(TS.n > 0, "every wavefront owns at least one tile");
  const int tid = threadIdx.x, l = tid & 63;
  typedef typename MfmaAcc<T>::type AccT;
  AccT acc[TS.n];
#pragma unroll
  for (int i = 0; i < TS.n; ++i) acc[i] = AccT{0, 0, 0, 0};
  // staging map (512 threads), t < ceil(NT / 2):
  //   F' slab and the X B slab (first half): k = tid >> 5, columns (tid & 31) + 32 t
  //   X A slab (second half): k = tid & 15, rows (tid >> 4) + 32 t
  // X values are loaded raw and their factor codes (2 bits per value) applied
  // when stashed.  Rows / columns beyond MV (odd NT) load element 0 and are
  // not stashed.
  constexpr int NS = (NT + 1) / 2;
  T rf[NS], rx0[NS], rx1[NS];
  int fx0 = 0, fx1 = 0;
  const int ka = tid & 15, ra = tid >> 4, kb4 = tid >> 5, cb = tid & 31;
  auto fetchF = [&](int k0) {
    const int kb = k0 >= MV ? k0 - MV : k0;
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      const int col = cb + 32 * t;
      const bool okc = (2 * NS == NT) || col < MV;
      rf[t] = c.F[okc ? (kb + kb4) * MV + col : 0];
    }
  };
  auto stashF = [&](int k0, int buf) {
    T (*D)[16 * NT + 1] = k0 >= MV ? Bs[buf] : As[buf];
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      const int col = cb + 32 * t;
      if ((2 * NS == NT) || col < MV) D[kb4][col] = rf[t];
    }
  };
  auto fetchX = [&](int k0, T* rx, int& fx) {
    const bool second = k0 >= MV;
    const int kb = second ? k0 - MV : k0;
    fx = 0;
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      int f;
      if (second) {
        const int r = ra + 32 * t;
        const bool okr = (2 * NS == NT) || r < MV;
        const int o = x3_off<FMT, T>(c, r, kb + ka, f);
        rx[t] = c.src[o];
        fx |= (okr ? f : 0) << (2 * t);
      } else {
        const int col = cb + 32 * t;
        const bool okc = (2 * NS == NT) || col < MV;
        const int o = x3_off<FMT, T>(c, kb + kb4, col, f);
        rx[t] = c.src[o];
        fx |= (okc ? f : 0) << (2 * t);
      }
    }
  };
  auto stashX = [&](int k0, int buf, const T* rx, int fx) {
    const bool second = k0 >= MV;
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      const T v = apply_code(rx[t], (fx >> (2 * t)) & 3);
      if (second) {
        const int r = ra + 32 * t;
        if ((2 * NS == NT) || r < MV) As[buf][ka][r] = v;
      } else {
        const int col = cb + 32 * t;
        if ((2 * NS == NT) || col < MV) Bs[buf][kb4][col] = v;
      }
    }
  };
  constexpr int NCH = 2 * MV / 16;                 // even, >= 10 for every instantiated NT
  // Chunk q from LDS buffer BUF = q % 2.  STAGE 3: stash chunk q+1 (F' and X,
  // the X values in register set (q+1) % 2 = BUF ^ 1), then load F' of chunk
  // q+2 and X of chunk q+3 into that register set; 2: no X load; 1: stash
  // only; 0: nothing.  The staging sits between the matrix-core groups, at a
  // K step that differs between the two wavefronts of a SIMD, so that one
  // wavefront's staging overlaps the other's matrix-core work.  Buffer,
  // register set and stage are compile-time, so the loop body has no
  // branches and the accumulators stay in place.
  auto chunk = [&](int q, auto buf_c, auto stage_c) {
    constexpr int BUF = decltype(buf_c)::value, STAGE = decltype(stage_c)::value;
    constexpr int KST = (WAVE >> 2) ? 2 : 0;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      T a[TS.nr], b[TS.nc];
#pragma unroll
      for (int t = 0; t < TS.nr; ++t) a[t] = As[BUF][ks * 4 + (l >> 4)][TS.rows[t] * 16 + (l & 15)];
#pragma unroll
      for (int t = 0; t < TS.nc; ++t) b[t] = Bs[BUF][ks * 4 + (l >> 4)][TS.cols[t] * 16 + (l & 15)];
#pragma unroll
      for (int n = 0; n < TS.n; ++n) acc[n] = mfma16x16x4(a[TS.ri[n]], b[TS.ci[n]], acc[n]);
      if constexpr (STAGE >= 1) {
        if (ks == KST) {
          stashF((q + 1) * 16, BUF ^ 1);
          if constexpr (BUF == 0) stashX((q + 1) * 16, BUF ^ 1, rx1, fx1);
          else stashX((q + 1) * 16, BUF ^ 1, rx0, fx0);
        }
      }
      if constexpr (STAGE >= 2) {
        if (ks == KST + 1) {
          fetchF((q + 2) * 16);                    // before the X loads: the next stash waits on it alone
          if constexpr (STAGE >= 3) {
            if constexpr (BUF == 0) fetchX((q + 3) * 16, rx1, fx1);
            else fetchX((q + 3) * 16, rx0, fx0);
          }
        }
      }
    }
    __syncthreads();
  };
  using B0 = std::integral_constant<int, 0>;
  using B1 = std::integral_constant<int, 1>;
  using S0 = std::integral_constant<int, 0>;
  using S1 = std::integral_constant<int, 1>;
  using S2 = std::integral_constant<int, 2>;
  using S3 = std::integral_constant<int, 3>;
  // prologue: chunk 0 in LDS buffer 0, F' and X of chunk 1 and X of chunk 2 in flight
  fetchF(0);
  fetchX(0, rx0, fx0);
  stashF(0, 0);
  stashX(0, 0, rx0, fx0);
  fetchF(16);
  fetchX(16, rx1, fx1);
  fetchX(32, rx0, fx0);
  __syncthreads();
  for (int q = 0; q < NCH - 4; q += 2) {
    chunk(q, B0{}, S3{});
    chunk(q + 1, B1{}, S3{});
  }
  chunk(NCH - 4, B0{}, S3{});
  chunk(NCH - 3, B1{}, S2{});
  chunk(NCH - 2, B0{}, S1{});
  chunk(NCH - 1, B1{}, S0{});
#pragma unroll
  for (int n = 0; n < TS.n; ++n)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = TS.ti[n] * 16 + mfma_row_t<T>(l, q), col = TS.tj[n] * 16 + (l & 15);
      y3<FMT, T>(c, r, col, acc[n][q], TS.ti[n] == TS.tj[n]);
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
