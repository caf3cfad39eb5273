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
#include "vv3.h"

namespace esmp2 {

// One batch matrix, one wavefront's tiles.  K runs over 2*mv in chunks of 16
// (k < mv: A = F', B = X; k >= mv: A = X, B = F'; the two halves taken in
// turns), each chunk staged in one of two LDS buffers while the other is
// multiplied.  The X operand (an HBM
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
  // K order: the two halves interleaved (chunk q = 2c: F'X over k in [16c, 16c+16);
  // q = 2c+1: XF' over the same k), so that the second read of an X slab --
  // the same stored data for a packed antisymmetric or a symmetric batch, and
  // the same F' rows -- follows the first while it is still in L2
  auto K0 = [&](int q) { return (q & 1) ? MV + 16 * (q >> 1) : 16 * (q >> 1); };
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
          stashF(K0(q + 1), BUF ^ 1);
          if constexpr (BUF == 0) stashX(K0(q + 1), BUF ^ 1, rx1, fx1);
          else stashX(K0(q + 1), BUF ^ 1, rx0, fx0);
        }
      }
      if constexpr (STAGE >= 2) {
        if (ks == KST + 1) {
          fetchF(K0(q + 2));                    // before the X loads: the next stash waits on it alone
          if constexpr (STAGE >= 3) {
            if constexpr (BUF == 0) fetchX(K0(q + 3), rx1, fx1);
            else fetchX(K0(q + 3), rx0, fx0);
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
  fetchF(K0(0));
  fetchX(K0(0), rx0, fx0);
  stashF(K0(0), 0);
  stashX(K0(0), 0, rx0, fx0);
  fetchF(K0(1));
  fetchX(K0(1), rx1, fx1);
  fetchX(K0(2), rx0, fx0);
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
  const int fmt = jb.z;
  const V3Ctx<T> c = v3_ctx(A, jb);
  switch (fmt) {
    case K3_PACK: vv3_dispatch<T, K3_PACK, NT>(c, As, Bs); break;
    case K3_PACKRED: vv3_dispatch<T, K3_PACKRED, NT>(c, As, Bs); break;
    case K3_DENSERED: vv3_dispatch<T, K3_DENSERED, NT>(c, As, Bs); break;
    case K3_S2PAIR: vv3_dispatch<T, K3_S2PAIR, NT>(c, As, Bs); break;
    default: vv3_dispatch<T, K3_S2DIAG, NT>(c, As, Bs); break;
  }
}

// One instantiation per object file (the build compiles this source once per
// (type, NT) pair, in parallel): ESMP2_VV3_T and ESMP2_VV3_NT select it.
#if defined(ESMP2_VV3_T) && defined(ESMP2_VV3_NT)
template __global__ void k_vv3<ESMP2_VV3_T, ESMP2_VV3_NT>(VVArgs<ESMP2_VV3_T>);
#endif

}  // namespace esmp2
