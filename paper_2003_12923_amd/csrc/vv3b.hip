// Sylvester products Y = F' X + X F' with BF16 operands and FP32 accumulation
// on the matrix cores (v_mfma_f32_16x16x16_bf16): the operator of the
// BF16 precision.  Vectors and every other sigma kernel stay in FP32; F' and X
// are read in FP32 and rounded to BF16 (nearest even) when staged in LDS.
// Same job list, tile lists and prefetch depths as the FP64/FP32 kernel
// (X three chunks ahead in two register sets, F' two ahead); the LDS slabs
// hold 16 consecutive k of each row / column contiguously, the operand order of
// the 16x16x16 instruction.
//
// Operand layout of one 16x16x16 BF16 step (l = lane):
//   A (16 x 16): lane l holds A[l % 16][4 (l / 16) + i], i = 0..3
//   B (16 x 16): lane l holds B[4 (l / 16) + i][l % 16]
//   D: accumulator i of lane l holds D[4 (l / 16) + i][l % 16]
#include <type_traits>
#include "vv3.h"

namespace esmp2 {

typedef short bf16x4 __attribute__((ext_vector_type(4)));

__device__ inline unsigned bf16_bits(float f) {     // round to nearest even; finite inputs
  const unsigned u = __float_as_uint(f);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

// four FP32 values as four packed BF16 (two 32-bit words)
__device__ inline uint2 pack_bf16x4(float a, float b, float c, float d) {
  return make_uint2(bf16_bits(a) | (bf16_bits(b) << 16), bf16_bits(c) | (bf16_bits(d) << 16));
}

constexpr int B3_PITCH = 20;      // BF16 per staged row: 16 k and 4 of padding (40 bytes)

template <int FMT, int NT, int WAVE>
__device__ __attribute__((always_inline)) inline void vv3b_body(const V3Ctx<float>& c, unsigned short* lds) {
  constexpr int MV = 16 * NT;
  constexpr int SLAB = MV * B3_PITCH;              // one slab: MV rows (or columns) x 16 k
  constexpr int BUFSZ = 2 * SLAB;                  // A slab, then B slab
  constexpr bool TRIKIND = (FMT == K3_PACK || FMT == K3_PACKRED || FMT == K3_S2DIAG);
  constexpr TileSet<NT, TRIKIND, WAVE> TS{};
  static_assert(TS.n > 0, "every wavefront owns at least one tile");
  const int tid = threadIdx.x, l = tid & 63;
  f32x4 acc[TS.n];
#pragma unroll
  for (int i = 0; i < TS.n; ++i) acc[i] = f32x4{0, 0, 0, 0};
  // staging items: a slab has MV x 4 quads of 4 consecutive k; thread tid takes
  // items tid + 512 u.  F' slabs and the X A slab: item q -> (row q >> 2, quad
  // q & 3); the X B slab (first half): item q -> (column q % MV, quad q / MV),
  // so that consecutive lanes read consecutive columns of an X row.
  constexpr int NQ = 4 * MV, NI = (NQ + V3_THREADS - 1) / V3_THREADS;
  float4 rf[NI];
  float rx0[NI][4], rx1[NI][4];
  int fx0 = 0, fx1 = 0;
  auto fetchF = [&](int k0) {
    const int kb = k0 >= MV ? k0 - MV : k0;
#pragma unroll
    for (int u = 0; u < NI; ++u) {
      const int q = tid + V3_THREADS * u;
      const bool ok = q < NQ;
      // F' is symmetric: both slabs are 16 consecutive entries of a row of F'
      const int o = ok ? (q >> 2) * MV + kb + 4 * (q & 3) : 0;
      rf[u] = *reinterpret_cast<const float4*>(c.F + o);
    }
  };
  auto stashF = [&](int k0, int buf) {
    unsigned short* D = lds + buf * BUFSZ + (k0 >= MV ? SLAB : 0);
#pragma unroll
    for (int u = 0; u < NI; ++u) {
      const int q = tid + V3_THREADS * u;
      if (q < NQ)
        *reinterpret_cast<uint2*>(D + (q >> 2) * B3_PITCH + 4 * (q & 3)) = pack_bf16x4(rf[u].x, rf[u].y, rf[u].z, rf[u].w);
    }
  };
  auto fetchX = [&](int k0, float (*rx)[4], int& fx) {
    const bool second = k0 >= MV;
    const int kb = second ? k0 - MV : k0;
    fx = 0;
#pragma unroll
    for (int u = 0; u < NI; ++u) {
      const int q = tid + V3_THREADS * u;
      const bool ok = q < NQ;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int f;
        int o;
        if (second) o = x3_off<FMT, float>(c, q >> 2, kb + 4 * (q & 3) + i, f);      // X[row][k]
        else o = x3_off<FMT, float>(c, kb + 4 * (q / MV) + i, q % MV, f);            // X[k][column]
        rx[u][i] = c.src[o];
        fx |= (ok ? f : 0) << (2 * (4 * u + i));
      }
    }
  };
  auto stashX = [&](int k0, int buf, const float (*rx)[4], int fx) {
    const bool second = k0 >= MV;
    unsigned short* D = lds + buf * BUFSZ + (second ? 0 : SLAB);
#pragma unroll
    for (int u = 0; u < NI; ++u) {
      const int q = tid + V3_THREADS * u;
      if (q < NQ) {
        float v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = apply_code(rx[u][i], (fx >> (2 * (4 * u + i))) & 3);
        const int e = second ? (q >> 2) * B3_PITCH + 4 * (q & 3) : (q % MV) * B3_PITCH + 4 * (q / MV);
        *reinterpret_cast<uint2*>(D + e) = pack_bf16x4(v[0], v[1], v[2], v[3]);
      }
    }
  };
  constexpr int NCH = 2 * MV / 16;
  // K order: the two halves interleaved (chunk q = 2c: F'X over k in [16c, 16c+16);
  // q = 2c+1: XF' over the same k), so that the second read of an X slab --
  // the same stored data for a packed antisymmetric or a symmetric batch, and
  // the same F' rows -- follows the first while it is still in L2
  auto K0 = [&](int q) { return (q & 1) ? MV + 16 * (q >> 1) : 16 * (q >> 1); };
  auto chunk = [&](int q, auto buf_c, auto stage_c) {
    constexpr int BUF = decltype(buf_c)::value, STAGE = decltype(stage_c)::value;
    const unsigned short* A = lds + BUF * BUFSZ;
    const unsigned short* B = A + SLAB;
    bf16x4 a[TS.nr], b[TS.nc];
#pragma unroll
    for (int t = 0; t < TS.nr; ++t)
      a[t] = *reinterpret_cast<const bf16x4*>(A + (TS.rows[t] * 16 + (l & 15)) * B3_PITCH + 4 * (l >> 4));
#pragma unroll
    for (int t = 0; t < TS.nc; ++t)
      b[t] = *reinterpret_cast<const bf16x4*>(B + (TS.cols[t] * 16 + (l & 15)) * B3_PITCH + 4 * (l >> 4));
#pragma unroll
    for (int n = 0; n < TS.n; ++n)
      acc[n] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[TS.ri[n]], b[TS.ci[n]], acc[n], 0, 0, 0);
    if constexpr (STAGE >= 1) {
      stashF(K0(q + 1), BUF ^ 1);
      if constexpr (BUF == 0) stashX(K0(q + 1), BUF ^ 1, rx1, fx1);
      else stashX(K0(q + 1), BUF ^ 1, rx0, fx0);
    }
    if constexpr (STAGE >= 2) {
      fetchF(K0(q + 2));
      if constexpr (STAGE >= 3) {
        if constexpr (BUF == 0) fetchX(K0(q + 3), rx1, fx1);
        else fetchX(K0(q + 3), rx0, fx0);
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
    for (int qq = 0; qq < 4; ++qq) {
      const int r = TS.ti[n] * 16 + mfma_row_t<float>(l, qq), col = TS.tj[n] * 16 + (l & 15);
      y3<FMT, float>(c, r, col, acc[n][qq], TS.ti[n] == TS.tj[n]);
    }
}

template <int FMT, int NT>
__device__ inline void vv3b_dispatch(const V3Ctx<float>& c, unsigned short* lds) {
  switch (threadIdx.x >> 6) {
    case 0: vv3b_body<FMT, NT, 0>(c, lds); break;
    case 1: vv3b_body<FMT, NT, 1>(c, lds); break;
    case 2: vv3b_body<FMT, NT, 2>(c, lds); break;
    case 3: vv3b_body<FMT, NT, 3>(c, lds); break;
    case 4: vv3b_body<FMT, NT, 4>(c, lds); break;
    case 5: vv3b_body<FMT, NT, 5>(c, lds); break;
    case 6: vv3b_body<FMT, NT, 6>(c, lds); break;
    default: vv3b_body<FMT, NT, 7>(c, lds); break;
  }
}

template <int NT>
__global__ __launch_bounds__(V3_THREADS, 1) void k_vv3b(VVArgs<float> A) {
  __shared__ __align__(16) unsigned short lds[2 * 2 * 16 * NT * B3_PITCH];
  const V3Ctx<float> c = v3_ctx(A, A.jobs4[blockIdx.x]);
  switch (A.jobs4[blockIdx.x].z) {
    case K3_PACK: vv3b_dispatch<K3_PACK, NT>(c, lds); break;
    case K3_PACKRED: vv3b_dispatch<K3_PACKRED, NT>(c, lds); break;
    case K3_DENSERED: vv3b_dispatch<K3_DENSERED, NT>(c, lds); break;
    case K3_S2PAIR: vv3b_dispatch<K3_S2PAIR, NT>(c, lds); break;
    default: vv3b_dispatch<K3_S2DIAG, NT>(c, lds); break;
  }
}

// One instantiation per object file, selected by ESMP2_VV3_NT (see vv3.hip).
#if defined(ESMP2_VV3_NT)
template __global__ void k_vv3b<ESMP2_VV3_NT>(VVArgs<float>);
#endif

}  // namespace esmp2
