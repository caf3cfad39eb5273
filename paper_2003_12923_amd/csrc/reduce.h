// Deterministic FP64 block reductions (wavefront DPP tree, then LDS).
#pragma once
#include <hip/hip_runtime.h>

// Wavefront sum through DPP lane moves (no LDS traffic): quad sums, 8- and
// 16-lane sums by mirrors, then rows 1 and 3 take rows 0 and 2 (row_bcast:15)
// and row 3 takes lanes 0-31 (row_bcast:31); lane 63 holds the total, read back
// into every lane.  A fixed order, the same in every wavefront.  All 64 lanes
// must be active.
template <int CTRL, int ROWS>
__device__ inline double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ inline double wave_sum(double v) {
  v += dpp_move<0xb1, 0xf>(v);     // quad_perm [1,0,3,2]
  v += dpp_move<0x4e, 0xf>(v);     // quad_perm [2,3,0,1]
  v += dpp_move<0x141, 0xf>(v);    // row_half_mirror
  v += dpp_move<0x140, 0xf>(v);    // row_mirror
  v += dpp_move<0x142, 0xa>(v);    // row_bcast:15 into rows 1 and 3
  v += dpp_move<0x143, 0xc>(v);    // row_bcast:31 into rows 2 and 3
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the workgroup (blockDim.x a multiple of 64, <= 1024); result valid in thread 0.
__device__ inline double block_sum(double v) {
  __shared__ double ws[16];
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) ws[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int k = 0; k < nw; ++k) r += ws[k];
  }
  return r;
}

// Compensated accumulation (Neumaier): value s with running error c.
struct Acc2 {
  double s = 0.0, c = 0.0;
  __device__ inline void add(double v) {
    double t = s + v;
    if (fabs(s) >= fabs(v)) c += (s - t) + v; else c += (v - t) + s;
    s = t;
  }
  __device__ inline void add(const Acc2& o) { add(o.s); c += o.c; }
  __device__ inline double value() const { return s + c; }
};

template <int CTRL, int ROWS>
__device__ inline Acc2 acc2_dpp_step(Acc2 a) {
  Acc2 b;
  b.s = dpp_move<CTRL, ROWS>(a.s);       // a disabled row receives (0, 0), which leaves (s, c) unchanged
  b.c = dpp_move<CTRL, ROWS>(a.c);
  a.add(b);
  return a;
}

// Compensated wavefront sum, the DPP order of wave_sum; every lane gets the total.
__device__ inline Acc2 wave_sum2(Acc2 a) {
  a = acc2_dpp_step<0xb1, 0xf>(a);
  a = acc2_dpp_step<0x4e, 0xf>(a);
  a = acc2_dpp_step<0x141, 0xf>(a);
  a = acc2_dpp_step<0x140, 0xf>(a);
  a = acc2_dpp_step<0x142, 0xa>(a);
  a = acc2_dpp_step<0x143, 0xc>(a);
  Acc2 r;
  const long long bs = __double_as_longlong(a.s), bc = __double_as_longlong(a.c);
  r.s = __longlong_as_double(((long long)__builtin_amdgcn_readlane((int)(bs >> 32), 63) << 32) |
                             (unsigned)__builtin_amdgcn_readlane((int)(bs & 0xffffffff), 63));
  r.c = __longlong_as_double(((long long)__builtin_amdgcn_readlane((int)(bc >> 32), 63) << 32) |
                             (unsigned)__builtin_amdgcn_readlane((int)(bc & 0xffffffff), 63));
  return r;
}

// Compensated workgroup sum; result valid in thread 0.
__device__ inline double block_sum2(Acc2 a) {
  __shared__ double ws[16], wc[16];
  a = wave_sum2(a);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) { ws[w] = a.s; wc[w] = a.c; }
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    Acc2 t;
    const int nw = blockDim.x >> 6;
    for (int k = 0; k < nw; ++k) { Acc2 u; u.s = ws[k]; u.c = wc[k]; t.add(u); }
    r = t.value();
  }
  return r;
}
