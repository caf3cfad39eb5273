// Kernel argument blocks of the sigma kernels, templated on the storage and
// arithmetic type T (double: the FP64 operator; float: the FP32 operator of
// the mixed-precision solve).
#pragma once
#include "common.h"

namespace esmp2 {

template <class T>
struct GatherArgs {
  Dims d;
  const T* x;
  const T* S;
  T* y;
  const T* fo;      // no x no
  const T* fv;      // nv x nv
  const T* fov;     // no x nv
  const T* side_tr;
  const T *t3_t, *t3_p1, *t3_p2, *h11_p1, *h11_p2, *h12_t, *h12_u1, *h12_u2;
  const T *h21_t, *h21_k, *h22_ut, *h22_i, *h22_uk;
};

template <class T>
struct VVArgs {
  Dims d;
  const T* x;            // input amplitudes (seven-box layout)
  const T* S;            // flip-symmetrised S2 (dense)
  T* y;                  // output
  const T* Fd;           // F_vv - omega/2, padded mv x mv (doubles boxes)
  const T* Fl;           // F_vv + kappa/2, padded mv x mv (L boxes)
  T* side_tr;            // transfer rows: [npo H1P2 batches][nv], then [(no-1)^2 H2P2][nv]
  const int2* jobs;      // (box, batch): generic Sylvester kernel
  const int4* jobs4;     // (box, batch or i, storage format, j): specialised Sylvester kernel
};

template <class T>
struct SideArgs {
  Dims d;
  const T* x;
  const T* fov;                     // f_{i a}, no x nv
  T *t3_t, *t3_p1, *t3_p2;          // [npo1][nv]
  T *h11_p1, *h11_p2;               // [npo][nv]
  T *h12_t, *h12_u1, *h12_u2;       // [npo][nv]
  T *h21_t, *h21_k;                 // [(no-1)^2][nv]
  T *h22_ut, *h22_i, *h22_uk;       // [(no-1)^2][nv]
};

// pair-index decode tables, entries (p << 16) | q with p < q
struct PairTables {
  const int* pv;     // virtual pairs of nv
  const int* pv1;    // virtual pairs of nv - 1
  const int* po;     // occupied pairs of no
  const int* po1;    // occupied pairs of no - 1
};

// Inner index of thread `tid` of a coupling chunk (256 threads).  The S2 box
// (dense nv x nv per batch) is cut into 16 x 16 tiles of (a, b), chunk.z =
// (tile row << 16) | tile column, so that a wavefront reads four 128-byte
// runs both of X[a][b] and of the transposed X[b][a] of a partner batch; every
// other box takes 256 consecutive inner indices from chunk.z.  Returns `inner`
// for a thread outside the box.
__device__ inline int chunk_inner(int box, int z, int tid, int nv, int inner) {
  if (box != B_S2) return z + tid;
  const int a = 16 * (z >> 16) + (tid >> 4), b = 16 * (z & 0xffff) + (tid & 15);
  return (a < nv && b < nv) ? a * nv + b : inner;
}

constexpr int GO = 8;   // inner (virtual-pair) indices per workgroup of the occupied-index kernel

template <class T> __global__ void k_sym_s2(Dims d, const T* x, T* S);
// workgroups of k_sym_s2: one per 32 x 32 block of (a, b) of each batch (i, j)
inline int64_t sym_s2_blocks(const Dims& d) {
  const int nt = (d.nv + 31) / 32;
  return (int64_t)d.no * d.no * nt * nt;
}
template <class T, int TW> __global__ void k_vv(VVArgs<T> A);
constexpr int V3_THREADS = 512;   // workgroup of the specialised Sylvester kernels: 8 wavefronts
template <class T, int NT> __global__ void k_vv3(VVArgs<T> A);
template <int NT> __global__ void k_vv3b(VVArgs<float> A);
template <class T> __global__ void k_side(SideArgs<T> A);
template <class T> __global__ void k_couple(GatherArgs<T> A, PairTables P, const int4* chunks);
template <class T> __global__ void k_oo(GatherArgs<T> A, int4 tiles0, int4 tiles1);
template <class T> __global__ void k_oo_plain(GatherArgs<T> A);

}  // namespace esmp2
