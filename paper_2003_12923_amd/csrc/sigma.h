// Kernel argument blocks of the sigma kernels.
#pragma once
#include "common.h"

namespace esmp2 {

struct GatherArgs {
  Dims d;
  const double* x;
  const double* S;
  double* y;
  const double* fo;      // no x no
  const double* fv;      // nv x nv
  const double* fov;     // no x nv
  const double* side_tr;
  const double *t3_t, *t3_p1, *t3_p2, *h11_p1, *h11_p2, *h12_t, *h12_u1, *h12_u2;
  const double *h21_t, *h21_k, *h22_ut, *h22_i, *h22_uk;
};

struct VVArgs {
  Dims d;
  const double* x;       // input amplitudes (seven-box layout)
  const double* S;       // flip-symmetrised S2 (dense)
  double* y;             // output
  const double* Fd;      // F_vv - omega/2, padded mv x mv (doubles boxes)
  const double* Fl;      // F_vv + kappa/2, padded mv x mv (L boxes)
  double* side_tr;       // transfer rows: [npo H1P2 batches][nv], then [(no-1)^2 H2P2][nv]
  const int2* jobs;      // (box, batch)
  const int4* jobs4;     // (box, batch or i, kind, j) for k_vv2
  GatherArgs ga;         // per-element coupling terms added in the epilogue (k_vv3)
  int use_ga;            // 0: Sylvester part only
};

struct SideArgs {
  Dims d;
  const double* x;
  const double* fov;     // f_{i a}, no x nv
  double *t3_t, *t3_p1, *t3_p2;          // [npo1][nv]
  double *h11_p1, *h11_p2;               // [npo][nv]
  double *h12_t, *h12_u1, *h12_u2;       // [npo][nv]
  double *h21_t, *h21_k;                 // [(no-1)^2][nv]
  double *h22_ut, *h22_i, *h22_uk;       // [(no-1)^2][nv]
};


__global__ void k_sym_s2(Dims d, const double* x, double* S);
template <int TW> __global__ void k_vv(VVArgs A);
__global__ void k_vv2(VVArgs A);
template <int NT> __global__ void k_vv3(VVArgs A);
__global__ void k_side(SideArgs A);
__global__ void k_gather(GatherArgs A);
__global__ void k_gather2(GatherArgs A, int4 tiles0, int4 tiles1);
__global__ void k_gather3(GatherArgs A, int4 tiles0, int4 tiles1);
__global__ void k_oo(GatherArgs A, int4 tiles0, int4 tiles1);
__global__ void k_couple(GatherArgs G, const int2* jobs);

}  // namespace esmp2
