// Krylov vector kernels: weighted dot products and fused preconditioned CG
// updates (FP64).  Inner-product weight w = 1 on the S2 box, 2 elsewhere
// (every other stored amplitude stands for a spin-flip pair of determinants).
#include "common.h"
#include "reduce.h"
#include "pcg.h"

namespace esmp2 {

__device__ inline double wgt(int64_t g, int64_t s0, int64_t s1) { return (g >= s0 && g < s1) ? 1.0 : 2.0; }

// partial[block] = sum_g w_g x_g y_g   (grid-stride, fixed grid -> deterministic)
__global__ __launch_bounds__(256) void k_dot(const double* x, const double* y, int64_t n, int64_t s0,
                                             int64_t s1, double* partial) {
  Acc2 acc;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x)
    acc.add(wgt(g, s0, s1) * x[g] * y[g]);
  double s = block_sum2(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// sc[k] = sum of partials[k*nb .. k*nb+nb-1]  for k < nsum (one block per sum)
__global__ void k_finish(const double* partial, int nb, double* sc, int base) {
  Acc2 acc;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) acc.add(partial[(int64_t)blockIdx.x * nb + i]);
  double s = block_sum2(acc);
  if (threadIdx.x == 0) sc[base + blockIdx.x] = s;
}

// alpha = sc[RHO] / sc[PQ];  x += alpha p;  r -= alpha q;
// partials of <r, D^-1 r>_W and <r, r>_W (two partial arrays of nb each)
__global__ __launch_bounds__(256) void k_update_xr(double* x, double* r, const double* p, const double* q,
                                                   const double* dinv, int64_t n, int64_t s0, int64_t s1,
                                                   const double* sc, double* partial) {
  const double alpha = sc[SC_RHO] / sc[SC_PQ];
  double rz = 0.0, rr = 0.0;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
    double rg = r[g] - alpha * q[g];
    x[g] += alpha * p[g];
    r[g] = rg;
    double w = wgt(g, s0, s1);
    rz += w * rg * rg * dinv[g];
    rr += w * rg * rg;
  }
  double a = block_sum(rz);
  double b = block_sum(rr);
  if (threadIdx.x == 0) { partial[blockIdx.x] = a; partial[gridDim.x + blockIdx.x] = b; }
}

// p = D^-1 r + beta p,  beta = sc[RHO_NEW] / sc[RHO]; then sc[RHO] = sc[RHO_NEW] (block 0 after use)
__global__ __launch_bounds__(256) void k_update_p(double* p, const double* r, const double* dinv, int64_t n,
                                                  const double* sc) {
  const double beta = sc[SC_RHO_NEW] / sc[SC_RHO];
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x)
    p[g] = dinv[g] * r[g] + beta * p[g];
}

__global__ void k_roll_rho(double* sc) {
  if (threadIdx.x == 0) sc[SC_RHO] = sc[SC_RHO_NEW];
}

// r = -b - y (y = A x0) or r = -b;  p = D^-1 r;  partials of <r, D^-1 r>, <r, r>
__global__ __launch_bounds__(256) void k_init(const double* b, const double* y, double* r, double* p,
                                              const double* dinv, int64_t n, int64_t s0, int64_t s1,
                                              double* partial) {
  double rz = 0.0, rr = 0.0;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
    double rg = -b[g] - (y ? y[g] : 0.0);
    r[g] = rg;
    p[g] = dinv[g] * rg;
    double w = wgt(g, s0, s1);
    rz += w * rg * rg * dinv[g];
    rr += w * rg * rg;
  }
  double a = block_sum(rz);
  double c = block_sum(rr);
  if (threadIdx.x == 0) { partial[blockIdx.x] = a; partial[gridDim.x + blockIdx.x] = c; }
}

// x += d (refinement); also used to copy
__global__ void k_axpy(double* y, const double* x, double a, int64_t n) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x)
    y[g] += a * x[g];
}

}  // namespace esmp2
