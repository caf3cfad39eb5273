#pragma once
#include "common.h"

namespace esmp2 {
enum { SC_RHO = 0, SC_PQ = 1, SC_RHO_NEW = 2, SC_RR = 3, SC_BX = 4, SC_XR = 5, SC_BB = 6, SC_TMP = 7, SC_N = 16 };
constexpr int PCG_BLOCKS = 1024;

__global__ void k_dot(const double* x, const double* y, int64_t n, int64_t s0, int64_t s1, double* partial);
__global__ void k_finish(const double* partial, int nb, double* sc, int base);
__global__ void k_update_xr(double* x, double* r, const double* p, const double* q, const double* dinv,
                            int64_t n, int64_t s0, int64_t s1, const double* sc, double* partial);
__global__ void k_update_p(double* p, const double* r, const double* dinv, int64_t n, const double* sc);
__global__ void k_roll_rho(double* sc);
__global__ void k_init(const double* b, const double* y, double* r, double* p, const double* dinv, int64_t n,
                       int64_t s0, int64_t s1, double* partial);
__global__ void k_axpy(double* y, const double* x, double a, int64_t n);
}  // namespace esmp2
