#pragma once
#include "common.h"

namespace esmp2 {
enum { SC_RHO = 0, SC_PQ = 1, SC_RHO_NEW = 2, SC_RR = 3, SC_BX = 4, SC_XR = 5, SC_BB = 6, SC_TMP = 7, SC_N = 16 };
// slots 8..15: the device-stopped solve's eight partial sums of <p, Ap>_W
constexpr int SC_PQ8 = 8, PQ_PARTS = 8;
constexpr int PCG_BLOCKS = 1024;

template <class T> __global__ void k_dot(const T* x, const T* y, int64_t n, int64_t s0, int64_t s1, double* partial);
__global__ void k_finish(const double* partial, int nb, double* sc, int base);
template <class T>
__global__ void k_update_r(T* r, const T* q, const float* dinv, int64_t n, int64_t s0, int64_t s1, const double* sc,
                           double* partial);
template <class T>
__global__ void k_update_px(T* x, T* p, const T* r, const float* dinv, int64_t n, const double* sc);
template <class T> __global__ void k_update_x(T* x, const T* p, int64_t n, const double* sc);
__global__ void k_roll_rho(double* sc);
__global__ void k_init(const double* b, const double* y, double* r, double* p, const float* dinv, int64_t n,
                       int64_t s0, int64_t s1, double* partial, double* xz);
__global__ void k_resid(const double* b, const double* y, double* r, int64_t n, int64_t s0, int64_t s1,
                        double* partial);
__global__ void k_init_inner(const double* r64, double scale, float* r, float* p, float* d,
                             const float* dinv, int64_t n, int64_t s0, int64_t s1, double* partial);
__global__ void k_refine(double* x, const float* d, double scale, int64_t n);
__global__ void k_to_f32(const double* a, float* b, int64_t n);
}  // namespace esmp2
