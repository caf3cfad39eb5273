// Krylov vector kernels: weighted dot products and fused preconditioned CG
// updates, for FP64 vectors and for the FP32 vectors of the inner solves of
// the mixed-precision refinement (whose reductions still accumulate in FP64).
// Inner-product weight w = 1 on the S2 box, 2 elsewhere (every other stored
// amplitude stands for a spin-flip pair of determinants).
#include "common.h"
#include "reduce.h"
#include "pcg.h"

namespace esmp2 {

__device__ inline double wgt(int64_t g, int64_t s0, int64_t s1) { return (g >= s0 && g < s1) ? 1.0 : 2.0; }

// Grid-stride vector kernels take PCG_U elements per thread per round (g,
// g + stride, ...; the same order as a plain grid-stride loop, so the same
// sums): all loads of a round are issued before its first store, which the
// compiler cannot do across the stores of a plain loop (the vectors may alias
// as far as it knows), and their latencies overlap.
constexpr int PCG_U = 4;

// Streaming accesses of the CG vector updates: nontemporal loads and stores
// (each vector is touched once per pass; keeping it out of the caches lets the
// pass run at a higher fraction of HBM bandwidth)
template <class T> __device__ __attribute__((always_inline)) inline T ldnt(const T* p) {
  return __builtin_nontemporal_load(p);
}
template <class T> __device__ __attribute__((always_inline)) inline void stnt(T v, T* p) {
  __builtin_nontemporal_store(v, p);
}

// partial[block] = sum_g w_g x_g y_g   (grid-stride, fixed grid -> deterministic)
template <class T>
__device__ __attribute__((always_inline)) inline void dot_body(const T* x, const T* y, int64_t n, int64_t s0, int64_t s1,
                                             double* partial, int bid_, int nb_) {
  Acc2 acc;
  const int64_t st = (int64_t)nb_ * blockDim.x;
  for (int64_t g0 = (int64_t)bid_ * blockDim.x + threadIdx.x; g0 < n; g0 += PCG_U * st) {
    T xv[PCG_U], yv[PCG_U];
#pragma unroll
    for (int u = 0; u < PCG_U; ++u) {
      const int64_t g = g0 + u * st, gg = g < n ? g : 0;
      xv[u] = ldnt(x + gg);
      yv[u] = ldnt(y + gg);
    }
#pragma unroll
    for (int u = 0; u < PCG_U; ++u) {
      const int64_t g = g0 + u * st;
      if (g < n) acc.add(wgt(g, s0, s1) * (double)xv[u] * (double)yv[u]);
    }
  }
  double s = block_sum2(acc);
  if (threadIdx.x == 0) partial[bid_] = s;
}

template <class T>
__global__ __launch_bounds__(256) void k_dot(const T* x, const T* y, int64_t n, int64_t s0, int64_t s1,
                                             double* partial) {
  dot_body<T>(x, y, n, s0, s1, partial, blockIdx.x, gridDim.x);
}

// sc[base + k] = sum of partials[k*nb .. k*nb+nb-1], one block per sum
__device__ __attribute__((always_inline)) inline void finish_body(const double* partial, int nb, double* sc, int base, int bid_, int nb_) {
  // each thread adds its indices i, i + blockDim.x, ... in that order; the
  // loads of eight of them are issued before the adds (a long partial list is
  // otherwise one load latency per element)
  Acc2 acc;
  const double* pp = partial + (int64_t)bid_ * nb;
  for (int i0 = threadIdx.x; i0 < nb; i0 += 8 * blockDim.x) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u * (int)blockDim.x;
      v[u] = i < nb ? pp[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc.add(v[u]);     // adding an exact zero leaves (s, c) unchanged
  }
  double s = block_sum2(acc);
  if (threadIdx.x == 0) sc[base + bid_] = s;
}

__global__ void k_finish(const double* partial, int nb, double* sc, int base) {
  finish_body(partial, nb, sc, base, blockIdx.x, gridDim.x);
}

// The preconditioner M = D^-1 is stored in FP32 (rounded once): any fixed
// symmetric positive diagonal is a valid Jacobi preconditioner, the iterates,
// residuals and E2 stay FP64, and the vector passes read half the bytes.
//
// alpha = sc[RHO] / sc[PQ];  r -= alpha q;  partials of <r, M r>_W and <r, r>_W
// (two partial arrays of gridDim.x each).  x is updated with p in k_update_px,
// which reads p anyway.
template <class T>
__device__ __attribute__((always_inline)) inline void update_r_body_a(T* r, const T* q, const float* dinv, int64_t n,
                                                    int64_t s0, int64_t s1, T alpha, double* partial, int bid_,
                                                    int nb_) {
  double rz = 0.0, rr = 0.0;
  const int64_t st = (int64_t)nb_ * blockDim.x;
  for (int64_t g0 = (int64_t)bid_ * blockDim.x + threadIdx.x; g0 < n; g0 += PCG_U * st) {
    T rv[PCG_U], qv[PCG_U];
    float dv[PCG_U];
#pragma unroll
    for (int u = 0; u < PCG_U; ++u) {
      const int64_t g = g0 + u * st, gg = g < n ? g : 0;
      rv[u] = ldnt(r + gg); qv[u] = ldnt(q + gg); dv[u] = ldnt(dinv + gg);
    }
#pragma unroll
    for (int u = 0; u < PCG_U; ++u) {
      const int64_t g = g0 + u * st;
      if (g < n) {
        const T rg = rv[u] - alpha * qv[u];
        stnt(rg, r + g);
        const double w = wgt(g, s0, s1), rd = (double)rg;
        rz += w * rd * rd * (double)dv[u];
        rr += w * rd * rd;
      }
    }
  }
  double a = block_sum(rz);
  double b = block_sum(rr);
  if (threadIdx.x == 0) { partial[bid_] = a; partial[nb_ + bid_] = b; }
}

template <class T>
__device__ __attribute__((always_inline)) inline void update_r_body(T* r, const T* q, const float* dinv, int64_t n, int64_t s0,
                                                  int64_t s1, const double* sc, double* partial, int bid_, int nb_) {
  update_r_body_a<T>(r, q, dinv, n, s0, s1, (T)(sc[SC_RHO] / sc[SC_PQ]), partial, bid_, nb_);
}

template <class T>
__global__ __launch_bounds__(256) void k_update_r(T* r, const T* q, const float* dinv, int64_t n, int64_t s0,
                                                  int64_t s1, const double* sc, double* partial) {
  update_r_body<T>(r, q, dinv, n, s0, s1, sc, partial, blockIdx.x, gridDim.x);
}

// alpha = sc[RHO] / sc[PQ], beta = sc[RHO_NEW] / sc[RHO]:  x += alpha p;  p = M r + beta p
// p = M r + beta p alone (a solve that keeps no x)
template <class T>
__device__ __attribute__((always_inline)) inline void update_p_body(T* p, const T* r, const float* dinv, int64_t n,
                                                  const double* sc, int bid_, int nb_) {
  const T beta = (T)(sc[SC_RHO_NEW] / sc[SC_RHO]);
  const int64_t st = (int64_t)nb_ * blockDim.x;
  for (int64_t g0 = (int64_t)bid_ * blockDim.x + threadIdx.x; g0 < n; g0 += PCG_U * st) {
    T pv[PCG_U], rv[PCG_U];
    float dv[PCG_U];
#pragma unroll
    for (int u = 0; u < PCG_U; ++u) {
      const int64_t g = g0 + u * st, gg = g < n ? g : 0;
      pv[u] = ldnt(p + gg); rv[u] = ldnt(r + gg); dv[u] = ldnt(dinv + gg);
    }
#pragma unroll
    for (int u = 0; u < PCG_U; ++u) {
      const int64_t g = g0 + u * st;
      if (g < n) stnt((T)dv[u] * rv[u] + beta * pv[u], p + g);
    }
  }
}

template <class T>
__device__ __attribute__((always_inline)) inline void update_px_body(T* x, T* p, const T* r, const float* dinv, int64_t n,
                                                   const double* sc, int bid_, int nb_) {
  const T alpha = (T)(sc[SC_RHO] / sc[SC_PQ]);
  const T beta = (T)(sc[SC_RHO_NEW] / sc[SC_RHO]);
  const int64_t st = (int64_t)nb_ * blockDim.x;
  for (int64_t g0 = (int64_t)bid_ * blockDim.x + threadIdx.x; g0 < n; g0 += PCG_U * st) {
    T xv[PCG_U], pv[PCG_U], rv[PCG_U];
    float dv[PCG_U];
#pragma unroll
    for (int u = 0; u < PCG_U; ++u) {
      const int64_t g = g0 + u * st, gg = g < n ? g : 0;
      xv[u] = ldnt(x + gg); pv[u] = ldnt(p + gg); rv[u] = ldnt(r + gg); dv[u] = ldnt(dinv + gg);
    }
#pragma unroll
    for (int u = 0; u < PCG_U; ++u) {
      const int64_t g = g0 + u * st;
      if (g < n) {
        stnt(xv[u] + alpha * pv[u], x + g);
        stnt((T)dv[u] * rv[u] + beta * pv[u], p + g);
      }
    }
  }
}

template <class T>
__global__ __launch_bounds__(256) void k_update_px(T* x, T* p, const T* r, const float* dinv, int64_t n,
                                                   const double* sc) {
  update_px_body<T>(x, p, r, dinv, n, sc, blockIdx.x, gridDim.x);
}

// x += alpha p, alpha = sc[RHO] / sc[PQ]: the update of the last iteration
template <class T>
__device__ __attribute__((always_inline)) inline void update_x_body(T* x, const T* p, int64_t n, const double* sc, int bid_, int nb_) {
  const T alpha = (T)(sc[SC_RHO] / sc[SC_PQ]);
  const int64_t st = (int64_t)nb_ * blockDim.x;
  for (int64_t g0 = (int64_t)bid_ * blockDim.x + threadIdx.x; g0 < n; g0 += PCG_U * st) {
    T xv[PCG_U], pv[PCG_U];
#pragma unroll
    for (int u = 0; u < PCG_U; ++u) {
      const int64_t g = g0 + u * st, gg = g < n ? g : 0;
      xv[u] = ldnt(x + gg); pv[u] = ldnt(p + gg);
    }
#pragma unroll
    for (int u = 0; u < PCG_U; ++u) {
      const int64_t g = g0 + u * st;
      if (g < n) stnt(xv[u] + alpha * pv[u], x + g);
    }
  }
}

template <class T>
__global__ __launch_bounds__(256) void k_update_x(T* x, const T* p, int64_t n, const double* sc) {
  update_x_body<T>(x, p, n, sc, blockIdx.x, gridDim.x);
}

__global__ void k_roll_rho(double* sc) {
  if (threadIdx.x == 0) sc[SC_RHO] = sc[SC_RHO_NEW];
}

// r = -b - y (y = A x0) or r = -b;  p = M r;  partials of <r, M r>, <r, r>;
// xz = 0 where given (the start x = 0); r not stored when null (a solve whose
// first iteration reads -b for r)
__device__ __attribute__((always_inline)) inline void init_body(const double* b, const double* y, double* r, double* p,
                                              const float* dinv, int64_t n, int64_t s0, int64_t s1,
                                              double* partial, int bid_, int nb_, double* xz = nullptr) {
  double rz = 0.0, rr = 0.0;
  const int64_t st = (int64_t)nb_ * blockDim.x;
  for (int64_t g0 = (int64_t)bid_ * blockDim.x + threadIdx.x; g0 < n; g0 += PCG_U * st) {
    double bv[PCG_U], yv[PCG_U];
    float dv[PCG_U];
#pragma unroll
    for (int u = 0; u < PCG_U; ++u) {
      const int64_t g = g0 + u * st, gg = g < n ? g : 0;
      bv[u] = ldnt(b + gg); yv[u] = y ? ldnt(y + gg) : 0.0; dv[u] = ldnt(dinv + gg);
    }
#pragma unroll
    for (int u = 0; u < PCG_U; ++u) {
      const int64_t g = g0 + u * st;
      if (g < n) {
        const double rg = -bv[u] - yv[u];
        if (r) stnt(rg, r + g);
        stnt((double)dv[u] * rg, p + g);
        if (xz) stnt(0.0, xz + g);
        const double w = wgt(g, s0, s1);
        rz += w * rg * rg * (double)dv[u];
        rr += w * rg * rg;
      }
    }
  }
  double a = block_sum(rz);
  double c = block_sum(rr);
  if (threadIdx.x == 0) { partial[bid_] = a; partial[nb_ + bid_] = c; }
}

__global__ __launch_bounds__(256) void k_init(const double* b, const double* y, double* r, double* p,
                                              const float* dinv, int64_t n, int64_t s0, int64_t s1,
                                              double* partial, double* xz) {
  init_body(b, y, r, p, dinv, n, s0, s1, partial, blockIdx.x, gridDim.x, xz);
}

// FP64 residual of the refinement: r = -b - y (y = A x, or NULL for x = 0);  partials of <r, r>_W
__global__ __launch_bounds__(256) void k_resid(const double* b, const double* y, double* r, int64_t n, int64_t s0,
                                               int64_t s1, double* partial) {
  Acc2 acc;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g0 < n; g0 += PCG_U * st) {
    double bv[PCG_U], yv[PCG_U];
#pragma unroll
    for (int u = 0; u < PCG_U; ++u) {
      const int64_t g = g0 + u * st, gg = g < n ? g : 0;
      bv[u] = ldnt(b + gg); yv[u] = y ? ldnt(y + gg) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < PCG_U; ++u) {
      const int64_t g = g0 + u * st;
      if (g < n) {
        const double rg = -bv[u] - yv[u];
        stnt(rg, r + g);
        acc.add(wgt(g, s0, s1) * rg * rg);
      }
    }
  }
  double s = block_sum2(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Start of an inner FP32 solve A d = r64 / s (s = scale, the norm of r64):
// r = fl(r64 / s), d = 0, p = D^-1 r; partials of <r, D^-1 r>, <r, r> (FP64 sums)
__global__ __launch_bounds__(256) void k_init_inner(const double* r64, double scale, float* r, float* p,
                                                    float* d, const float* dinv, int64_t n, int64_t s0, int64_t s1,
                                                    double* partial) {
  const double inv = 1.0 / scale;
  double rz = 0.0, rr = 0.0;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g0 < n; g0 += PCG_U * st) {
    double rv[PCG_U];
    float dv[PCG_U];
#pragma unroll
    for (int u = 0; u < PCG_U; ++u) {
      const int64_t g = g0 + u * st, gg = g < n ? g : 0;
      rv[u] = ldnt(r64 + gg); dv[u] = ldnt(dinv + gg);
    }
#pragma unroll
    for (int u = 0; u < PCG_U; ++u) {
      const int64_t g = g0 + u * st;
      if (g < n) {
        const float rg = (float)(rv[u] * inv);
        stnt(rg, r + g);
        stnt(0.f, d + g);
        stnt(dv[u] * rg, p + g);
        const double w = wgt(g, s0, s1), rd = (double)rg;
        rz += w * rd * rd * (double)dv[u];
        rr += w * rd * rd;
      }
    }
  }
  double a = block_sum(rz);
  double c = block_sum(rr);
  if (threadIdx.x == 0) { partial[blockIdx.x] = a; partial[gridDim.x + blockIdx.x] = c; }
}

// x += scale d, the refinement update in FP64
__global__ __launch_bounds__(256) void k_refine(double* x, const float* d, double scale, int64_t n) {
  const double s = scale;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g0 < n; g0 += PCG_U * st) {
    double xv[PCG_U];
    float dv[PCG_U];
#pragma unroll
    for (int u = 0; u < PCG_U; ++u) {
      const int64_t g = g0 + u * st, gg = g < n ? g : 0;
      xv[u] = ldnt(x + gg); dv[u] = ldnt(d + gg);
    }
#pragma unroll
    for (int u = 0; u < PCG_U; ++u) {
      const int64_t g = g0 + u * st;
      if (g < n) stnt(xv[u] + s * (double)dv[u], x + g);
    }
  }
}

// b = fl32(a), round to nearest
__global__ void k_to_f32(const double* a, float* b, int64_t n) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x)
    b[g] = (float)a[g];
}

// up to five FP64 -> FP32 conversions in one launch (the Fock blocks of an operator)
struct ToF32Set {
  const double* a[5];
  float* b[5];
  int64_t n[5];
};

__global__ void k_to_f32_set(ToF32Set t) {
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  const int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
  for (int k = 0; k < 5; ++k)
    for (int64_t g = g0; g < t.n[k]; g += st) t.b[k][g] = (float)t.a[k][g];
}

template __global__ void k_dot<double>(const double*, const double*, int64_t, int64_t, int64_t, double*);
template __global__ void k_dot<float>(const float*, const float*, int64_t, int64_t, int64_t, double*);
template __global__ void k_update_r<double>(double*, const double*, const float*, int64_t, int64_t, int64_t,
                                           const double*, double*);
template __global__ void k_update_r<float>(float*, const float*, const float*, int64_t, int64_t, int64_t,
                                          const double*, double*);
template __global__ void k_update_px<double>(double*, double*, const double*, const float*, int64_t, const double*);
template __global__ void k_update_px<float>(float*, float*, const float*, const float*, int64_t, const double*);
template __global__ void k_update_x<double>(double*, const double*, int64_t, const double*);
template __global__ void k_update_x<float>(float*, const float*, int64_t, const double*);

}  // namespace esmp2
