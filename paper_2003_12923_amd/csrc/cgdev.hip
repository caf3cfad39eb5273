// One state's FP64 conjugate gradient in the pinned-semicanonical basis with
// its convergence test and stop on the device.  The host queues iteration
// i + 1 before it reads the outcome of iteration i, so the GPU never waits for
// the host; a state that has stopped turns the kernels of the queued iteration
// into no-ops.  The kernels are those of the host-driven loop (same bodies,
// same sums), each with a check of the control word first.
//
// Control word (device memory), one iteration:
//   pq finish    LAST -> DONE (the queued iteration after the last one);
//                RUN: rho <- rho_new (from the second iteration on), eight
//                partial sums of <p, Ap>_W (eight workgroups)
//   update_r     RUN only; every workgroup adds the eight parts in one order
//                (workgroup 0 also stores the sum for the later kernels)
//   finish_r     RUN only: <r, M r>_W, <r, r>_W, then the test: p.Ap <= 0 ->
//                DONE (not SPD); ||r||_W / ||b||_W <= tol or max_iter -> LAST
//                (||b||_W^2 in sc[SC_BB] from the start)
//   update_px    RUN: x += alpha p, p = M r + beta p;  LAST: x += alpha p and
//                the parts of the Hylleraas dots <b, x>_W, <x, r>_W
// The first iteration of a solve from x = 0 (first = 1) takes r = -b and
// x = alpha p without reading r or x: the start stores neither.
// A solve from x = 0 whose x nobody reads (no_x) keeps no x at all: for the
// iterates of conjugate gradient from zero <b, p_i>_W = -rho_i and
// <x_k, r_k>_W = 0, so the Hylleraas value <b, x>_W - <x, r>_W is the sum
// -sum_i alpha_i rho_i, which update_r adds up in sc[SC_BX] (sc[SC_XR] = 0);
// update_px then writes p only and the last update has nothing to do.
#include "common.h"
#include "sigma.h"
#include "pcg.h"
#include "reduce.h"

namespace esmp2 {

enum { CG_RUN = 0, CG_LAST = 1, CG_DONE = 2 };

struct CgCtl {
  int mode, it, status, pad;
  double rel;     // last ||r||_W / ||b||_W
};

// The start: ||b||_W^2 into sc[SC_BB] (from <r, r>_W when r = -b), the
// relative residual (from the host's value or from sc), RUN unless it is
// already within tol (or not a number: b = 0).
__global__ void kd_ctl_init(CgCtl* c, double* sc, int from_zero, double tol, double rel0, int rel_on_device) {
  if (threadIdx.x == 0) {
    sc[SC_BX] = 0.0;
    sc[SC_XR] = 0.0;
    if (from_zero) sc[SC_BB] = sc[SC_PQ];
    const double rel = rel_on_device ? sqrt(sc[SC_PQ]) / sqrt(sc[SC_BB]) : rel0;
    c->mode = rel > tol ? CG_RUN : CG_DONE;
    c->it = 0;
    c->status = ESMP2_OK;
    c->rel = rel;
  }
}

__global__ __launch_bounds__(256) void kd_sym(Dims d, const double* x, double* S, const CgCtl* c) {
  if (c->mode != CG_RUN) return;
  sym_s2_body<double>(d, x, S, blockIdx.x, gridDim.x);
}

template <int MV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MV <= 160 ? 5 : 4))) void kd_gemv(GemvArgs<double> A, const CgCtl* c) {
  if (c->mode != CG_RUN) return;
  gemv_body<double, MV>(A, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void kd_arrow(ArrowArgs<double> A, PairTables P, const int4* chunks, double* pq,
                                                const CgCtl* c) {
  if (c->mode != CG_RUN) return;
  arrow_body<double>(A, P, chunks, pq, blockIdx.x, gridDim.x);
}

// PQ_PARTS workgroups: part k of the arrow kernel's per-chunk parts into sc[SC_PQ8 + k]
__global__ __launch_bounds__(1024) void kd_finish_pq(const double* pq, int nb, double* sc, CgCtl* c) {
  const int mode = c->mode;
  if (mode == CG_LAST) {
    if (threadIdx.x == 0 && blockIdx.x == 0) c->mode = CG_DONE;
    return;
  }
  if (mode != CG_RUN) return;
  if (threadIdx.x == 0 && blockIdx.x == 0 && c->it > 0) sc[SC_RHO] = sc[SC_RHO_NEW];
  const int lo = (int)((int64_t)nb * blockIdx.x / PQ_PARTS), hi = (int)((int64_t)nb * (blockIdx.x + 1) / PQ_PARTS);
  finish_body(pq + lo, hi - lo, sc + SC_PQ8 + blockIdx.x, 0, 0, 1);
}

// <p, Ap>_W from its eight parts (the same order in every workgroup)
__device__ inline double pq_sum(const double* sc) {
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < PQ_PARTS; ++k) s += sc[SC_PQ8 + k];
  return s;
}

__global__ __launch_bounds__(256) void kd_update_r(double* r, const double* q, const float* dinv, int64_t n,
                                                   int64_t s0, int64_t s1, const double* sc, double* partial,
                                                   double* scw, const CgCtl* c, const double* b, int first,
                                                   int no_x) {
  if (c->mode != CG_RUN) return;
  const double pq = pq_sum(sc);
  const double alpha = sc[SC_RHO] / pq;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    scw[SC_PQ] = pq;
    if (no_x && pq > 0.0) scw[SC_BX] -= alpha * sc[SC_RHO];   // Hylleraas value of the iterates
  }
  if (!first) {
    update_r_body_a<double>(r, q, dinv, n, s0, s1, alpha, partial, blockIdx.x, gridDim.x);
    return;
  }
  // r = -b - alpha q (the same sums as update_r_body with r = -b)
  double rz = 0.0, rr = 0.0;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g0 < n; g0 += PCG_U * st) {
    double bv[PCG_U], qv[PCG_U];
    float dv[PCG_U];
#pragma unroll
    for (int u = 0; u < PCG_U; ++u) {
      const int64_t g = g0 + u * st, gg = g < n ? g : 0;
      bv[u] = ldnt(b + gg); qv[u] = ldnt(q + gg); dv[u] = ldnt(dinv + gg);
    }
#pragma unroll
    for (int u = 0; u < PCG_U; ++u) {
      const int64_t g = g0 + u * st;
      if (g < n) {
        const double rg = -bv[u] - alpha * qv[u];
        stnt(rg, r + g);
        const double w = wgt(g, s0, s1);
        rz += w * rg * rg * (double)dv[u];
        rr += w * rg * rg;
      }
    }
  }
  double a = block_sum(rz);
  double d = block_sum(rr);
  if (threadIdx.x == 0) { partial[blockIdx.x] = a; partial[gridDim.x + blockIdx.x] = d; }
}

// two blocks: sc[SC_RHO_NEW], sc[SC_RR]; block 1 then takes the decision.
// Block 0 may read the control word after block 1 has changed it and skip
// rho_new: no stopped state reads rho_new.
__global__ __launch_bounds__(1024) void kd_finish_r(const double* partial, int nb, double* sc, CgCtl* c, double tol,
                                                    int max_iter) {
  if (c->mode != CG_RUN) return;
  finish_body(partial, nb, sc, SC_RHO_NEW, blockIdx.x, 2);
  if (blockIdx.x != 1 || threadIdx.x != 0) return;
  const double pq = sc[SC_PQ];
  if (!(pq > 0.0)) {
    c->status = ESMP2_NOT_SPD;
    c->mode = CG_DONE;
    return;
  }
  const int it = c->it + 1;
  const double rel = sqrt(sc[SC_RR]) / sqrt(sc[SC_BB]);
  c->it = it;
  c->rel = rel;
  if (rel <= tol || it >= max_iter) {
    if (rel > tol) c->status = ESMP2_NOT_CONVERGED;
    c->mode = CG_LAST;
  }
}

__global__ __launch_bounds__(256) void kd_update_px(double* x, double* p, const double* r, const double* b,
                                                    const float* dinv, int64_t n, int64_t s0, int64_t s1,
                                                    const double* sc, double* partial, const CgCtl* c, int first,
                                                    int no_x) {
  const int mode = c->mode;
  if (no_x) {            // p = M r + beta p only
    if (mode == CG_RUN) update_p_body<double>(p, r, dinv, n, sc, blockIdx.x, gridDim.x);
    return;
  }
  if (mode == CG_RUN && !first) {
    update_px_body<double>(x, p, r, dinv, n, sc, blockIdx.x, gridDim.x);
    return;
  }
  if (mode == CG_RUN) {     // x = alpha p;  p = M r + beta p
    const double alpha = sc[SC_RHO] / sc[SC_PQ];
    const double beta = sc[SC_RHO_NEW] / sc[SC_RHO];
    const int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g0 < n; g0 += PCG_U * st) {
      double pv[PCG_U], rv[PCG_U];
      float dv[PCG_U];
#pragma unroll
      for (int u = 0; u < PCG_U; ++u) {
        const int64_t g = g0 + u * st, gg = g < n ? g : 0;
        pv[u] = ldnt(p + gg); rv[u] = ldnt(r + gg); dv[u] = ldnt(dinv + gg);
      }
#pragma unroll
      for (int u = 0; u < PCG_U; ++u) {
        const int64_t g = g0 + u * st;
        if (g < n) {
          stnt(0.0 + alpha * pv[u], x + g);
          stnt((double)dv[u] * rv[u] + beta * pv[u], p + g);
        }
      }
    }
    return;
  }
  if (mode != CG_LAST) return;
  // x += alpha p, with the weighted dots of the new x against b and r
  const double alpha = sc[SC_RHO] / sc[SC_PQ];
  Acc2 bx, xr;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g0 < n; g0 += PCG_U * st) {
    double xv[PCG_U], pv[PCG_U], bv[PCG_U], rv[PCG_U];
#pragma unroll
    for (int u = 0; u < PCG_U; ++u) {
      const int64_t g = g0 + u * st, gg = g < n ? g : 0;
      xv[u] = first ? 0.0 : ldnt(x + gg); pv[u] = ldnt(p + gg); bv[u] = ldnt(b + gg); rv[u] = ldnt(r + gg);
    }
#pragma unroll
    for (int u = 0; u < PCG_U; ++u) {
      const int64_t g = g0 + u * st;
      if (g < n) {
        const double xn = xv[u] + alpha * pv[u];
        stnt(xn, x + g);
        const double w = wgt(g, s0, s1);
        bx.add(w * bv[u] * xn);
        xr.add(w * xn * rv[u]);
      }
    }
  }
  const double a = block_sum2(bx);
  const double d = block_sum2(xr);
  if (threadIdx.x == 0) { partial[blockIdx.x] = a; partial[gridDim.x + blockIdx.x] = d; }
}

}  // namespace esmp2
