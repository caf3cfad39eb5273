// Many independent states solved together (the batched workload): the
// conjugate-gradient iterations of every state in the same kernel launches,
// one launch per step for all states, with each state's scalars, its
// convergence test and its stop decided on the device.  The host only reads
// how many states are still iterating, once per iteration.
//
// A launch covers the blocks of every state back to back; a block finds its
// state from a table of first blocks and runs the one-state kernel body with
// its local block index.  A state that has stopped leaves its blocks at once.
// The operator is the one of the pinned-semicanonical basis (arrow kernels),
// applied to p into q.  No x is kept (the batch returns energies only): each
// state's E2_DL is the Hylleraas value of its iterates, -sum_i alpha_i rho_i
// (for conjugate gradient from zero <b, p_i>_W = -rho_i and <x_k, r_k>_W = 0),
// added up in sc[SC_BX] as the state iterates (sc[SC_XR] = 0).
#include "common.h"
#include "sigma.h"
#include "pcg.h"
#include "reduce.h"

namespace esmp2 {

constexpr int BATCH_CG_BLOCKS = 128;    // blocks per state of the vector kernels

enum { BS_RUN = 0, BS_LAST = 1, BS_DONE = 2 };

struct BState {
  // operator (x = p, y = q)
  Dims d;
  GemvArgs<double> gv;
  ArrowArgs<double> aa;
  PairTables pt;
  const int4* chunks;
  int nsym, ngemv, nchunks;
  // Krylov vectors and scalars (the handle's)
  double *r, *p, *q, *sc, *partial, *pq, *S;
  const double* b;
  const float* dinv;
  int64_t n;
  // device-side control
  int mode;            // BS_RUN: iterating; BS_LAST: the last update done, stop; BS_DONE
  int it, status;      // iterations done, esmp2_status
  double rel;          // last ||r||_W / ||b||_W
};

// state and local block of a block of a launch whose states own `first[s]` ..
// `first[s+1]-1` (first[ns] = total)
__device__ inline int state_of(const int* first, int ns, int blk, int& local) {
  int lo = 0, hi = ns - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= blk) lo = mid;
    else hi = mid - 1;
  }
  local = blk - first[lo];
  return lo;
}

__global__ __launch_bounds__(256) void kb_sym(const BState* S, const int* first, int ns) {
  int local;
  const int s = state_of(first, ns, blockIdx.x, local);
  const BState& B = S[s];
  if (B.mode != BS_RUN) return;
  sym_s2_body<double>(B.d, (const double*)B.p, B.S, local, B.nsym);
}

template <int MV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MV <= 160 ? 5 : 4))) void kb_gemv(const BState* S, const int* first, int ns) {
  int local;
  const int s = state_of(first, ns, blockIdx.x, local);
  const BState& B = S[s];
  if (B.mode != BS_RUN) return;
  gemv_body<double, MV>(B.gv, local, B.ngemv);
}

__global__ __launch_bounds__(256) void kb_arrow(const BState* S, const int* first, int ns) {
  int local;
  const int s = state_of(first, ns, blockIdx.x, local);
  const BState& B = S[s];
  if (B.mode != BS_RUN) return;
  arrow_body<double>(B.aa, B.pt, B.chunks, B.pq, local, B.nchunks);
}

// sc[SC_PQ] = sum of the arrow kernel's per-chunk parts; one block per state
__global__ __launch_bounds__(1024) void kb_finish_pq(BState* S) {
  BState& B = S[blockIdx.x];
  if (B.mode != BS_RUN) return;
  finish_body(B.pq, B.nchunks, B.sc, SC_PQ, 0, 1);
}

// r -= alpha q and the partials of <r, M r>, <r, r>; BATCH_CG_BLOCKS per state
__global__ __launch_bounds__(256) void kb_update_r(BState* S) {
  BState& B = S[blockIdx.x / BATCH_CG_BLOCKS];
  if (B.mode != BS_RUN) return;
  update_r_body<double>(B.r, (const double*)B.q, B.dinv, B.n, B.d.off[1], B.d.off[2], (const double*)B.sc,
                        B.partial, blockIdx.x % BATCH_CG_BLOCKS, BATCH_CG_BLOCKS);
}

// sc[SC_RHO_NEW], sc[SC_RR] from the partials; two blocks per state
__global__ __launch_bounds__(1024) void kb_finish_r(BState* S) {
  BState& B = S[blockIdx.x >> 1];
  if (B.mode != BS_RUN) return;
  finish_body(B.partial, BATCH_CG_BLOCKS, B.sc, SC_RHO_NEW, blockIdx.x & 1, 2);
}

// convergence and the stop, per state on the device; counts the states that
// keep iterating into *active
__global__ void kb_check(BState* S, int ns, double tol, int max_iter, int* active) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ns) return;
  BState& B = S[s];
  if (B.mode != BS_RUN) return;
  const double* sc = B.sc;
  if (!(sc[SC_PQ] > 0.0)) {
    B.status = ESMP2_NOT_SPD;
    B.mode = BS_DONE;
    return;
  }
  B.sc[SC_BX] -= (sc[SC_RHO] / sc[SC_PQ]) * sc[SC_RHO];     // alpha_i rho_i of this iteration
  B.it += 1;
  B.rel = sqrt(sc[SC_RR] / sc[SC_BB]);
  if (B.rel <= tol || B.it >= max_iter) {
    B.mode = BS_LAST;
    if (B.rel > tol) B.status = ESMP2_NOT_CONVERGED;
  } else {
    atomicAdd(active, 1);
  }
}

// p = M r + beta p for a state that goes on; BATCH_CG_BLOCKS per state
__global__ __launch_bounds__(256) void kb_update(BState* S) {
  BState& B = S[blockIdx.x / BATCH_CG_BLOCKS];
  const int bid = blockIdx.x % BATCH_CG_BLOCKS;
  if (B.mode == BS_RUN)
    update_p_body<double>(B.p, (const double*)B.r, B.dinv, B.n, (const double*)B.sc, bid, BATCH_CG_BLOCKS);
}

// rho <- rho_new for the states that go on; BS_LAST -> BS_DONE
__global__ void kb_roll(BState* S, int ns) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ns) return;
  BState& B = S[s];
  if (B.mode == BS_RUN) B.sc[SC_RHO] = B.sc[SC_RHO_NEW];
  else if (B.mode == BS_LAST) B.mode = BS_DONE;
}

// start (x = 0): r = -b, p = M r, partials of <r, M r>, <r, r>, and <b, b>
__global__ __launch_bounds__(256) void kb_init(BState* S) {
  BState& B = S[blockIdx.x / BATCH_CG_BLOCKS];
  const int bid = blockIdx.x % BATCH_CG_BLOCKS;
  init_body(B.b, (const double*)nullptr, B.r, B.p, B.dinv, B.n, B.d.off[1], B.d.off[2], B.partial, bid,
            BATCH_CG_BLOCKS);
}

__global__ __launch_bounds__(256) void kb_dot_bb(BState* S) {
  BState& B = S[blockIdx.x / BATCH_CG_BLOCKS];
  dot_body<double>(B.b, B.b, B.n, B.d.off[1], B.d.off[2], B.partial + 2 * BATCH_CG_BLOCKS,
                   blockIdx.x % BATCH_CG_BLOCKS, BATCH_CG_BLOCKS);
}

// sc[SC_RHO] = <r, M r>, sc[SC_RR] = <r, r> and sc[SC_BB] = <b, b> of the start;
// three blocks per state
__global__ __launch_bounds__(1024) void kb_finish_init(BState* S) {
  BState& B = S[blockIdx.x / 3];
  const int k = blockIdx.x % 3;
  if (k == 0) finish_body(B.partial, BATCH_CG_BLOCKS, B.sc, SC_RHO, 0, 2);
  else if (k == 1) finish_body(B.partial, BATCH_CG_BLOCKS, B.sc, SC_RR - 1, 1, 2);
  else finish_body(B.partial + 2 * BATCH_CG_BLOCKS, BATCH_CG_BLOCKS, B.sc, SC_BB, 0, 1);
}

// a state converged at the start stops with zero iterations
__global__ void kb_zero(int* v) {
  if (threadIdx.x == 0) v[0] = 0;
}

__global__ void kb_start(BState* S, int ns, double tol, int* active) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ns) return;
  BState& B = S[s];
  B.it = 0;
  B.status = ESMP2_OK;
  B.sc[SC_BX] = 0.0;
  B.sc[SC_XR] = 0.0;
  B.rel = sqrt(B.sc[SC_RR] / B.sc[SC_BB]);
  if (B.rel <= tol) {
    B.mode = BS_DONE;
  } else {
    B.mode = BS_RUN;
    atomicAdd(active, 1);
  }
}

}  // namespace esmp2
