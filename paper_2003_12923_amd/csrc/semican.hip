// The first-order problem in the pinned-semicanonical basis.
//
// Doubles + L-triples are mapped onto themselves by any rotation of the
// occupied orbitals other than t and of the virtuals other than t' (an
// L-triple keeps t among its holes and t' among its particles, Sec. II.B and
// the Q F Q replacement of Sec. II.C), so A = (H0 - E0) restricted to D + L
// is covariant under such rotations and E2_DL = -b^T A^-1 b is unchanged.
// Rotating so that the non-pinned Fock blocks F_oo[1:,1:] and F_vv[1:,1:] are
// diagonal leaves an operator whose off-diagonal part is only the Fock row
// of t / t' and f_ov, so Jacobi-preconditioned CG converges in far fewer
// iterations.  The right-hand side is built in the TOP basis and rotated
// once; the solution is rotated back on request.
//
// Amplitude rotation of one box: unpack to a dense tensor X[P][Q][A][B] over
// the box's free-index ranges, contract each index with the matching block of
// the rotation (four GEMMs), pack.
#include "common.h"
#include "sigma.h"
#include "reduce.h"

namespace esmp2 {

// dst (m x m, contiguous) = src[off + r*ld + c]
__global__ void k_block_copy(const double* src, int64_t off, int ld, int m, double* dst) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < m * m; e += gridDim.x * blockDim.x)
    dst[e] = src[off + (int64_t)(e / m) * ld + (e % m)];
}

// eigenpair of a 1 x 1 matrix
__global__ void k_eig1(const double* A, double* evals, double* Y) {
  evals[0] = A[0];
  Y[0] = 1.0;
}

// T (n x n) = identity with T[1:, 1:] = Y (Y: (n-1) x (n-1), column k = eigenvector k).
// Each eigenvector is signed so that its largest-magnitude entry is positive.
__global__ __launch_bounds__(64) void k_embed_rotation(const double* Y, int n, double* T) {
  // one wavefront per column c of T
  const int m = n - 1, c = blockIdx.x, l = threadIdx.x;
  if (c == 0) {
    for (int r = l; r < n; r += 64) T[r * n] = r == 0 ? 1.0 : 0.0;
    return;
  }
  const double sg = col_sign(Y + (c - 1), m, m, l);
  if (l == 0) T[c] = 0.0;
  for (int r = 1 + l; r < n; r += 64) T[r * n + c] = sg * Y[(r - 1) * m + (c - 1)];
}

// T (n x n) = blkdiag(To, Tv)
__global__ void k_blkdiag(const double* To, const double* Tv, int no, int nv, double* T) {
  const int n = no + nv;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n * n; e += gridDim.x * blockDim.x) {
    const int r = e / n, c = e % n;
    double v = 0.0;
    if (r < no && c < no) v = To[r * no + c];
    else if (r >= no && c >= no) v = Tv[(r - no) * nv + (c - no)];
    T[e] = v;
  }
}

// Fock blocks of the operator from the rotated Fock matrix Fh, with the
// TOP-basis constants omega and kappa (they read TOP orbitals' diagonal
// elements, which the rotation does not preserve).
__global__ void k_fock_blocks(const double* Fh, int no, int nv, int mv, double om, double ka, double* fo,
                              double* fv, double* fov, double* eo, double* ev, double* Fd, double* Fl) {
  const int n = no + nv;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < (int64_t)mv * mv) {
    const int a = g / mv, b = g % mv;
    const double v = (a < nv && b < nv) ? 0.5 * (Fh[(no + a) * n + no + b] + Fh[(no + b) * n + no + a]) : 0.0;
    Fd[g] = v + ((a == b && a < nv) ? -0.5 * om : 0.0);
    Fl[g] = v + ((a == b && a < nv) ? 0.5 * ka : 0.0);
    if (a < nv && b < nv) fv[a * nv + b] = v;
  }
  if (g < no * no) fo[g] = Fh[(g / no) * n + g % no];
  if (g < no * nv) fov[g] = Fh[(g / nv) * n + no + g % nv];
  if (g < no) eo[g] = Fh[g * n + g];
  if (g < nv) ev[g] = Fh[(no + g) * n + no + g];
}

// free-index ranges of a box: occupied from lo_o, virtual from lo_v (0 or 1)
__host__ __device__ inline void box_ranges(int box, int& lo_o, int& lo_v) {
  lo_o = (box == B_T3 || box == B_H21 || box == B_H22) ? 1 : 0;
  lo_v = (box == B_T3 || box == B_H12 || box == B_H22) ? 1 : 0;
}

// dense[P][Q][A][B] (ranges ro = no - lo_o, rv = nv - lo_v) of one box of x
__global__ void k_unpack_box(Dims d, int box, const double* x, double* dense) {
  int lo_o, lo_v;
  box_ranges(box, lo_o, lo_v);
  const int ro = d.no - lo_o, rv = d.nv - lo_v;
  const int64_t n = (int64_t)ro * ro * rv * rv;
  Look<double> L{d, x, x + d.off[B_S2]};
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int B = (int)(e % rv), A = (int)((e / rv) % rv);
    const int64_t o = e / ((int64_t)rv * rv);
    const int Q = (int)(o % ro) + lo_o, P = (int)(o / ro) + lo_o;
    const int a = A + lo_v, b = B + lo_v;
    double v;
    switch (box) {
      case B_T2: v = L.T2(P, Q, a, b); break;
      case B_S2: v = L.St(P, Q, a, b); break;      // raw S2 amplitudes (S = x of the S2 box)
      case B_T3: v = L.T3(P, Q, a, b); break;
      case B_H11: v = L.H11(P, Q, a, b); break;
      case B_H12: v = L.H12(P, Q, a, b); break;
      case B_H21: v = L.H21(P, Q, a, b); break;
      default: v = L.H22(P, Q, a, b); break;
    }
    dense[e] = v;
  }
}

// one box of y from dense[P][Q][A][B] (its unique elements)
__global__ void k_pack_box(Dims d, int box, const double* dense, double* y) {
  int lo_o, lo_v;
  box_ranges(box, lo_o, lo_v);
  const int ro = d.no - lo_o, rv = d.nv - lo_v;
  const int64_t n = d.off[box + 1] - d.off[box];
  const bool anti_o = (box == B_T2 || box == B_T3 || box == B_H11 || box == B_H12);
  const bool anti_v = (box == B_T2 || box == B_T3 || box == B_H11 || box == B_H21);
  const int64_t inner = anti_v ? (int64_t)rv * (rv - 1) / 2 : (int64_t)rv * rv;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int o = (int)(e / inner), v = (int)(e % inner);
    int P, Q, A, B;
    if (anti_o) tri_pq(o, ro, P, Q); else { P = o / ro; Q = o % ro; }
    if (anti_v) tri_pq(v, rv, A, B); else { A = v / rv; B = v % rv; }
    y[d.off[box] + e] = dense[(((int64_t)P * ro + Q) * rv + A) * rv + B];
  }
}

// Rotation of one occupied index of dense[P][Q][v] (ranges ro, ro, nvv):
//   which = 1: out[P][Q'][v] = sum_Q G(Q, Q') in[P][Q][v]
//   which = 0: out[P'][Q][v] = sum_P G(P, P') in[P][Q][v]
// G(c, c') = Gm[c*sr + c'*sc], staged in LDS.  Thread per (fixed occupied index, v):
// ro coalesced loads, ro^2 multiply-adds, ro coalesced stores; R >= ro is the
// compile-time bound that keeps the accumulators in registers.
template <int R>
__global__ __launch_bounds__(256) void k_rot_occ(const double* in, double* out, const double* Gm, int64_t sr,
                                                 int64_t sc, int ro, int64_t nvv, int which) {
  __shared__ double G[R * R];
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) {
    const int c = e / R, c2 = e % R;
    G[e] = (c < ro && c2 < ro) ? Gm[c * sr + c2 * sc] : 0.0;
  }
  __syncthreads();
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int f = blockIdx.y;                          // the occupied index that stays
  if (v >= nvv) return;
  double acc[R];
#pragma unroll
  for (int c2 = 0; c2 < R; ++c2) acc[c2] = 0.0;
#pragma unroll
  for (int c = 0; c < R; ++c) {
    if (c < ro) {
      const int64_t src = which == 1 ? ((int64_t)f * ro + c) * nvv + v : ((int64_t)c * ro + f) * nvv + v;
      const double y = in[src];
#pragma unroll
      for (int c2 = 0; c2 < R; ++c2) acc[c2] += G[c * R + c2] * y;
    }
  }
#pragma unroll
  for (int c2 = 0; c2 < R; ++c2) {
    if (c2 < ro) {
      const int64_t dst = which == 1 ? ((int64_t)f * ro + c2) * nvv + v : ((int64_t)c2 * ro + f) * nvv + v;
      out[dst] = acc[c2];
    }
  }
}

// ---------------------------------------------------------------------------
// Fock operator of the reference's density: F = h + J[gamma] - K[gamma]/2
// ---------------------------------------------------------------------------
// gamma (spin-summed, input orbital basis): 2 delta - C C^T (occupied block),
// C^T C (virtual block), zero between them
__global__ void k_ref_density(const double* C, int no, int nv, double* gam) {
  const int n = no + nv;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n * n; e += gridDim.x * blockDim.x) {
    const int p = e / n, q = e % n;
    double v = 0.0;
    if (p < no && q < no) {
      for (int a = 0; a < nv; ++a) v -= C[p * nv + a] * C[q * nv + a];
      if (p == q) v += 2.0;
    } else if (p >= no && q >= no) {
      for (int i = 0; i < no; ++i) v += C[i * nv + (p - no)] * C[i * nv + (q - no)];
    }
    gam[e] = v;
  }
}

// d[Q] = sum_rs B[Q][r][s] gamma[r][s]; one workgroup per Q
__global__ __launch_bounds__(256) void k_coulomb_weights(const double* B, const double* gam, int n, double* d) {
  const double* b = B + (int64_t)blockIdx.x * n * n;
  double acc = 0.0;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) acc += b[e] * gam[e];
  const double s = block_sum(acc);
  if (threadIdx.x == 0) d[blockIdx.x] = s;
}

// F = h + sum_Q d[Q] B[Q] - K / 2
__global__ void k_fock_combine(const double* hcore, const double* B, const double* d, const double* K, int n,
                               int naux, double* F) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n * n; e += gridDim.x * blockDim.x) {
    double j = 0.0;
    for (int Q = 0; Q < naux; ++Q) j += d[Q] * B[(int64_t)Q * n * n + e];
    F[e] = hcore[e] + j - 0.5 * K[e];
  }
}

template __global__ void k_rot_occ<16>(const double*, double*, const double*, int64_t, int64_t, int, int64_t, int);
template __global__ void k_rot_occ<32>(const double*, double*, const double*, int64_t, int64_t, int, int64_t, int);
template __global__ void k_rot_occ<64>(const double*, double*, const double*, int64_t, int64_t, int, int64_t, int);

}  // namespace esmp2
