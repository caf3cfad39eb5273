// Dense linear algebra for the TOP-basis rotation (paper Sec. II.A):
//   - a batched FP64 matrix-core GEMM with arbitrary strides,
//   - one-sided Jacobi SVD of the singles coefficients C (n_occ x n_vir),
//   - cyclic Jacobi eigensolver for the Fock matrix restricted to the span of
//     the additional virtual orbitals (semicanonical AVOs),
//   - assembly of the orthogonal rotation R.
#include "common.h"
#include "mfma.h"
#include <math.h>

namespace esmp2 {

// ---------------------------------------------------------------------------
// C[b] = alpha * A[b] * B[b] + beta * C[b]
//   A(i,k) = A[b*sAb + i*sAi + k*sAk],  B(k,j) = B[b*sBb + k*sBk + j*sBj],
//   C(i,j) = C[b*sCb + i*sCi + j*sCj].  Tile 64x64x16, 4 wavefronts of 32x32.
// ---------------------------------------------------------------------------
struct GemmArgs {
  const double* A; const double* B; double* C;
  int M, N, K;
  int64_t sAb, sAi, sAk, sBb, sBk, sBj, sCb, sCi, sCj;
  double alpha, beta;
};

__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  __shared__ double As[16][64 + 1];
  __shared__ double Bs[16][64 + 1];
  const int b = blockIdx.z;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const double* A = g.A + b * g.sAb;
  const double* Bm = g.B + b * g.sBb;
  f64x4 acc[2][2];
  for (int i = 0; i < 2; ++i) for (int j = 0; j < 2; ++j) acc[i][j] = (f64x4){0, 0, 0, 0};
  const bool a_kfast = (g.sAk == 1);
  const bool b_jfast = (g.sBj == 1) || (g.sBk != 1);
  for (int k0 = 0; k0 < g.K; k0 += 16) {
    for (int r = 0; r < 4; ++r) {
      int e = tid + 256 * r;
      int mm, kk;
      if (a_kfast) { mm = e >> 4; kk = e & 15; } else { mm = e & 63; kk = e >> 6; }
      int gi = m0 + mm, gk = k0 + kk;
      As[kk][mm] = (gi < g.M && gk < g.K) ? A[gi * g.sAi + gk * g.sAk] : 0.0;
      int nn;
      if (b_jfast) { nn = e & 63; kk = e >> 6; } else { nn = e >> 4; kk = e & 15; }
      int gj = n0 + nn;
      gk = k0 + kk;
      Bs[kk][nn] = (gj < g.N && gk < g.K) ? Bm[gk * g.sBk + gj * g.sBj] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      double a0 = As[ks * 4 + (l >> 4)][wm + (l & 15)];
      double a1 = As[ks * 4 + (l >> 4)][wm + 16 + (l & 15)];
      double b0 = Bs[ks * 4 + (l >> 4)][wn + (l & 15)];
      double b1 = Bs[ks * 4 + (l >> 4)][wn + 16 + (l & 15)];
      acc[0][0] = mfma16x16x4(a0, b0, acc[0][0]);
      acc[0][1] = mfma16x16x4(a0, b1, acc[0][1]);
      acc[1][0] = mfma16x16x4(a1, b0, acc[1][0]);
      acc[1][1] = mfma16x16x4(a1, b1, acc[1][1]);
    }
    __syncthreads();
  }
  double* C = g.C + b * g.sCb;
  for (int ti = 0; ti < 2; ++ti)
    for (int tj = 0; tj < 2; ++tj)
      for (int i = 0; i < 4; ++i) {
        int gi = m0 + wm + ti * 16 + mfma_row(l, i);
        int gj = n0 + wn + tj * 16 + (l & 15);
        if (gi < g.M && gj < g.N) {
          double v = g.alpha * acc[ti][tj][i];
          int64_t o = gi * g.sCi + gj * g.sCj;
          C[o] = (g.beta == 0.0) ? v : v + g.beta * C[o];
        }
      }
}

hipError_t gemm(hipStream_t s, int batch, const GemmArgs& g) {
  if (g.M <= 0 || g.N <= 0 || batch <= 0) return hipSuccess;
  dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, batch);
  hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, g);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// One-sided Jacobi SVD of C (no x nv, no <= nv, no <= 64, no*nv <= 8192):
// rows of C are rotated pairwise until mutually orthogonal; C = U diag(lam) Vt.
// Outputs (descending lam, sign convention of the TOP basis):
//   lam[no], U[no][no] (column l = occupied TOP orbital l), V[nv][no].
// Round-robin pairing; one wavefront per pair.  Single workgroup (1024 threads).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_svd_jacobi(const double* __restrict__ Cin, int no, int nv,
                                                     double* lam, double* U, double* V, int* info) {
  extern __shared__ double sm[];
  double* C = sm;                 // no*nv
  double* Us = C + no * nv;       // no*no
  __shared__ int order[66];
  __shared__ double nrm[64];
  __shared__ int rotated;
  const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63, nwave = blockDim.x >> 6;
  for (int e = tid; e < no * nv; e += blockDim.x) C[e] = Cin[e];
  for (int e = tid; e < no * no; e += blockDim.x) Us[e] = (e / no == e % no) ? 1.0 : 0.0;
  const int P = (no + 1) / 2 * 2;   // players (one dummy if odd)
  __syncthreads();
  int sweep = 0;
  for (; sweep < 60; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int r = 0; r < P - 1; ++r) {
      for (int pr = wave; pr < P / 2; pr += nwave) {
        auto player = [&](int k) { return k == 0 ? 0 : 1 + (k - 1 + r) % (P - 1); };
        int p = player(pr), q = player(P - 1 - pr);
        if (p > q) { int t = p; p = q; q = t; }
        if (q >= no) continue;
        double al = 0, be = 0, ga = 0;
        for (int a = l; a < nv; a += 64) {
          double x = C[p * nv + a], y = C[q * nv + a];
          al += x * x; be += y * y; ga += x * y;
        }
        for (int o = 32; o > 0; o >>= 1) {
          al += __shfl_xor(al, o); be += __shfl_xor(be, o); ga += __shfl_xor(ga, o);
        }
        if (fabs(ga) > 1e-15 * sqrt(al * be) && fabs(ga) > 1e-300) {
          double ze = (be - al) / (2.0 * ga);
          double t = (ze >= 0 ? 1.0 : -1.0) / (fabs(ze) + sqrt(1.0 + ze * ze));
          double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
          for (int a = l; a < nv; a += 64) {
            double x = C[p * nv + a], y = C[q * nv + a];
            C[p * nv + a] = c * x - s * y;
            C[q * nv + a] = s * x + c * y;
          }
          for (int k = l; k < no; k += 64) {
            double x = Us[k * no + p], y = Us[k * no + q];
            Us[k * no + p] = c * x - s * y;
            Us[k * no + q] = s * x + c * y;
          }
          if (l == 0) rotated = 1;
        }
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }
  // norms and descending order
  for (int k = wave; k < no; k += nwave) {
    double s2 = 0;
    for (int a = l; a < nv; a += 64) s2 += C[k * nv + a] * C[k * nv + a];
    for (int o = 32; o > 0; o >>= 1) s2 += __shfl_xor(s2, o);
    if (l == 0) nrm[k] = sqrt(s2);
  }
  __syncthreads();
  if (tid == 0) {
    for (int k = 0; k < no; ++k) order[k] = k;
    for (int i = 0; i < no; ++i)
      for (int j = i + 1; j < no; ++j)
        if (nrm[order[j]] > nrm[order[i]]) { int t = order[i]; order[i] = order[j]; order[j] = t; }
    info[0] = sweep;
  }
  __syncthreads();
  // outputs with the sign convention: U column largest-|entry| positive
  for (int k = wave; k < no; k += nwave) {
    int src = order[k];
    double best = 0; int bi = 0;
    if (l == 0) {
      for (int i = 0; i < no; ++i) {
        double v = fabs(Us[i * no + src]);
        if (v > best) { best = v; bi = i; }
      }
    }
    bi = __shfl(bi, 0);
    double sg = Us[bi * no + src] < 0 ? -1.0 : 1.0;
    double lk = nrm[src];
    if (l == 0) lam[k] = lk;
    for (int i = l; i < no; i += 64) U[i * no + k] = sg * Us[i * no + src];
    double inv = lk > 0 ? sg / lk : 0.0;
    for (int a = l; a < nv; a += 64) V[a * no + k] = inv * C[src * nv + a];
  }
  __syncthreads();
  // rank-deficient rows: complete V by Gram-Schmidt against unit vectors
  if (wave == 0) {
    double lmax = lam[0];
    for (int k = 0; k < no; ++k) {
      if (lam[k] > 1e-12 * lmax) continue;
      for (int e = 0; e < nv; ++e) {
        // candidate e_e orthogonalised against columns 0..k-1 (twice)
        for (int a = l; a < nv; a += 64) V[a * no + k] = (a == e) ? 1.0 : 0.0;
        for (int pass = 0; pass < 2; ++pass)
          for (int m = 0; m < no; ++m) {
            if (m == k || (m > k && lam[m] <= 1e-12 * lmax)) continue;
            double d = 0;
            for (int a = l; a < nv; a += 64) d += V[a * no + m] * V[a * no + k];
            for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o);
            for (int a = l; a < nv; a += 64) V[a * no + k] -= d * V[a * no + m];
          }
        double s2 = 0;
        for (int a = l; a < nv; a += 64) s2 += V[a * no + k] * V[a * no + k];
        for (int o = 32; o > 0; o >>= 1) s2 += __shfl_xor(s2, o);
        if (s2 > 0.25) {
          double inv = 1.0 / sqrt(s2);
          for (int a = l; a < nv; a += 64) V[a * no + k] *= inv;
          break;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// M = P F_vv P + shift * V V^T with P = 1 - V V^T (nv x nv), whose spectrum is
// {shift (n_occ-fold, span of the TOP virtuals)} + {eigenvalues of F in the AVO
// span}.  W = F_vv V and G = V^T F_vv V are formed first.
// ---------------------------------------------------------------------------
__global__ void k_fv_times_v(const double* F, int n, int no, int nv, const double* V, double* W) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nv * no) return;
  int a = e / no, k = e % no;
  double s = 0;
  for (int b = 0; b < nv; ++b) s += F[(no + a) * n + no + b] * V[b * no + k];
  W[a * no + k] = s;
}

__global__ void k_vt_w(const double* V, const double* W, int no, int nv, double* G) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= no * no) return;
  int k = e / no, m = e % no;
  double s = 0;
  for (int a = 0; a < nv; ++a) s += V[a * no + k] * W[a * no + m];
  G[k * no + m] = s;
}

__global__ void k_build_m(const double* F, int n, int no, int nv, const double* V, const double* W,
                          const double* G, double shift, double* M) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nv * nv) return;
  int a = e / nv, b = e % nv;
  double s = F[(no + a) * n + no + b];
  for (int k = 0; k < no; ++k) {
    s -= V[a * no + k] * W[b * no + k] + W[a * no + k] * V[b * no + k];
    double t = 0;
    for (int m = 0; m < no; ++m) t += (G[k * no + m] + (k == m ? shift : 0.0)) * V[b * no + m];
    s += V[a * no + k] * t;
  }
  M[a * nv + b] = s;
}

// ---------------------------------------------------------------------------
// Cyclic (round-robin parallel) Jacobi eigensolver for a symmetric n x n matrix
// held packed (upper triangle) in LDS.  Rotation parameters of every round are
// written to `rot` (2 doubles per pair); eigenvalues to `evals`.  The
// eigenvectors are formed afterwards by k_jacobi_vectors.
// rot layout: [sweep][round][pair] (c, s), P/2 pairs per round, P-1 rounds.
// ---------------------------------------------------------------------------
__device__ inline int pk(int r, int c, int n) {   // packed upper index (r <= c)
  return r * n - r * (r - 1) / 2 + (c - r);
}

__global__ __launch_bounds__(1024) void k_eig_jacobi(const double* __restrict__ Min, int n, int max_sweeps,
                                                     double* rot, double* evals, int* info) {
  extern __shared__ double A[];          // n(n+1)/2 packed
  __shared__ double cs[2 * 256];
  __shared__ int pp[256], qq[256];
  __shared__ double offs[1024 / 64];
  __shared__ double tot[1024 / 64];
  __shared__ int done;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int P = (n + 1) / 2 * 2, npair = P / 2;
  for (int r = 0; r < n; ++r)
    for (int c = r + tid; c < n; c += nt) A[pk(r, c, n)] = Min[r * n + c];
  __syncthreads();
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    // convergence test: off-diagonal vs diagonal Frobenius norm, both summed
    // directly (a difference of the two would drown the test in cancellation)
    double off = 0, dg = 0;
    for (int r = 0; r < n; ++r)
      for (int c = r + 1 + tid; c < n; c += nt) { double v = A[pk(r, c, n)]; off += v * v; }
    for (int r = tid; r < n; r += nt) { double v = A[pk(r, r, n)]; dg += v * v; }
    for (int o = 32; o > 0; o >>= 1) { off += __shfl_xor(off, o); dg += __shfl_xor(dg, o); }
    if ((tid & 63) == 0) { offs[tid >> 6] = off; tot[tid >> 6] = dg; }
    __syncthreads();
    if (tid == 0) {
      double so = 0, sd = 0;
      for (int w = 0; w < nt / 64; ++w) { so += offs[w]; sd += tot[w]; }
      done = (so <= 1e-34 * sd);
    }
    __syncthreads();
    if (done) break;
    for (int r = 0; r < P - 1; ++r) {
      for (int k = tid; k < npair; k += nt) {
        auto player = [&](int x) { return x == 0 ? 0 : 1 + (x - 1 + r) % (P - 1); };
        int p = player(k), q = player(P - 1 - k);
        if (p > q) { int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0;
        if (q < n) {
          double apq = A[pk(p, q, n)];
          if (apq != 0.0) {
            double tau = (A[pk(q, q, n)] - A[pk(p, p, n)]) / (2.0 * apq);
            double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        pp[k] = p; qq[k] = q;
        cs[2 * k] = c; cs[2 * k + 1] = s;
        int64_t o = ((int64_t)sweep * (P - 1) + r) * npair + k;
        rot[2 * o] = c; rot[2 * o + 1] = s;
      }
      __syncthreads();
      // A <- J^T A J, block by block over pairs (X, Y) with X <= Y
      int nblk = npair * (npair + 1) / 2;
      for (int bi = tid; bi < nblk; bi += nt) {
        // decode bi -> (X, Y), X <= Y
        int X = 0, rem = bi;
        while (rem >= npair - X) { rem -= npair - X; ++X; }
        int Y = X + rem;
        int x0 = pp[X], x1 = qq[X], y0 = pp[Y], y1 = qq[Y];
        double cx = cs[2 * X], sx = cs[2 * X + 1], cy = cs[2 * Y], sy = cs[2 * Y + 1];
        bool vx1 = x1 < n, vy1 = y1 < n;
        auto get = [&](int r, int c) -> double {
          return (r <= c) ? A[pk(r, c, n)] : A[pk(c, r, n)];
        };
        auto put = [&](int r, int c, double v) {
          if (r <= c) A[pk(r, c, n)] = v; else A[pk(c, r, n)] = v;
        };
        if (X == Y) {
          if (!vx1) continue;
          double app = get(x0, x0), aqq = get(x1, x1), apq = get(x0, x1);
          double t = (cx != 0.0) ? sx / cx : 0.0;
          put(x0, x0, app - t * apq);
          put(x1, x1, aqq + t * apq);
          put(x0, x1, 0.0);
        } else {
          // rows (x0,x1) with J_X, columns (y0,y1) with J_Y; J = [c s; -s c]
          double a00 = get(x0, y0);
          double a01 = vy1 ? get(x0, y1) : 0.0;
          double a10 = vx1 ? get(x1, y0) : 0.0;
          double a11 = (vx1 && vy1) ? get(x1, y1) : 0.0;
          // left: rows' = J_X^T rows
          double b00 = cx * a00 - sx * a10, b01 = cx * a01 - sx * a11;
          double b10 = sx * a00 + cx * a10, b11 = sx * a01 + cx * a11;
          // right: cols' = cols J_Y
          double c00 = b00 * cy - b01 * sy, c01 = b00 * sy + b01 * cy;
          double c10 = b10 * cy - b11 * sy, c11 = b10 * sy + b11 * cy;
          put(x0, y0, c00);
          if (vy1) put(x0, y1, c01);
          if (vx1) put(x1, y0, c10);
          if (vx1 && vy1) put(x1, y1, c11);
        }
      }
      __syncthreads();
    }
  }
  for (int r = tid; r < n; r += nt) evals[r] = A[pk(r, r, n)];
  if (tid == 0) info[0] = sweep;
}

// Z = J_1 J_2 ... J_R applied to the identity; one row of Z per workgroup of
// one wavefront: z <- z J with z'_p = c z_p - s z_q, z'_q = s z_p + c z_q.
// Z[n][n] row-major.  Launch: grid n, block 64, dynamic LDS n doubles.
__global__ __launch_bounds__(64) void k_jacobi_vectors(const double* rot, int n, const int* sweeps, double* Z) {
  extern __shared__ double zr[];
  const int l = threadIdx.x;
  const int row = blockIdx.x;
  for (int c = l; c < n; c += 64) zr[c] = (c == row) ? 1.0 : 0.0;
  __syncthreads();
  const int P = (n + 1) / 2 * 2, npair = P / 2;
  const int ns = sweeps[0];
  for (int sw = 0; sw < ns; ++sw)
    for (int r = 0; r < P - 1; ++r) {
      int64_t base = ((int64_t)sw * (P - 1) + r) * npair;
      for (int k = l; k < npair; k += 64) {
        int p = (k == 0) ? 0 : 1 + (k - 1 + r) % (P - 1);
        int q = 1 + (P - 1 - k - 1 + r) % (P - 1);
        if (p > q) { int t = p; p = q; q = t; }
        if (q >= n) continue;
        double c = rot[2 * (base + k)], s = rot[2 * (base + k) + 1];
        double zp = zr[p], zq = zr[q];
        zr[p] = c * zp - s * zq;
        zr[q] = s * zp + c * zq;
      }
      __syncthreads();
    }
  for (int c = l; c < n; c += 64) Z[(int64_t)row * n + c] = zr[c];
}

// Sort eigenpairs ascending, drop the n_occ lowest (the TOP-virtual span held at
// `shift`), sign each AVO (largest-|entry| positive) and assemble the rotation
//   R[:no,:no] = U,  R[no:, no:no+no] = V,  R[no:, 2no:] = AVOs.
__global__ void k_assemble_r(const double* U, const double* V, const double* Z, const double* evals,
                             int no, int nv, double* R, double* avo_eps) {
  __shared__ int order[1024];
  const int n = no + nv;
  const int tid = threadIdx.x;
  if (tid == 0) {
    for (int k = 0; k < nv; ++k) order[k] = k;
    for (int i = 1; i < nv; ++i) {          // insertion sort by eigenvalue
      int key = order[i]; double kv = evals[key]; int j = i - 1;
      while (j >= 0 && evals[order[j]] > kv) { order[j + 1] = order[j]; --j; }
      order[j + 1] = key;
    }
  }
  __syncthreads();
  for (int e = tid; e < n * n; e += blockDim.x) R[e] = 0.0;
  __syncthreads();
  for (int e = tid; e < no * no; e += blockDim.x) R[(e / no) * n + (e % no)] = U[e];
  for (int e = tid; e < nv * no; e += blockDim.x) R[(no + e / no) * n + no + (e % no)] = V[e];
  for (int k = tid; k < nv - no; k += blockDim.x) {
    int src = order[no + k];
    // eigenvector = column src of Z (Z rows are e_r^T J...; A = Z diag Z^T)
    double best = 0, sg = 1.0;
    for (int a = 0; a < nv; ++a) {
      double v = Z[a * nv + src];
      if (fabs(v) > best) { best = fabs(v); sg = v < 0 ? -1.0 : 1.0; }
    }
    for (int a = 0; a < nv; ++a) R[(no + a) * n + 2 * no + k] = sg * Z[a * nv + src];
    avo_eps[k] = evals[src];
  }
}

}  // namespace esmp2
