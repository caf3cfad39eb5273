// Dense linear algebra for the TOP-basis rotation (paper Sec. II.A):
//   - a batched FP64 matrix-core GEMM with arbitrary strides,
//   - one-sided Jacobi SVD of the singles coefficients C (n_occ x n_vir),
//   - a symmetric eigensolver (Householder tridiagonalisation, multisection on
//     Sturm counts, twisted-factorisation eigenvectors) for the Fock matrix
//     restricted to the span of the additional virtual orbitals (semicanonical
//     AVOs) and to the non-pinned occupied and virtual orbitals,
//   - assembly of the orthogonal rotation R.
#include "common.h"
#include "mfma.h"
#include "reduce.h"
#include <math.h>
#include <rocblas/rocblas.h>
#include <algorithm>
#include <vector>

namespace esmp2 {

// ---------------------------------------------------------------------------
// C[b] = alpha * A[b] * B[b] + beta * C[b]
//   A(i,k) = A[b*sAb + i*sAi + k*sAk],  B(k,j) = B[b*sBb + k*sBk + j*sBj],
//   C(i,j) = C[b*sCb + i*sCi + j*sCj].  Tile 64x64x16, 4 wavefronts of 32x32,
//   double-buffered K chunks.
// ---------------------------------------------------------------------------
struct GemmArgs {
  const double* A; const double* B; double* C;
  int M, N, K;
  int64_t sAb, sAi, sAk, sBb, sBk, sBj, sCb, sCi, sCj;
  double alpha, beta;
};

__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  __shared__ double As[2][16][64 + 1];
  __shared__ double Bs[2][16][64 + 1];
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
  // K chunks of 16 through two LDS buffers: the next chunk is loaded into
  // registers while the current one is multiplied (loads always in bounds: an
  // element outside the matrix reads element 0 and is replaced by zero)
  double ra[4], rb[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + 256 * r;
      int mm, kk;
      if (a_kfast) { mm = e >> 4; kk = e & 15; } else { mm = e & 63; kk = e >> 6; }
      const int gi = m0 + mm, gk = k0 + kk;
      const bool oka = gi < g.M && gk < g.K;
      const double va = A[oka ? gi * g.sAi + gk * g.sAk : 0];
      ra[r] = oka ? va : 0.0;
      int nn;
      if (b_jfast) { nn = e & 63; kk = e >> 6; } else { nn = e >> 4; kk = e & 15; }
      const int gj = n0 + nn, gk2 = k0 + kk;
      const bool okb = gj < g.N && gk2 < g.K;
      const double vb = Bm[okb ? gk2 * g.sBk + gj * g.sBj : 0];
      rb[r] = okb ? vb : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + 256 * r;
      int mm, kk;
      if (a_kfast) { mm = e >> 4; kk = e & 15; } else { mm = e & 63; kk = e >> 6; }
      As[buf][kk][mm] = ra[r];
      int nn;
      if (b_jfast) { nn = e & 63; kk = e >> 6; } else { nn = e >> 4; kk = e & 15; }
      Bs[buf][kk][nn] = rb[r];
    }
  };
  load(0);
  store(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < g.K; k0 += 16) {
    const bool more = k0 + 16 < g.K;
    if (more) load(k0 + 16);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      double a0 = As[buf][ks * 4 + (l >> 4)][wm + (l & 15)];
      double a1 = As[buf][ks * 4 + (l >> 4)][wm + 16 + (l & 15)];
      double b0 = Bs[buf][ks * 4 + (l >> 4)][wn + (l & 15)];
      double b1 = Bs[buf][ks * 4 + (l >> 4)][wn + 16 + (l & 15)];
      acc[0][0] = mfma16x16x4(a0, b0, acc[0][0]);
      acc[0][1] = mfma16x16x4(a0, b1, acc[0][1]);
      acc[1][0] = mfma16x16x4(a1, b0, acc[1][0]);
      acc[1][1] = mfma16x16x4(a1, b1, acc[1][1]);
    }
    // the other buffer was last read before the previous barrier
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
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

// the hand-written kernel (allocates nothing)
hipError_t gemm_native(hipStream_t s, int batch, const GemmArgs& g) {
  if (g.M <= 0 || g.N <= 0 || batch <= 0) return hipSuccess;
  dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, batch);
  hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, g);
  return hipGetLastError();
}

// rocBLAS handle of this host thread on the current device (created on first
// use, kept until the process ends); null if it cannot be created
static rocblas_handle blas_handle() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return nullptr;
  thread_local std::vector<rocblas_handle> hs;
  if ((int)hs.size() <= dev) hs.resize(dev + 1, nullptr);
  if (!hs[dev] && rocblas_create_handle(&hs[dev]) != rocblas_status_success) hs[dev] = nullptr;
  return hs[dev];
}

// One column-major operand of rocBLAS from a strided one: element (r, c) of an
// R x C matrix at r * sr + c * sc.  Unit row stride: op N, ld = sc; unit column
// stride: op T of the stored C x R matrix, ld = sr.  False if neither is unit or
// the leading dimension is too small.
static bool blas_operand(int64_t sr, int64_t sc, int R, int C, rocblas_operation& op, rocblas_int& ld) {
  if (sr == 1 && sc >= R && sc <= INT32_MAX) { op = rocblas_operation_none; ld = (rocblas_int)std::max<int64_t>(sc, 1); return true; }
  if (sc == 1 && sr >= C && sr <= INT32_MAX) { op = rocblas_operation_transpose; ld = (rocblas_int)std::max<int64_t>(sr, 1); return true; }
  if (R == 1 && sc == 1) { op = rocblas_operation_none; ld = 1; return true; }
  if (C == 1 && sr == 1) { op = rocblas_operation_none; ld = (rocblas_int)std::max(R, 1); return true; }
  return false;
}

// C[b] = alpha A[b] B[b] + beta C[b] for plain strided operands through rocBLAS
// (one strided-batched DGEMM); false when the layout has no such form or the
// call fails before anything is queued
static bool gemm_blas(hipStream_t s, int batch, const GemmArgs& g) {
  if (g.K <= 0) return false;
  rocblas_handle bh = blas_handle();
  if (!bh || rocblas_set_stream(bh, s) != rocblas_status_success) return false;
  rocblas_operation oa, ob;
  rocblas_int la, lb;
  rocblas_status st;
  if (g.sCj == 1 && g.sCi >= g.N && g.sCi <= INT32_MAX) {
    // row-major C: C^T (N x M) = B^T (N x K) A^T (K x M)
    if (!blas_operand(g.sBj, g.sBk, g.N, g.K, ob, lb) || !blas_operand(g.sAk, g.sAi, g.K, g.M, oa, la)) return false;
    st = rocblas_dgemm_strided_batched(bh, ob, oa, g.N, g.M, g.K, &g.alpha, g.B, lb, g.sBb, g.A, la, g.sAb, &g.beta,
                                       g.C, (rocblas_int)g.sCi, g.sCb, batch);
  } else if (g.sCi == 1 && g.sCj >= g.M && g.sCj <= INT32_MAX) {
    // column-major C: C (M x N) = A (M x K) B (K x N)
    if (!blas_operand(g.sAi, g.sAk, g.M, g.K, oa, la) || !blas_operand(g.sBk, g.sBj, g.K, g.N, ob, lb)) return false;
    st = rocblas_dgemm_strided_batched(bh, oa, ob, g.M, g.N, g.K, &g.alpha, g.A, la, g.sAb, g.B, lb, g.sBb, &g.beta,
                                       g.C, (rocblas_int)g.sCj, g.sCb, batch);
  } else {
    return false;
  }
  return st == rocblas_status_success;
}

hipError_t gemm(hipStream_t s, int batch, const GemmArgs& g) {
  if (g.M <= 0 || g.N <= 0 || batch <= 0) return hipSuccess;
  if (gemm_blas(s, batch, g)) return hipGetLastError();
  return gemm_native(s, batch, g);
}

// 1/q: the hardware reciprocal estimate refined by two Newton steps (relative
// error at the level of the FP64 rounding)
__device__ inline double rcp_refined(double q) {
  double r = __builtin_amdgcn_rcp(q);
  r = fma(fma(-q, r, 1.0), r, r);
  r = fma(fma(-q, r, 1.0), r, r);
  return r;
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
        // the two rows stay in registers (nv <= 192: three columns per lane)
        double xr[3], yr[3];
        double al = 0, be = 0, ga = 0;
#pragma unroll
        for (int u = 0; u < 3; ++u) {
          const int a = l + 64 * u;
          xr[u] = a < nv ? C[p * nv + a] : 0.0;
          yr[u] = a < nv ? C[q * nv + a] : 0.0;
          al += xr[u] * xr[u]; be += yr[u] * yr[u]; ga += xr[u] * yr[u];
        }
        al = wave_sum(al);
        be = wave_sum(be);
        ga = wave_sum(ga);
        if (ga * ga > 1e-30 * (al * be) && fabs(ga) > 1e-300) {
          // the angle only sets how well ga is annihilated (refined reciprocals
          // suffice); c = (1 + t^2)^(-1/2) to the rounding level keeps the
          // rotation orthogonal
          const double ze = (be - al) * (0.5 * rcp_refined(ga));
          const double t = (ze >= 0 ? 1.0 : -1.0) * rcp_refined(fabs(ze) + sqrt(1.0 + ze * ze));
          const double w = 1.0 + t * t;
          double c = __builtin_amdgcn_rsq(w);
          c = fma(0.5 * c, fma(-w * c, c, 1.0), c);
          c = fma(0.5 * c, fma(-w * c, c, 1.0), c);
          const double s = c * t;
#pragma unroll
          for (int u = 0; u < 3; ++u) {
            const int a = l + 64 * u;
            if (a < nv) {
              C[p * nv + a] = c * xr[u] - s * yr[u];
              C[q * nv + a] = s * xr[u] + c * yr[u];
            }
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
    s2 = wave_sum(s2);
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

}  // namespace esmp2

namespace esmp2 {

// ---------------------------------------------------------------------------
// Semicanonical AVOs, tridiagonal route.
//  1. k_complement_qr / k_complement_apply: Householder QR of the TOP virtuals
//     V (nv x no); Q2 = the last m = nv - no columns of H_0 ... H_{no-1}
//     (orthonormal complement), one wavefront per column.
//  2. F_avo = Q2^T F_vv Q2 (GEMMs).
//  3. k_tridiag: Householder tridiagonalisation of F_avo (packed in LDS),
//     T = P^T F_avo P, P = G_0 ... G_{m-3}.
//  4. k_tri_eig: eigenvalue k of T by wavefront multisection on Sturm counts,
//     eigenvector by a twisted factorisation of T - lambda.
//  5. k_cluster_mgs: Gram-Schmidt inside clusters of (nearly) equal eigenvalues.
//  6. k_backtransform: Y = P Yt, one column per workgroup.
//  AVO = Q2 Y, followed by a first-order Loewdin step (caller).
// ---------------------------------------------------------------------------

// Single workgroup (256 threads).  Vin: nv x no row-major.  Householder QR of
// Vin; reflector j (entries j..nv-1, zero above) into refl[j*nv + i], its
// coefficient into refl[no*nv + j].
__global__ __launch_bounds__(1024) void k_complement_qr(const double* Vin, int nv, int no, double* refl) {
  extern __shared__ double sm[];
  // nv x no working copy, column j reduced in place; rows padded to no + 1 so
  // that a wavefront walking one column spreads over the LDS banks
  const int ld = no + 1;
  double* W = sm;
  double* vv = W + nv * ld;          // reflectors: no x nv (row j = reflector j, entries j..nv-1)
  __shared__ double beta[64];
  __shared__ double red[16];
  const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63, nw = blockDim.x >> 6;
  for (int e = tid; e < nv * no; e += blockDim.x) W[(e / no) * ld + e % no] = Vin[e];
  __syncthreads();
  for (int j = 0; j < no; ++j) {
    double s = 0.0;
    for (int i = j + 1 + tid; i < nv; i += blockDim.x) s += W[i * ld + j] * W[i * ld + j];
    s = wave_sum(s);
    if (l == 0) red[wave] = s;
    __syncthreads();
    double sig = 0.0;
    for (int w = 0; w < nw; ++w) sig += red[w];
    double x0 = W[j * ld + j];
    double nrm = sqrt(x0 * x0 + sig);
    double alpha = (x0 >= 0) ? -nrm : nrm;
    double v0 = x0 - alpha;
    double vtv = v0 * v0 + sig;
    double b = (vtv > 0) ? 2.0 / vtv : 0.0;
    for (int i = tid; i < nv; i += blockDim.x) vv[j * nv + i] = (i < j) ? 0.0 : (i == j ? v0 : W[i * ld + j]);
    if (tid == 0) beta[j] = b;
    __syncthreads();
    // apply H_j = 1 - b v v^T to the remaining columns c > j (one wave per column)
    for (int c = j + 1 + wave; c < no; c += nw) {
      double t = 0.0;
      for (int i = l; i < nv; i += 64) if (i >= j) t += vv[j * nv + i] * W[i * ld + c];
      t = wave_sum(t) * b;
      for (int i = l; i < nv; i += 64) if (i >= j) W[i * ld + c] -= t * vv[j * nv + i];
    }
    __syncthreads();
  }
  for (int e = tid; e < no * nv; e += blockDim.x) refl[e] = vv[e];
  for (int j = tid; j < no; j += blockDim.x) refl[no * nv + j] = beta[j];
}

// Q2 (nv x m, m = nv - no) column c = H_0 H_1 ... H_{no-1} e_{no+c}: the
// orthonormal complement of the TOP virtuals.  One wavefront per column; lane
// l owns rows l, l + 64, l + 128 (nv <= 192).
// dst[i] = src[i*ld], i < n (a column of a row-major matrix)
__global__ void k_take_column(const double* src, int ld, int n, double* dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[(int64_t)i * ld];
}

__global__ __launch_bounds__(64) void k_complement_apply(const double* refl, int nv, int no, double* Q2) {
  const int c = blockIdx.x, l = threadIdx.x, m = nv - no;
  const double* beta = refl + no * nv;
  double q[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) q[k] = (l + 64 * k == no + c) ? 1.0 : 0.0;
  for (int j = no - 1; j >= 0; --j) {
    const double* v = refl + j * nv;
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int i = l + 64 * k;
      if (i < nv && i >= j) t += v[i] * q[k];
    }
    t = wave_sum(t) * beta[j];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int i = l + 64 * k;
      if (i < nv && i >= j) q[k] -= t * v[i];
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int i = l + 64 * k;
    if (i < nv) Q2[i * m + c] = q[k];
  }
}

__device__ inline int pk(int r, int c, int n) {   // packed upper index (r <= c)
  return r * n - r * (r - 1) / 2 + (c - r);
}

// Householder tridiagonalisation.  Ain: m x m row-major symmetric.  Single
// workgroup of 1024 threads, A packed (upper) in dynamic LDS.
// Outputs: refl (m x m, row k = reflector k on entries k+1..m-1), rbeta[m],
// d[m] (diagonal), e[m] (e[k] = T[k][k+1]).
// Step k needs two barriers: the scalars of the reflector (the norm of row k
// beyond the first subdiagonal) and K = b v.p / 2 are short reductions that
// every wavefront computes for itself; v is read straight from row k of A
// (untouched by step k's update), and w = p - K v is formed inside the
// rank-2 update.
__global__ __launch_bounds__(1024) void k_tridiag(const double* Ain, int m, double* refl, double* rbeta,
                                                  double* d, double* e) {
  extern __shared__ double A[];
  __shared__ double p[256];
  const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63, nw = blockDim.x >> 6;
  for (int r = 0; r < m; ++r)
    for (int c = r + tid; c < m; c += blockDim.x) A[pk(r, c, m)] = Ain[r * m + c];
  __syncthreads();
  for (int k = 0; k < m - 2; ++k) {
    // reflector scalars, in every wavefront (same reduction order everywhere)
    double s = 0.0;
    for (int i = k + 2 + l; i < m; i += 64) { const double x = A[pk(k, i, m)]; s += x * x; }
    const double sig = wave_sum(s);
    const double x0 = A[pk(k, k + 1, m)];
    double b = 0.0, alpha = x0, v0 = 0.0;
    if (sig > 0.0) {
      const double nrm = sqrt(x0 * x0 + sig);
      alpha = (x0 >= 0) ? -nrm : nrm;
      v0 = x0 - alpha;
      b = 2.0 / (v0 * v0 + sig);
    }
    // v_i = v0 (i = k+1), A[k][i] (i > k+1); zero when the row is already reduced.
    // Row r of the packed matrix starts at pk(r, r): A[r][c] = A[pk(r, r) - r + c].
    const int rk = pk(k, k, m) - k;
    auto vv = [&](int i) -> double { return b > 0.0 ? (i == k + 1 ? v0 : A[rk + i]) : 0.0; };
    for (int i = k + 1 + tid; i < m; i += blockDim.x) refl[k * m + i] = vv(i);
    if (tid == 0) { rbeta[k] = b; e[k] = alpha; }
    if (b > 0.0) {
      // p = b A22 v : 8 threads per row, thread `part` over j = k+1+part, k+9+part, ...
      // in increasing order: below the diagonal from column i of the rows above,
      // then along row i (no per-element test of which triangle holds A[i][j])
      const int len = m - k - 1;
      for (int t = tid; t < len * 8; t += blockDim.x) {
        const int i = k + 1 + t / 8, part = t % 8;
        double acc = 0.0;
        int j = k + 1 + part;
        for (; j < i; j += 8) acc += A[pk(j, j, m) - j + i] * vv(j);
        const int ri = pk(i, i, m) - i;
        for (; j < m; j += 8) acc += A[ri + j] * vv(j);
        // sum of the 8 lanes of the row (whole groups of 8 are active together)
        acc += dpp_move<0xb1, 0xf>(acc);     // quad_perm [1,0,3,2]
        acc += dpp_move<0x4e, 0xf>(acc);     // quad_perm [2,3,0,1]
        acc += dpp_move<0x141, 0xf>(acc);    // row_half_mirror: the other quad of the 8
        if (part == 0) p[i] = b * acc;
      }
      __syncthreads();
      double kk = 0.0;
      for (int i = k + 1 + l; i < m; i += 64) kk += vv(i) * p[i];
      const double K = 0.5 * b * wave_sum(kk);
      // A22 -= v w^T + w v^T (upper part), w = p - K v
      for (int i = k + 1 + wave; i < m; i += nw) {
        const double vi = vv(i), wi = p[i] - K * vi;
        const int ri = pk(i, i, m) - i;
        for (int j = i + l; j < m; j += 64) {
          const double vj = vv(j);
          A[ri + j] -= vi * (p[j] - K * vj) + wi * vj;
        }
      }
    }
    __syncthreads();
  }
  for (int i = tid; i < m; i += blockDim.x) d[i] = A[pk(i, i, m)];
  if (tid == 0 && m >= 2) e[m - 2] = A[pk(m - 2, m - 1, m)];
  if (tid == 0) e[m - 1] = 0.0;
  if (m == 1 && tid == 0) e[0] = 0.0;
}

// Largest tridiagonal order the eigensolver stages in LDS (callers keep m below it).
constexpr int TRI_MAX = 256;

// Number of eigenvalues of the tridiagonal (d, e) smaller than x; e2 = e^2.
// d and e2 live in LDS (all lanes read the same element: a broadcast).
// 1/q from the hardware reciprocal estimate and two Newton steps (relative
// error at the level of the FP64 rounding): the Sturm recurrence's one division
// per step is its critical path, and the IEEE division sequence is several times
// longer
__device__ inline double recip(double q) {
  double r = __builtin_amdgcn_rcp(q);
  r = fma(fma(-q, r, 1.0), r, r);
  r = fma(fma(-q, r, 1.0), r, r);
  return r;
}

__device__ inline int sturm_count(const double* d, const double* e2, int m, double x, double tiny) {
  int cnt = 0;
  double q = d[0] - x;
  if (q < 0) ++cnt;
  for (int i = 1; i < m; ++i) {
    if (fabs(q) < tiny) q = -tiny;
    q = d[i] - x - e2[i - 1] * recip(q);
    if (q < 0) ++cnt;
  }
  return cnt;
}

// One workgroup (64 threads) per eigenvalue k (ascending): evals[k], and the
// eigenvector into Z[k*m + i] (row k of Z).  m <= TRI_MAX.
__global__ __launch_bounds__(64) void k_tri_eig(const double* d, const double* e, int m, double* evals, double* Z) {
  const int k = blockIdx.x, l = threadIdx.x;
  __shared__ double ds[TRI_MAX], es[TRI_MAX], e2s[TRI_MAX];
  __shared__ double Dp[TRI_MAX], Dm[TRI_MAX], y[TRI_MAX];
  for (int i = l; i < m; i += 64) {
    ds[i] = d[i];
    es[i] = e[i];
    e2s[i] = e[i] * e[i];
  }
  __syncthreads();
  // Gershgorin interval
  double lo = 1e300, hi = -1e300;
  for (int i = l; i < m; i += 64) {
    const double r = (i > 0 ? fabs(es[i - 1]) : 0.0) + (i < m - 1 ? fabs(es[i]) : 0.0);
    lo = fmin(lo, ds[i] - r);
    hi = fmax(hi, ds[i] + r);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o));
    hi = fmax(hi, __shfl_xor(hi, o));
  }
  {
    const double span = fmax(hi - lo, 1e-300);
    lo -= 1e-3 * span;
    hi += 1e-3 * span;
  }
  const double tnorm = fmax(fabs(lo), fabs(hi));
  const double tiny = 1e-300 + 1e-30 * tnorm;
  // multisection: 64 Sturm counts per step shrink the bracket of eigenvalue k 65-fold
  for (int it = 0; it < 40; ++it) {
    const double x = lo + (hi - lo) * (double)(l + 1) / 65.0;
    const int c = sturm_count(ds, e2s, m, x, tiny);
    // first lane whose point has more than k eigenvalues below it
    const unsigned long long mask = __ballot(c > k);
    const int first = mask ? __ffsll((long long)mask) - 1 : 64;
    const double nlo = (first == 0) ? lo : lo + (hi - lo) * (double)first / 65.0;
    const double nhi = (first == 64) ? hi : lo + (hi - lo) * (double)(first + 1) / 65.0;
    lo = nlo;
    hi = nhi;
    if (hi - lo <= 4.0 * 2.220446049250313e-16 * fmax(fabs(lo), fabs(hi)) + 1e-300) break;
  }
  const double lam = 0.5 * (lo + hi);
  // twisted factorisation of T - lam: lane 0 runs the forward pivots D+, lane 1
  // the backward pivots D- (the same recurrence on the reversed arrays)
  if (l < 2) {
    const bool fw = (l == 0);
    double* D = fw ? Dp : Dm;
    int i0 = fw ? 0 : m - 1;
    double q = ds[i0] - lam;
    D[i0] = q;
    for (int s = 1; s < m; ++s) {
      const int i = fw ? s : m - 1 - s;
      const double ee = fw ? e2s[i - 1] : e2s[i];
      if (fabs(q) < tiny) q = (q < 0 ? -tiny : tiny);
      q = ds[i] - lam - ee / q;
      D[i] = q;
    }
  }
  __syncthreads();
  // twist index r: smallest |gamma_i| = |D+_i + D-_i - (d_i - lam)|
  double best = 1e300;
  int r = m;
  for (int i = l; i < m; i += 64) {
    const double g = fabs(Dp[i] + Dm[i] - (ds[i] - lam));
    if (g < best) { best = g; r = i; }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ob = __shfl_xor(best, o);
    const int orr = __shfl_xor(r, o);
    if (ob < best || (ob == best && orr < r)) { best = ob; r = orr; }
  }
  if (r >= m) r = 0;
  // eigenvector: 1 at r, lane 0 recurs downwards from r, lane 1 upwards
  if (l < 2) {
    const bool dn = (l == 0);
    if (dn) y[r] = 1.0;
    double v = 1.0;
    if (dn) {
      for (int i = r - 1; i >= 0; --i) {
        double q = Dp[i];
        if (fabs(q) < tiny) q = (q < 0 ? -tiny : tiny);
        v = -(es[i] / q) * v;
        y[i] = v;
      }
    } else {
      for (int i = r + 1; i < m; ++i) {
        double q = Dm[i];
        if (fabs(q) < tiny) q = (q < 0 ? -tiny : tiny);
        v = -(es[i - 1] / q) * v;
        y[i] = v;
      }
    }
  }
  __syncthreads();
  double nrm = 0.0;
  for (int i = l; i < m; i += 64) nrm += y[i] * y[i];
  nrm = wave_sum(nrm);
  const double inv = 1.0 / sqrt(nrm);
  if (l == 0) evals[k] = lam;
  for (int i = l; i < m; i += 64) Z[(size_t)k * m + i] = y[i] * inv;
}

// Gram-Schmidt of eigenvectors inside clusters (relative gap below 1e-6).
// Single workgroup of 64 threads; cheap when there are no clusters.
__global__ __launch_bounds__(64) void k_cluster_mgs(const double* evals, int m, double* Z) {
  const int l = threadIdx.x;
  double tn = 0.0;
  for (int k = 0; k < m; ++k) tn = fmax(tn, fabs(evals[k]));
  int start = 0;
  for (int k = 1; k < m; ++k) {
    if (evals[k] - evals[k - 1] > 1e-6 * tn) { start = k; continue; }
    double* zk = Z + (size_t)k * m;
    for (int pass = 0; pass < 2; ++pass)
      for (int j = start; j < k; ++j) {
        const double* zj = Z + (size_t)j * m;
        double t = 0.0;
        for (int i = l; i < m; i += 64) t += zj[i] * zk[i];
        t = wave_sum(t);
        for (int i = l; i < m; i += 64) zk[i] -= t * zj[i];
        __syncthreads();
      }
    double s = 0.0;
    for (int i = l; i < m; i += 64) s += zk[i] * zk[i];
    s = wave_sum(s);
    double inv = 1.0 / sqrt(s);
    for (int i = l; i < m; i += 64) zk[i] *= inv;
    __syncthreads();
  }
}

// Y[:, k] = G_0 ... G_{m-3} Z[k, :]; one workgroup (64 threads) per column.
// Each lane keeps its entries of the column (i = l + 64 s) in registers; the
// reflector coefficients sit in LDS and the entries of the next BT_AHEAD
// reflectors are in flight while it applies the current one (one reflector's
// arithmetic is far shorter than a load's latency).
constexpr int BT_AHEAD = 3;

__global__ __launch_bounds__(64) void k_backtransform(const double* refl, const double* rbeta, int m,
                                                      const double* Z, double* Y) {
  constexpr int S = TRI_MAX / 64;
  const int k = blockIdx.x, l = threadIdx.x;
  __shared__ double sb[TRI_MAX];
  for (int j = l; j < m; j += 64) sb[j] = j <= m - 3 ? rbeta[j] : 0.0;
  double y[S], buf[BT_AHEAD + 1][S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int i = l + 64 * s;
    y[s] = (i < m) ? Z[(size_t)k * m + i] : 0.0;
  }
  // reflector j (entries i > j) into buf slot (j0 - j) % (BT_AHEAD + 1)
  auto load = [&](int j, double* dst) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int i = l + 64 * s;
      dst[s] = (j >= 0 && i < m && i > j) ? refl[(size_t)j * m + i] : 0.0;
    }
  };
  const int j0 = m - 3;
#pragma unroll
  for (int a = 0; a < BT_AHEAD; ++a) load(j0 - a, buf[a]);
  __syncthreads();
  for (int j = j0; j >= 0; j -= BT_AHEAD + 1) {
    // BT_AHEAD + 1 reflectors per pass so that the slots have fixed names
#pragma unroll
    for (int a = 0; a <= BT_AHEAD; ++a) {
      const int jj = j - a;
      if (jj < 0) break;
      load(jj - BT_AHEAD, buf[(a + BT_AHEAD) % (BT_AHEAD + 1)]);
      const double b = sb[jj];
      if (b != 0.0) {
        const double* cur = buf[a];
        double t = 0.0;
#pragma unroll
        for (int s = 0; s < S; ++s) t += cur[s] * y[s];
        t = wave_sum(t) * b;
#pragma unroll
        for (int s = 0; s < S; ++s) y[s] -= t * cur[s];
      }
    }
  }
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int i = l + 64 * s;
    if (i < m) Y[(size_t)i * m + k] = y[s];
  }
}

// Sign of column x[0], x[ld], ..., x[(len-1) ld] that makes its first entry of
// largest magnitude positive (+1 for a zero column), for the 64 lanes of a
// wavefront: lane-local first maxima, then the larger magnitude and on a tie
// the smaller index, which is the first maximum of the whole column.
__device__ inline double col_sign(const double* x, int len, int ld, int l) {
  double best = 0.0, val = 0.0;
  int idx = 1 << 30;
  for (int i = l; i < len; i += 64) {
    const double y = x[(int64_t)i * ld];
    if (fabs(y) > best) { best = fabs(y); val = y; idx = i; }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double b2 = __shfl_xor(best, o), v2 = __shfl_xor(val, o);
    const int i2 = __shfl_xor(idx, o);
    if (b2 > best || (b2 == best && i2 < idx)) { best = b2; val = v2; idx = i2; }
  }
  return val < 0 ? -1.0 : 1.0;
}

// R[:no,:no] = U,  R[no:, no:2no] = V,  R[no:, 2no + c] = AVO[:, c] (signed:
// largest-|entry| positive);  avo_eps[c] = eigenvalue c.  One wavefront per
// column of R.
__global__ __launch_bounds__(64) void k_assemble_r2(const double* U, const double* V, const double* AVO,
                                                    const double* evals, int no, int nv, double* R, double* avo_eps) {
  const int n = no + nv, m = nv - no, col = blockIdx.x, l = threadIdx.x;
  if (col < no) {
    for (int r = l; r < n; r += 64) R[r * n + col] = r < no ? U[r * no + col] : 0.0;
  } else if (col < 2 * no) {
    for (int r = l; r < n; r += 64) R[r * n + col] = r >= no ? V[(r - no) * no + (col - no)] : 0.0;
  } else {
    const int c = col - 2 * no;
    const double sg = col_sign(AVO + c, nv, m, l);
    for (int r = l; r < n; r += 64) R[r * n + col] = r >= no ? sg * AVO[(r - no) * m + c] : 0.0;
    if (l == 0) avo_eps[c] = evals[c];
  }
}

}  // namespace esmp2
