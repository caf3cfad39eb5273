// sigma = (H0 - E0) x on doubles + L-triples (paper Sec. II.C, modified Q F Q).
//
// The Fock operator acts on every index slot of every amplitude.  Per box:
//   * virtual pair (the dominant N_o^2 N_v^3 work; the paper's hand-coded
//     "mixed-spin L-triples x Fock" term is its largest part): a batched
//     Sylvester product Y = F' X + X F' on matrix cores, F' = F_vv + c/2 with
//     the box's diagonal constant c (-omega on doubles, f_t't' - f_tt - omega on
//     L-triples), boxes with t' excluded embedded with a zero row/column;
//   * occupied pair, box transfers (a pinned TOP index moved by one Fock
//     element), doubles <-> L-triples couplings through f_ov: a per-element
//     gather (plus per-batch side contractions over one virtual index).
// S2 enters flip-symmetrised (S~ = (x + flip x)/2).
#include "common.h"
#include "mfma.h"
#include "sigma.h"

namespace esmp2 {

// ---------------------------------------------------------------------------
// amplitude lookups with antisymmetry (zero where the Pauli principle forbids)
// ---------------------------------------------------------------------------
template <class T>
struct Look {
  // Branch-free: the load is always issued (at the box's first element when
  // the Pauli principle forbids the amplitude) and the exact zero or the sign
  // of the reordering applied by a select, so that a caller's lookups issue
  // back to back and their latencies overlap.
  Dims d;
  const T* x;
  const T* S;      // flip-symmetrised S2, dense [i][j][a][b]
  __device__ T T2(int i, int j, int a, int b) const {
    const bool z = (i == j) | (a == b);
    const T s = ((i > j) != (a > b)) ? T(-1) : T(1);
    const int64_t k = z ? 0 : (int64_t)tri_idx(min(i, j), max(i, j), d.no) * d.npv + tri_idx(min(a, b), max(a, b), d.nv);
    const T v = x[d.off[B_T2] + k];
    return z ? T(0) : s * v;
  }
  __device__ T T3(int j, int k, int b, int c) const {      // all indices >= 1
    const bool z = (j == k) | (b == c);
    const T s = ((j > k) != (b > c)) ? T(-1) : T(1);
    const int64_t o = z ? 0
                        : (int64_t)tri_idx(min(j, k) - 1, max(j, k) - 1, d.no - 1) * d.npv1 +
                              tri_idx(min(b, c) - 1, max(b, c) - 1, d.nv - 1);
    const T v = x[d.off[B_T3] + o];
    return z ? T(0) : s * v;
  }
  __device__ T H11(int j, int k, int b, int c) const {
    const bool z = (j == k) | (b == c);
    const T s = ((j > k) != (b > c)) ? T(-1) : T(1);
    const int64_t o = z ? 0 : (int64_t)tri_idx(min(j, k), max(j, k), d.no) * d.npv + tri_idx(min(b, c), max(b, c), d.nv);
    const T v = x[d.off[B_H11] + o];
    return z ? T(0) : s * v;
  }
  __device__ T H12(int j, int k, int a, int c) const {     // a, c >= 1
    const bool z = j == k;
    const T s = j > k ? T(-1) : T(1);
    const int m1 = d.nv - 1;
    const int64_t o = z ? 0 : ((int64_t)tri_idx(min(j, k), max(j, k), d.no) * m1 + (a - 1)) * m1 + (c - 1);
    const T v = x[d.off[B_H12] + o];
    return z ? T(0) : s * v;
  }
  __device__ T H21(int i, int k, int b, int c) const {     // i, k >= 1
    const bool z = b == c;
    const T s = b > c ? T(-1) : T(1);
    const int64_t o = z ? 0 : ((int64_t)(i - 1) * (d.no - 1) + (k - 1)) * d.npv + tri_idx(min(b, c), max(b, c), d.nv);
    const T v = x[d.off[B_H21] + o];
    return z ? T(0) : s * v;
  }
  __device__ T H22(int i, int k, int a, int c) const {     // all >= 1
    int m1 = d.nv - 1;
    return x[d.off[B_H22] + (((int64_t)(i - 1) * (d.no - 1) + (k - 1)) * m1 + (a - 1)) * m1 + (c - 1)];
  }
  __device__ T St(int i, int j, int a, int b) const {
    return S[(((int64_t)i * d.no + j) * d.nv + a) * d.nv + b];
  }
};

// ---------------------------------------------------------------------------
// S~ = (x_S2 + sg flip x_S2)/2, flip: (i,j,a,b) -> (j,i,b,a); sg = +1 singlet, -1 triplet
// ---------------------------------------------------------------------------
template <class T>
__device__ __attribute__((always_inline)) inline void sym_s2_body(Dims d, const T* x, T* S, int bid_, int nb_) {
  // one 32 x 32 block of (a, b) of one batch (i, j); the partner block (j, i)
  // is read in its own (row-major) order and transposed through LDS
  __shared__ T tl[32][33];
  const int nv = d.nv, nt = (nv + 31) / 32;
  const int blk = (int)xcd_remap<16>(bid_, nb_);
  const int o = blk / (nt * nt), t = blk - o * (nt * nt);
  const int i = o / d.no, j = o - i * d.no;
  const int a0 = (t / nt) * 32, b0 = (t % nt) * 32;
  const int64_t nv2 = (int64_t)nv * nv;
  const T* s2 = x + d.off[B_S2];
  const T* P = s2 + ((int64_t)j * d.no + i) * nv2;
  const T* X = s2 + ((int64_t)i * d.no + j) * nv2;
  T* Sd = S + ((int64_t)i * d.no + j) * nv2;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
  for (int r = ty; r < 32; r += 8) {
    const int b = b0 + r, a = a0 + tx;
    tl[r][tx] = (b < nv && a < nv) ? P[b * nv + a] : T(0);
  }
  __syncthreads();
  const T sg = T(d.sg);
#pragma unroll
  for (int r = ty; r < 32; r += 8) {
    const int a = a0 + r, b = b0 + tx;
    if (a < nv && b < nv) Sd[a * nv + b] = T(0.5) * (X[a * nv + b] + sg * tl[tx][r]);
  }
}

template <class T>
__global__ __launch_bounds__(256) void k_sym_s2(Dims d, const T* x, T* S) {
  sym_s2_body<T>(d, x, S, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// Batched Sylvester product on matrix cores.  One job = one batch matrix of one
// box, embedded in an mv x mv matrix (mv = nv padded to 16).  Output block of
// (32 TW) x (32 TW) per workgroup, 4 wavefronts of TW x TW 16x16 tiles.
// K loop: k < mv uses A = F', B = X; k >= mv uses A = X, B = F'.
// ---------------------------------------------------------------------------
enum Fmt { F_PACK = 0, F_PACK_RED = 1, F_DENSE_RED = 2, F_DENSE = 3 };

template <class T>
struct JobView {
  int fmt, m;            // storage format and its matrix dimension
  const T* src;          // this batch's storage
  T* dst;
  T* tr;               // transfer row (row 0 of the embedded product) or null
};

template <class T>
__device__ inline JobView<T> job_view(const VVArgs<T>& A, int box, int batch) {
  const Dims& d = A.d;
  JobView<T> v;
  v.tr = nullptr;
  int64_t o = d.off[box];
  switch (box) {
    case B_T2: case B_H11: case B_H21:
      v.fmt = F_PACK; v.m = d.nv; o += (int64_t)batch * d.npv; break;
    case B_T3:
      v.fmt = F_PACK_RED; v.m = d.nv - 1; o += (int64_t)batch * d.npv1; break;
    case B_H12: case B_H22:
      v.fmt = F_DENSE_RED; v.m = d.nv - 1; o += (int64_t)batch * (d.nv - 1) * (d.nv - 1);
      v.tr = A.side_tr + ((box == B_H12 ? 0 : d.npo) + (int64_t)batch) * d.nv;
      break;
    default:
      v.fmt = F_DENSE; v.m = d.nv; break;
  }
  if (box == B_S2) {
    v.src = A.S + (int64_t)batch * d.nv * d.nv;
    v.dst = A.y + d.off[B_S2] + (int64_t)batch * d.nv * d.nv;
  } else {
    v.src = A.x + o;
    v.dst = A.y + o;
  }
  return v;
}

// element (r, c) of the embedded batch matrix
template <class T>
__device__ inline T xget(const JobView<T>& v, int r, int c) {
  switch (v.fmt) {
    case F_PACK: {
      if (r >= v.m || c >= v.m || r == c) return 0.0;
      return r < c ? v.src[tri_idx(r, c, v.m)] : -v.src[tri_idx(c, r, v.m)];
    }
    case F_PACK_RED: {
      if (r == 0 || c == 0 || r > v.m || c > v.m || r == c) return 0.0;
      return r < c ? v.src[tri_idx(r - 1, c - 1, v.m)] : -v.src[tri_idx(c - 1, r - 1, v.m)];
    }
    case F_DENSE_RED: {
      if (r == 0 || c == 0 || r > v.m || c > v.m) return 0.0;
      return v.src[(r - 1) * v.m + (c - 1)];
    }
    default:
      if (r >= v.m || c >= v.m) return 0.0;
      return v.src[r * v.m + c];
  }
}

template <class T>
__device__ inline void yput(const JobView<T>& v, int r, int c, T val) {
  switch (v.fmt) {
    case F_PACK:
      if (r < c && c < v.m) v.dst[tri_idx(r, c, v.m)] = val;
      break;
    case F_PACK_RED:
      if (r >= 1 && r < c && c <= v.m) v.dst[tri_idx(r - 1, c - 1, v.m)] = val;
      break;
    case F_DENSE_RED:
      if (c >= 1 && c <= v.m && r <= v.m) {
        if (r >= 1) v.dst[(r - 1) * v.m + (c - 1)] = val;
        else v.tr[c] = val;
      }
      break;
    default:
      if (r < v.m && c < v.m) v.dst[r * v.m + c] = val;
  }
}

template <class T, int TW>
__global__ __launch_bounds__(256) void k_vv(VVArgs<T> A) {
  constexpr int BR = 32 * TW;
  __shared__ T As[16][BR + 1];
  __shared__ T Bs[16][BR + 1];
  const int2 jb = A.jobs[blockIdx.x];
  const int box = jb.x;
  const JobView<T> v = job_view(A, box, jb.y);
  const T* F = (box == B_T2 || box == B_S2) ? A.Fd : A.Fl;
  const int mv = A.d.mv;
  const int R0 = blockIdx.y * BR, C0 = blockIdx.z * BR;
  const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63;
  const int wr = (wave >> 1) * TW * 16, wc = (wave & 1) * TW * 16;
  typedef typename MfmaAcc<T>::type AccT;
  AccT acc[TW][TW];
#pragma unroll
  for (int i = 0; i < TW; ++i)
#pragma unroll
    for (int j = 0; j < TW; ++j) acc[i][j] = AccT{0, 0, 0, 0};
  for (int k0 = 0; k0 < 2 * mv; k0 += 16) {
    const bool second = k0 >= mv;
    const int kb = second ? k0 - mv : k0;
    for (int e = tid; e < BR * 16; e += 256) {
      int r = e >> 4, kk = e & 15;
      int gr = R0 + r, gk = kb + kk;
      T val = 0;
      if (gr < mv) val = second ? xget(v, gr, gk) : F[gr * mv + gk];
      As[kk][r] = val;
    }
    for (int e = tid; e < BR * 16; e += 256) {
      int c = e % BR, kk = e / BR;
      int gc = C0 + c, gk = kb + kk;
      T val = 0;
      if (gc < mv) val = second ? F[gk * mv + gc] : xget(v, gk, gc);
      Bs[kk][c] = val;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      T a[TW], b[TW];
#pragma unroll
      for (int t = 0; t < TW; ++t) {
        a[t] = As[ks * 4 + (l >> 4)][wr + t * 16 + (l & 15)];
        b[t] = Bs[ks * 4 + (l >> 4)][wc + t * 16 + (l & 15)];
      }
#pragma unroll
      for (int i = 0; i < TW; ++i)
#pragma unroll
        for (int j = 0; j < TW; ++j) acc[i][j] = mfma16x16x4(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int ti = 0; ti < TW; ++ti)
#pragma unroll
    for (int tj = 0; tj < TW; ++tj)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int r = R0 + wr + ti * 16 + mfma_row_t<T>(l, i);
        int c = C0 + wc + tj * 16 + (l & 15);
        yput(v, r, c, acc[ti][tj][i]);
      }
}


// ---------------------------------------------------------------------------
// Side contractions over one virtual index, per batch of an L box:
//   row   v[c] = sum_x w[x] X[x][c],   column  u[a] = sum_x X[a][x] w[x],
// with w a column of f_ov (index 0 = t, or the batch's occupied indices).
// Output layout: side[slot][batch][nv] for each (box, slot), see sigma.h.
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(256) void k_side(SideArgs<T> A) {
  const Dims& d = A.d;
  const int no = d.no, nv = d.nv;
  const int job = blockIdx.x;
  Look<T> L{d, A.x, nullptr};
  const T* fov = A.fov;                 // fov[i*nv + a]
  int box, batch;
  if (job < d.npo1) { box = B_T3; batch = job; }
  else if (job < d.npo1 + d.npo) { box = B_H11; batch = job - d.npo1; }
  else if (job < d.npo1 + 2 * d.npo) { box = B_H12; batch = job - d.npo1 - d.npo; }
  else if (job < d.npo1 + 2 * d.npo + (no - 1) * (no - 1)) { box = B_H21; batch = job - d.npo1 - 2 * d.npo; }
  else { box = B_H22; batch = job - d.npo1 - 2 * d.npo - (no - 1) * (no - 1); }
  // lane -> output column c (64 per workgroup along y), wavefront -> a quarter
  // of the contracted range; partial sums meet in LDS
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = blockIdx.y * 64 + lane;
  const bool col = c < nv;
  const int b0 = (box == B_H11 || box == B_H21) ? 0 : 1;
  const int lo = b0 + (nv - b0) * wave / 4, hi = b0 + (nv - b0) * (wave + 1) / 4;
  T r0 = 0, r1 = 0, r2 = 0;
  int p = 0, q = 0;
  if (box == B_T3) {
    tri_pq(batch, no - 1, p, q); ++p; ++q;
    if (col && c >= 1)
      for (int x = lo; x < hi; ++x) {
        const T xv = L.T3(p, q, x, c);
        r0 += fov[x] * xv; r1 += fov[p * nv + x] * xv; r2 += fov[q * nv + x] * xv;
      }
  } else if (box == B_H11) {
    tri_pq(batch, no, p, q);
    if (col)
      for (int x = lo; x < hi; ++x) {
        const T xv = L.H11(p, q, x, c);
        r0 += fov[p * nv + x] * xv; r1 += fov[q * nv + x] * xv;
      }
  } else if (box == B_H12) {
    tri_pq(batch, no, p, q);
    if (col && c >= 1)
      for (int x = lo; x < hi; ++x) {
        r0 += fov[x] * L.H12(p, q, x, c);             // sum_a f_{a t} X[a][c]
        const T xr = L.H12(p, q, c, x);                // row c (= a), column x
        r1 += xr * fov[p * nv + x]; r2 += xr * fov[q * nv + x];
      }
  } else if (box == B_H21) {
    p = batch / (no - 1) + 1; q = batch % (no - 1) + 1;
    if (col)
      for (int x = lo; x < hi; ++x) {
        const T xv = L.H21(p, q, x, c);
        r0 += fov[x] * xv; r1 += fov[q * nv + x] * xv;
      }
  } else {
    p = batch / (no - 1) + 1; q = batch % (no - 1) + 1;
    if (col && c >= 1)
      for (int x = lo; x < hi; ++x) {
        const T xr = L.H22(p, q, c, x);                // row c (= a), column x
        r0 += xr * fov[x]; r2 += xr * fov[q * nv + x];
        r1 += fov[p * nv + x] * L.H22(p, q, x, c);     // sum_a f_{a i} X[a][c]
      }
  }
  __shared__ T part[3][4][64];
  part[0][wave][lane] = r0; part[1][wave][lane] = r1; part[2][wave][lane] = r2;
  __syncthreads();
  if (wave != 0 || !col) return;
  T s[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) s[k] = part[k][0][lane] + part[k][1][lane] + part[k][2][lane] + part[k][3][lane];
  const int64_t o = (int64_t)batch * nv + c;
  switch (box) {
    case B_T3: A.t3_t[o] = s[0]; A.t3_p1[o] = s[1]; A.t3_p2[o] = s[2]; break;
    case B_H11: A.h11_p1[o] = s[0]; A.h11_p2[o] = s[1]; break;
    case B_H12: A.h12_t[o] = s[0]; A.h12_u1[o] = s[1]; A.h12_u2[o] = s[2]; break;
    case B_H21: A.h21_t[o] = s[0]; A.h21_k[o] = s[1]; break;
    default: A.h22_ut[o] = s[0]; A.h22_i[o] = s[1]; A.h22_uk[o] = s[2]; break;
  }
}

// ---------------------------------------------------------------------------
// Per-element couplings other than the two Fock contractions over the free
// index pairs: box transfers through a pinned TOP index (f_{t' a}, f_{m t}),
// doubles <-> L-triples through f_ov (with the side contractions of k_side),
// y += ... (the virtual-pair part is already in y, k_oo adds the occupied
// pair part).  One workgroup per chunk of 256 inner indices of one batch
// matrix, one thread per amplitude; virtual pairs decoded from tables.
// ---------------------------------------------------------------------------
// box of amplitude g and its index within the box (a box holds < 2^31 amplitudes)
__device__ inline int box_of_g(const Dims& d, int64_t g, int& loc) {
  int k = 0;
  while (k < 6 && g >= d.off[k + 1]) ++k;
  loc = (int)(g - d.off[k]);
  return k;
}

// Coupling terms of amplitude (box, batch, v) (occupied indices p0, q0 of the
// batch): box transfers through a pinned TOP index and doubles <-> L-triples
// through f_ov.
template <class T>
__device__ __attribute__((always_inline)) inline T couple_terms(const GatherArgs<T>& A, const PairTables& P, int box,
                                                                int batch, int p0, int q0, int v) {
  const Dims& d = A.d;
  const int no = d.no, nv = d.nv, m1 = nv - 1;
  Look<T> L{d, A.x, A.S};
  const T* fo = A.fo;     // fo[m*no + i]
  const T* fv = A.fv;     // fv[a*nv + b]
  const T* fov = A.fov;   // fov[i*nv + a]
  auto FOV = [&](int i, int a) { return fov[i * nv + a]; };
  const T ftt = FOV(0, 0);
  T y = 0;
  switch (box) {
    case B_T2: {
      const int i = p0, j = q0, t = P.pv[v], a = t >> 16, b = t & 0xffff;
      // from the L-triples: the same-spin T3L directly, the mixed-spin boxes
      // through their spin-flip partners (amplitude sg x)
      T ys = 0;
      if (i >= 1 && a >= 1) y += ftt * L.T3(i, j, a, b);
      ys += ftt * L.H11(i, j, a, b);
      if (i == 0) {
        if (a >= 1) {
#pragma unroll 4
          for (int m = 1; m < no; ++m) y -= FOV(m, 0) * L.T3(m, j, a, b);
        }
#pragma unroll 4
        for (int m = 1; m < no; ++m) ys += FOV(m, 0) * L.H21(m, j, a, b);
      }
      if (a == 0) {
        if (i >= 1) y -= A.t3_t[tri_idx(i - 1, j - 1, no - 1) * nv + b];
        ys += A.h12_t[batch * nv + b];
        if (i == 0) {
#pragma unroll 4
          for (int m = 1; m < no; ++m) {
            const bool lt = m < j;
            const int pi = (m == j) ? 0 : tri_idx(min(m, j) - 1, max(m, j) - 1, no - 1);
            const T tv = (lt ? A.t3_p1 : A.t3_p2)[pi * nv + b];
            y += lt ? tv : (m > j ? -tv : T(0));
            ys += A.h22_i[((m - 1) * (no - 1) + (j - 1)) * nv + b];
          }
        }
      }
      y += T(d.sg) * ys;
      break;
    }
    case B_S2: {
      const int i = p0, j = q0, a = v / nv, b = v - a * nv;
      // d(p,q,x,z) + sg d(q,p,z,x): de-excitation of the mixed-spin L-triples and their flip partners
      for (int rep = 0; rep < 2; ++rep) {
        const int p = rep ? j : i, q = rep ? i : j, xx = rep ? b : a, z = rep ? a : b;
        T dd = 0;
        if (p == 0) {
          if (xx == 0) {
#pragma unroll 4
            for (int m = 0; m < no; ++m) {
              const bool lt = m < q;
              const int pi = (m == q) ? 0 : tri_idx(min(m, q), max(m, q), no);
              const T tv = (lt ? A.h11_p1 : A.h11_p2)[pi * nv + z];
              dd += lt ? tv : (m > q ? -tv : T(0));
            }
          } else if (z >= 1) {
#pragma unroll 4
            for (int m = 0; m < no; ++m) dd += FOV(m, 0) * L.H12(m, q, xx, z);
          } else {
#pragma unroll 4
            for (int m = 0; m < no; ++m) {
              const bool lt = m < q;
              const int pi = (m == q) ? 0 : tri_idx(min(m, q), max(m, q), no);
              const T tv = (lt ? A.h12_u1 : A.h12_u2)[pi * nv + xx];
              dd += lt ? -tv : (m > q ? tv : T(0));
            }
          }
        } else if (q >= 1) {
          if (xx == 0) dd += A.h21_t[((p - 1) * (no - 1) + (q - 1)) * nv + z];
          else if (z >= 1) dd += ftt * L.H22(p, q, xx, z);
          else dd -= A.h22_ut[((p - 1) * (no - 1) + (q - 1)) * nv + xx];
        } else {
          if (xx == 0) {
#pragma unroll 4
            for (int m = 1; m < no; ++m) dd -= A.h21_k[((p - 1) * (no - 1) + (m - 1)) * nv + z];
          } else if (z >= 1) {
#pragma unroll 4
            for (int m = 1; m < no; ++m) dd -= FOV(m, 0) * L.H22(p, m, xx, z);
          } else {
#pragma unroll 4
            for (int m = 1; m < no; ++m) dd += A.h22_uk[((p - 1) * (no - 1) + (m - 1)) * nv + xx];
          }
        }
        y += (rep ? T(d.sg) : T(1)) * dd;
      }
      break;
    }
    case B_T3: {
      const int j = p0, k = q0, t = P.pv1[v], b = (t >> 16) + 1, c = (t & 0xffff) + 1;
      y += ftt * L.T2(j, k, b, c) - FOV(j, 0) * L.T2(0, k, b, c) + FOV(k, 0) * L.T2(0, j, b, c)
         - FOV(0, b) * L.T2(j, k, 0, c) + FOV(j, b) * L.T2(0, k, 0, c) - FOV(k, b) * L.T2(0, j, 0, c)
         + FOV(0, c) * L.T2(j, k, 0, b) - FOV(j, c) * L.T2(0, k, 0, b) + FOV(k, c) * L.T2(0, j, 0, b);
      break;
    }
    case B_H11: {
      const int j = p0, k = q0, t = P.pv[v], b = t >> 16, c = t & 0xffff;
      if (j == 0) {
#pragma unroll 4
        for (int m = 1; m < no; ++m) y -= fo[m * no + 0] * L.H21(m, k, b, c);
      }
      y += T(d.sg) * ftt * L.T2(j, k, b, c);                 // flip partner of T2 (down-down)
      y += FOV(j, b) * L.St(0, k, 0, c) - FOV(k, b) * L.St(0, j, 0, c)
         - FOV(j, c) * L.St(0, k, 0, b) + FOV(k, c) * L.St(0, j, 0, b);
      break;
    }
    case B_H12: {
      const int j = p0, k = q0, a = v / m1 + 1, c = v - (a - 1) * m1 + 1;
      y += fv[a * nv + 0] * L.H11(j, k, 0, c);
      if (j == 0) {
#pragma unroll 4
        for (int m = 1; m < no; ++m) y -= fo[m * no + 0] * L.H22(m, k, a, c);
      }
      y += T(d.sg) * FOV(0, a) * L.T2(j, k, 0, c);
      y += FOV(j, 0) * L.St(0, k, a, c) - FOV(k, 0) * L.St(0, j, a, c)
         - FOV(j, c) * L.St(0, k, a, 0) + FOV(k, c) * L.St(0, j, a, 0);
      break;
    }
    case B_H21: {
      const int i = p0, k = q0, t = P.pv[v], b = t >> 16, c = t & 0xffff;
      y -= fo[0 * no + i] * L.H11(0, k, b, c);
      y += T(d.sg) * FOV(i, 0) * L.T2(0, k, b, c);
      y += FOV(0, b) * L.St(i, k, 0, c) - FOV(k, b) * L.St(i, 0, 0, c)
         - FOV(0, c) * L.St(i, k, 0, b) + FOV(k, c) * L.St(i, 0, 0, b);
      break;
    }
    default: {
      const int i = p0, k = q0, a = v / m1 + 1, c = v - (a - 1) * m1 + 1;
      y -= fo[0 * no + i] * L.H12(0, k, a, c);
      y += fv[a * nv + 0] * L.H21(i, k, 0, c);
      y += T(d.sg) * FOV(i, a) * L.T2(0, k, 0, c);
      y += ftt * L.St(i, k, a, c) - FOV(k, 0) * L.St(i, 0, a, c)
         - FOV(0, c) * L.St(i, k, a, 0) + FOV(k, c) * L.St(i, 0, a, 0);
      break;
    }
  }
  return y;
}

template <class T>
__global__ __launch_bounds__(256) void k_couple(GatherArgs<T> A, PairTables P, const int4* chunks) {
  const Dims& d = A.d;
  // chunk: (box, batch, first inner index or S2 tile, (p << 16) | q occupied indices of the batch)
  const int4 ch = chunks[xcd_remap<32>(blockIdx.x, gridDim.x)];
  const int box = ch.x, batch = ch.y;
  const int p0 = ch.w >> 16, q0 = ch.w & 0xffff;
  const int nv = d.nv, m1 = nv - 1;
  int inner;
  switch (box) {
    case B_T2: case B_H11: case B_H21: inner = d.npv; break;
    case B_S2: inner = nv * nv; break;
    case B_T3: inner = d.npv1; break;
    default: inner = m1 * m1; break;
  }
  const int v = chunk_inner(box, ch.z, (int)threadIdx.x, nv, inner);
  if (v >= inner) return;
  T* yp = A.y + d.off[box] + (int64_t)batch * inner + v;
  const T y0 = *yp;                  // issued ahead of the lookups: its latency overlaps theirs
  const T y = couple_terms(A, P, box, batch, p0, q0, v);
  *yp = y0 + y;
}

}  // namespace esmp2

namespace esmp2 {

// ---------------------------------------------------------------------------
// Occupied-index Fock action on matrix cores, y += -(F_o X_v + X_v F_o) for
// every inner index v of every box (F_o restricted to the box's occupied
// range), plus the two box-transfer rows that the Sylvester kernel produces
// (H1P2 -> H1P1 and H2P2 -> H2P1 through f_{t' E}).  One workgroup: one box,
// GO consecutive inner indices, all occupied batches staged in LDS.
// ---------------------------------------------------------------------------

constexpr int OO_THREADS = 256, OO_R = 8;

template <class T>
__global__ __launch_bounds__(OO_THREADS) void k_oo(GatherArgs<T> A, int4 tiles0, int4 tiles1) {
  extern __shared__ __align__(16) unsigned char sm_raw[];
  T* sm = reinterpret_cast<T*>(sm_raw);
  const Dims& d = A.d;
  const int no = d.no, nv = d.nv;
  const int tstart[8] = {0, tiles0.x, tiles0.y, tiles0.z, tiles0.w, tiles1.x, tiles1.y, tiles1.z};
  const int blk = (int)xcd_remap<16>(blockIdx.x, gridDim.x);
  int box = 0;
  while (box < 6 && blk >= tstart[box + 1]) ++box;
  const int t0 = (blk - tstart[box]) * GO;
  int nbat, inner, n, sh;
  bool anti;
  switch (box) {
    case B_T2: case B_H11: nbat = d.npo; inner = d.npv; n = no; sh = 0; anti = true; break;
    case B_S2: nbat = no * no; inner = nv * nv; n = no; sh = 0; anti = false; break;
    case B_T3: nbat = d.npo1; inner = d.npv1; n = no - 1; sh = 1; anti = true; break;
    case B_H12: nbat = d.npo; inner = (nv - 1) * (nv - 1); n = no; sh = 0; anti = true; break;
    case B_H21: nbat = (no - 1) * (no - 1); inner = d.npv; n = no - 1; sh = 1; anti = false; break;
    default: nbat = (no - 1) * (no - 1); inner = (nv - 1) * (nv - 1); n = no - 1; sh = 1; anti = false; break;
  }
  T* tin = sm;                                      // nbat x (GO+1)
  T* tout = tin + nbat * (GO + 1);                  // nbat x (GO+1)
  int* xi = (int*)(tout + nbat * (GO + 1));         // 16 x 16
  const T* src = (box == B_S2) ? A.S : A.x + d.off[box];
  const int tw = min(GO, inner - t0);
  const int tid = threadIdx.x;
  const int ne = nbat * GO;
  T* y = A.y + d.off[box];
  // y of the first output round, issued with the staging so that its latency
  // overlaps the staging and the matrix-core products (no other kernel writes
  // y meanwhile; the workgroups own disjoint parts of it)
  T vy0[OO_R];
#pragma unroll
  for (int u = 0; u < OO_R; ++u) {
    const int e = u * OO_THREADS + tid;
    const int o = e / GO, vl = e % GO;
    vy0[u] = (e < ne && vl < tw) ? y[(int64_t)o * inner + t0 + vl] : T(0);
  }
  // staging: OO_R elements per thread per round, all loads of a round issued
  // before the first LDS store, so their latencies overlap
  for (int e0 = 0; e0 < ne; e0 += OO_R * OO_THREADS) {
    T vin[OO_R], vtr[OO_R];
#pragma unroll
    for (int u = 0; u < OO_R; ++u) {
      const int e = e0 + u * OO_THREADS + tid;
      const int o = e / GO, vl = e % GO;
      const bool ok = e < ne && vl < tw;
      vin[u] = ok ? src[(int64_t)o * inner + t0 + vl] : T(0);
      // box-transfer rows (inner pairs (t', c) are the first nv-1 packed pairs)
      const bool trow = ok && (box == B_H11 || box == B_H21) && t0 + vl < nv - 1;
      vtr[u] = trow ? A.side_tr[((box == B_H11 ? 0 : (int64_t)d.npo) + o) * nv + (t0 + vl + 1)] : T(0);
    }
#pragma unroll
    for (int u = 0; u < OO_R; ++u) {
      const int e = e0 + u * OO_THREADS + tid;
      if (e < ne) {
        const int o = e / GO, vl = e % GO;
        tin[o * (GO + 1) + vl] = vin[u];
        tout[o * (GO + 1) + vl] = vtr[u];
      }
    }
  }
  {
    int p = tid >> 4, q = tid & 15, code = 0;
    if (p < n && q < n) {
      if (!anti) code = p * n + q + 1;
      else if (p < q) code = tri_idx(p, q, n) + 1;
      else if (p > q) code = -(tri_idx(q, p, n) + 1);
    }
    xi[tid] = code;
  }
  __syncthreads();
  const int wave = tid >> 6, l = tid & 63;
  const int r16 = l & 15, k4 = l >> 4;
  const T* fo = A.fo;
  auto Fs = [&](int p, int q) -> T { return (p < n && q < n) ? fo[(p + sh) * no + (q + sh)] : T(0); };
  T fa[4], fb[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    fa[s] = Fs(r16, 4 * s + k4);
    fb[s] = Fs(4 * s + k4, r16);
  }
  for (int vl = wave; vl < tw; vl += 4) {
    auto X = [&](int p, int q) -> T {
      int code = xi[p * 16 + q];
      if (code == 0) return T(0);
      T val = tin[((code > 0 ? code : -code) - 1) * (GO + 1) + vl];
      return code > 0 ? val : -val;
    };
    typename MfmaAcc<T>::type acc = {0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      acc = mfma16x16x4(fa[s], X(4 * s + k4, r16), acc);
      acc = mfma16x16x4(X(r16, 4 * s + k4), fb[s], acc);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = mfma_row_t<T>(l, q), c = r16;
      if (r < n && c < n && (!anti || r < c)) {
        const int bidx = anti ? tri_idx(r, c, n) : r * n + c;
        tout[bidx * (GO + 1) + vl] -= acc[q];
      }
    }
  }
  __syncthreads();
  for (int e0 = 0; e0 < ne; e0 += OO_R * OO_THREADS) {
    T vy[OO_R];
#pragma unroll
    for (int u = 0; u < OO_R; ++u) {
      const int e = e0 + u * OO_THREADS + tid;
      const int o = e / GO, vl = e % GO;
      vy[u] = e0 == 0 ? vy0[u] : (e < ne && vl < tw) ? y[(int64_t)o * inner + t0 + vl] : T(0);
    }
#pragma unroll
    for (int u = 0; u < OO_R; ++u) {
      const int e = e0 + u * OO_THREADS + tid;
      const int o = e / GO, vl = e % GO;
      if (e < ne && vl < tw) y[(int64_t)o * inner + t0 + vl] = vy[u] + tout[o * (GO + 1) + vl];
    }
  }
}


// Occupied-index Fock action and the two transfer rows, one thread per
// amplitude: the fallback of k_oo when an occupied range exceeds one 16 x 16
// matrix-core tile or the staged batches exceed the LDS.
template <class T>
__global__ __launch_bounds__(256) void k_oo_plain(GatherArgs<T> A) {
  const Dims& d = A.d;
  int64_t g = (int64_t)xcd_remap<16>(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (g >= d.off[7]) return;
  const int no = d.no, nv = d.nv;
  Look<T> L{d, A.x, A.S};
  const T* fo = A.fo;
  int loc;
  const int box = box_of_g(d, g, loc);
  T y = 0;
  switch (box) {
    case B_T2: {
      int i, j, a, b;
      tri_pq(loc / d.npv, no, i, j); tri_pq(loc % d.npv, nv, a, b);
      for (int m = 0; m < no; ++m) y -= fo[m * no + i] * L.T2(m, j, a, b) + fo[m * no + j] * L.T2(i, m, a, b);
      break;
    }
    case B_S2: {
      int r = loc;
      int b = r % nv; r /= nv;
      int a = r % nv; r /= nv;
      int j = r % no, i = r / no;
      for (int m = 0; m < no; ++m) y -= fo[m * no + i] * L.St(m, j, a, b) + fo[m * no + j] * L.St(i, m, a, b);
      break;
    }
    case B_T3: {
      int j, k, b, c;
      tri_pq(loc / d.npv1, no - 1, j, k); tri_pq(loc % d.npv1, nv - 1, b, c);
      ++j; ++k; ++b; ++c;
      for (int m = 1; m < no; ++m) y -= fo[m * no + j] * L.T3(m, k, b, c) + fo[m * no + k] * L.T3(j, m, b, c);
      break;
    }
    case B_H11: {
      int j, k, b, c;
      tri_pq(loc / d.npv, no, j, k); tri_pq(loc % d.npv, nv, b, c);
      for (int m = 0; m < no; ++m) y -= fo[m * no + j] * L.H11(m, k, b, c) + fo[m * no + k] * L.H11(j, m, b, c);
      if (b == 0) y += A.side_tr[(int64_t)tri_idx(j, k, no) * nv + c];
      break;
    }
    case B_H12: {
      const int m1 = nv - 1;
      int j, k;
      tri_pq(loc / (m1 * m1), no, j, k);
      const int a = (loc % (m1 * m1)) / m1 + 1, c = loc % m1 + 1;
      for (int m = 0; m < no; ++m) y -= fo[m * no + j] * L.H12(m, k, a, c) + fo[m * no + k] * L.H12(j, m, a, c);
      break;
    }
    case B_H21: {
      const int o = loc / d.npv;
      const int i = o / (no - 1) + 1, k = o % (no - 1) + 1;
      int b, c;
      tri_pq(loc % d.npv, nv, b, c);
      for (int m = 1; m < no; ++m) y -= fo[m * no + i] * L.H21(m, k, b, c) + fo[m * no + k] * L.H21(i, m, b, c);
      if (b == 0) y += A.side_tr[((int64_t)d.npo + o) * nv + c];
      break;
    }
    default: {
      const int m1 = nv - 1;
      const int o = loc / (m1 * m1);
      const int i = o / (no - 1) + 1, k = o % (no - 1) + 1;
      const int a = (loc % (m1 * m1)) / m1 + 1, c = loc % m1 + 1;
      for (int m = 1; m < no; ++m) y -= fo[m * no + i] * L.H22(m, k, a, c) + fo[m * no + k] * L.H22(i, m, a, c);
      break;
    }
  }
  A.y[g] += y;
}

#define ESMP2_SIGMA_INSTANCES(T)                                                        \
  template __global__ void k_sym_s2<T>(Dims, const T*, T*);                             \
  template __global__ void k_vv<T, 1>(VVArgs<T>);                                       \
  template __global__ void k_vv<T, 2>(VVArgs<T>);                                       \
  template __global__ void k_vv<T, 3>(VVArgs<T>);                                       \
  template __global__ void k_vv<T, 4>(VVArgs<T>);                                       \
  template __global__ void k_vv<T, 5>(VVArgs<T>);                                       \
  template __global__ void k_side<T>(SideArgs<T>);                                      \
  template __global__ void k_couple<T>(GatherArgs<T>, PairTables, const int4*);          \
  template __global__ void k_oo<T>(GatherArgs<T>, int4, int4);                          \
  template __global__ void k_oo_plain<T>(GatherArgs<T>);
ESMP2_SIGMA_INSTANCES(double)
ESMP2_SIGMA_INSTANCES(float)
#undef ESMP2_SIGMA_INSTANCES

}  // namespace esmp2
