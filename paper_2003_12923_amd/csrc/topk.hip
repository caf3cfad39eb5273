// ESMP2-TOP(k): k transition-orbital pairs treated as large (paper Sec. II.C:
// the L-triples are those containing a large TOP; k = n_occ is TOP(all), the
// N^6 limit of Sec. III.B, Table II).
//
// Layout: the doubles (T2, S2) of the one-TOP layout, then for every large
// TOP s = 0 .. k-1 the five L-boxes of the one-TOP layout written for TOP s
// in place of TOP 0 (occupied orbitals 0 and s swapped, virtuals 0' and s'
// swapped).  A triple that contains a larger TOP r < s belongs to set r; its
// slot in set s is masked (held at zero).  Amplitudes keep the one-TOP
// layout's meaning (operator-string phase, spin-flip partner sg x, S2
// flip-symmetrised); s0[g] is the canonical phase of element g's operator
// string (spin-orbitals alpha then beta, each ascending), so that s0[g] x[g]
// is the coefficient of the element's own determinant.
//
// The operator is applied on determinants, one thread per element: for the
// element's own determinant D0, (F - E0) Psi at D0 is the diagonal plus every
// single spin-orbital replacement D' of D0 inside D + L, with matrix element
// f_uv (-1)^(n(u) + n(v) - [u < v]) (u removed, v added, n(.) = occupied
// spin-orbitals of D0 below).  The replacements are: a hole refilled from
// another occupied orbital, a particle moved to another virtual, a triple's
// particle de-excited into one of its holes, and a double excited into a
// triple that contains a large TOP (candidates restricted by the TOPs the
// double already holds; each triple counted once, under the largest TOP it
// contains).  The position of D' is closed-form arithmetic on its indices.
// Work per element is O(N_o + N_v): the path is for correctness at the sizes
// of the tests, not tuned like the one-TOP kernels.
#include "common.h"
#include "sigma.h"
#include "reduce.h"

namespace esmp2 {

struct TopkArgs {
  Dims d;               // one-TOP dimensions and box offsets
  int k;                // large TOPs
  int64_t L1;           // amplitudes of one set of L-boxes: off[7] - off[2]
  int64_t namp;         // off[2] + k L1
  const double* Ft;     // TOP-basis Fock matrix (N x N)
  double omega, sg;
  const signed char* s0;
};

__device__ inline int relab(int x, int s) { return x == 0 ? s : (x == s ? 0 : x); }

// own determinant of element g: spin-orbitals (spin N + spatial, virtuals at
// spatial n_occ + a), nh = 2 or 3 holes / particles; set, box; false if masked
__device__ inline bool topk_decode(const TopkArgs& A, int64_t g, int* h, int* p, int& nh, int& set, int& box) {
  const Dims& d = A.d;
  const int no = d.no, nv = d.nv, N = d.n, m1 = nv - 1;
  int64_t g1 = g;
  set = 0;
  if (g >= d.off[2]) {
    set = (int)((g - d.off[2]) / A.L1);
    g1 = d.off[2] + (g - d.off[2]) % A.L1;
  }
  int k = 0;
  while (k < 6 && g1 >= d.off[k + 1]) ++k;
  box = k;
  const int loc = (int)(g1 - d.off[k]);
  const int s = set;
  auto O = [&](int spin, int i) { return spin * N + relab(i, s); };
  auto V = [&](int spin, int a) { return spin * N + no + relab(a, s); };
  switch (box) {
    case B_T2: {
      int i, j, a, b;
      tri_pq(loc / d.npv, no, i, j); tri_pq(loc % d.npv, nv, a, b);
      h[0] = i; h[1] = j; p[0] = no + a; p[1] = no + b; nh = 2;
      return true;
    }
    case B_S2: {
      int r = loc;
      const int b = r % nv; r /= nv;
      const int a = r % nv; r /= nv;
      const int j = r % no, i = r / no;
      h[0] = i; h[1] = N + j; p[0] = no + a; p[1] = N + no + b; nh = 2;
      return true;
    }
    case B_T3: {
      int j, c, b, kk;
      tri_pq(loc / d.npv1, no - 1, j, kk); tri_pq(loc % d.npv1, nv - 1, b, c);
      h[0] = O(0, 0); h[1] = O(0, j + 1); h[2] = O(0, kk + 1);
      p[0] = V(0, 0); p[1] = V(0, b + 1); p[2] = V(0, c + 1);
      break;
    }
    case B_H11: {
      int j, kk, b, c;
      tri_pq(loc / d.npv, no, j, kk); tri_pq(loc % d.npv, nv, b, c);
      h[0] = O(0, 0); h[1] = O(1, j); h[2] = O(1, kk);
      p[0] = V(0, 0); p[1] = V(1, b); p[2] = V(1, c);
      break;
    }
    case B_H12: {
      int j, kk;
      tri_pq(loc / (m1 * m1), no, j, kk);
      const int a = (loc % (m1 * m1)) / m1 + 1, c = loc % m1 + 1;
      h[0] = O(0, 0); h[1] = O(1, j); h[2] = O(1, kk);
      p[0] = V(0, a); p[1] = V(1, 0); p[2] = V(1, c);
      break;
    }
    case B_H21: {
      const int o = loc / d.npv;
      const int i = o / (no - 1) + 1, kk = o % (no - 1) + 1;
      int b, c;
      tri_pq(loc % d.npv, nv, b, c);
      h[0] = O(0, i); h[1] = O(1, 0); h[2] = O(1, kk);
      p[0] = V(0, 0); p[1] = V(1, b); p[2] = V(1, c);
      break;
    }
    default: {
      const int o = loc / (m1 * m1);
      const int i = o / (no - 1) + 1, kk = o % (no - 1) + 1;
      const int a = (loc % (m1 * m1)) / m1 + 1, c = loc % m1 + 1;
      h[0] = O(0, i); h[1] = O(1, 0); h[2] = O(1, kk);
      p[0] = V(0, a); p[1] = V(1, 0); p[2] = V(1, c);
      break;
    }
  }
  nh = 3;
  // masked: the triple holds a larger TOP r < s (it belongs to set r)
  for (int r = 0; r < s; ++r) {
    bool hr = false, pr = false;
    for (int q = 0; q < 3; ++q) { hr |= (h[q] % N) == r; pr |= (p[q] % N) == no + r; }
    if (hr && pr) return false;
  }
  return true;
}

// element holding determinant (h, p) (nh holes / particles, any order): its
// index and whether (h, p) is that element's own determinant (else its
// spin-flip partner); -1 if the determinant is not in D + L
__device__ inline int64_t topk_pos(const TopkArgs& A, const int* h, const int* p, int nh, bool& own) {
  const Dims& d = A.d;
  const int no = d.no, nv = d.nv, N = d.n;
  int nup = 0;
  for (int q = 0; q < nh; ++q) nup += h[q] < N;
  if (nh == 2) {
    if (nup != 1) {                   // same spin: T2, own if alpha
      own = nup == 2;
      int i = h[0] % N, j = h[1] % N, a = p[0] % N - no, b = p[1] % N - no;
      if (i > j) { const int t = i; i = j; j = t; }
      if (a > b) { const int t = a; a = b; b = t; }
      return d.off[B_T2] + (int64_t)tri_idx(i, j, no) * d.npv + tri_idx(a, b, nv);
    }
    own = true;                        // S2: alpha hole i, beta hole j, alpha particle a, beta particle b
    const int i = h[0] < N ? h[0] : h[1], j = (h[0] < N ? h[1] : h[0]) - N;
    const int a = (p[0] < N ? p[0] : p[1]) - no, b = (p[0] < N ? p[1] : p[0]) - N - no;
    return d.off[B_S2] + (((int64_t)i * no + j) * nv + a) * nv + b;
  }
  // triples: the largest TOP contained (smallest index) owns it
  int s = -1;
  for (int r = 0; r < A.k && s < 0; ++r) {
    bool hr = false, pr = false;
    for (int q = 0; q < 3; ++q) { hr |= (h[q] % N) == r; pr |= (p[q] % N) == no + r; }
    if (hr && pr) s = r;
  }
  if (s < 0) return -1;
  // orientation: the own determinant has three alpha holes (same spin) or one
  // (mixed spin); otherwise the determinant is the flip partner
  own = (nup == 3 || nup == 1);
  const bool same = (nup == 3 || nup == 0);
  const int upspin = own ? 0 : 1;     // spin that plays "alpha" in the own orientation
  const int64_t base = d.off[2] + (int64_t)s * A.L1 - d.off[2];
  if (same) {
    int x[3], y[3];
    for (int q = 0; q < 3; ++q) { x[q] = relab(h[q] % N, s); y[q] = relab(p[q] % N - no, s); }
    // sort ascending (x[0] = 0 and y[0] = 0 after the relabelling: TOP s is held)
    for (int i = 1; i < 3; ++i)
      for (int j = i; j > 0 && x[j - 1] > x[j]; --j) { const int t = x[j]; x[j] = x[j - 1]; x[j - 1] = t; }
    for (int i = 1; i < 3; ++i)
      for (int j = i; j > 0 && y[j - 1] > y[j]; --j) { const int t = y[j]; y[j] = y[j - 1]; y[j - 1] = t; }
    return base + d.off[B_T3] + (int64_t)tri_idx(x[1] - 1, x[2] - 1, no - 1) * d.npv1 +
           tri_idx(y[1] - 1, y[2] - 1, nv - 1);
  }
  int i = -1, j = -1, kk = -1, a = -1, b = -1, c = -1;
  for (int q = 0; q < 3; ++q) {
    const int sp = h[q] / N, x = relab(h[q] % N, s);
    if (sp == upspin) i = x;
    else if (j < 0) j = x;
    else kk = x;
    const int spp = p[q] / N, y = relab(p[q] % N - no, s);
    if (spp == upspin) a = y;
    else if (b < 0) b = y;
    else c = y;
  }
  if (j > kk) { const int t = j; j = kk; kk = t; }
  if (b > c) { const int t = b; b = c; c = t; }
  const int m1 = nv - 1;
  if (i == 0 && a == 0) return base + d.off[B_H11] + (int64_t)tri_idx(j, kk, no) * d.npv + tri_idx(b, c, nv);
  if (i == 0) return base + d.off[B_H12] + ((int64_t)tri_idx(j, kk, no) * m1 + (a - 1)) * m1 + (c - 1);
  if (a == 0) return base + d.off[B_H21] + ((int64_t)(i - 1) * (no - 1) + (kk - 1)) * d.npv + tri_idx(b, c, nv);
  return base + d.off[B_H22] + (((int64_t)(i - 1) * (no - 1) + (kk - 1)) * m1 + (a - 1)) * m1 + (c - 1);
}

// occupied spin-orbitals of determinant (h, p) below spin-orbital v
__device__ inline int nbelow(int v, const int* h, const int* p, int nh, int no, int N) {
  int c = v < N ? min(v, no) : no + min(v - N, no);
  for (int q = 0; q < nh; ++q) c += (p[q] < v) - (h[q] < v);
  return c;
}

// amplitude of element e's own determinant in the operator-string convention
// (S2 flip-symmetrised)
template <class T>
__device__ inline double own_amp(const TopkArgs& A, const T* x, int64_t e) {
  const Dims& d = A.d;
  if (e >= d.off[B_S2] && e < d.off[B_S2 + 1]) {
    int r = (int)(e - d.off[B_S2]);
    const int nv = d.nv, no = d.no;
    const int b = r % nv; r /= nv;
    const int a = r % nv; r /= nv;
    const int j = r % no, i = r / no;
    const int64_t pe = d.off[B_S2] + (((int64_t)j * no + i) * nv + b) * nv + a;
    return 0.5 * ((double)x[e] + A.sg * (double)x[pe]);
  }
  return (double)x[e];
}

// coefficient of determinant (h, p) in Psi (0 outside D + L)
template <class T>
__device__ inline double det_coeff(const TopkArgs& A, const T* x, const int* h, const int* p, int nh) {
  bool own = true;
  const int64_t e = topk_pos(A, h, p, nh, own);
  if (e < 0) return 0.0;
  return (own ? 1.0 : A.sg) * (double)A.s0[e] * own_amp(A, x, e);
}

__device__ inline bool holds(const int* v, int n, int x) {
  bool r = false;
  for (int q = 0; q < n; ++q) r |= v[q] == x;
  return r;
}

// y = (H0 - E0) x on D + L of TOP(k), one thread per element; T: the storage of x and y
// (FP64, or FP32 for the inner solves of the mixed-precision refinement), arithmetic in FP64
template <class T>
__global__ __launch_bounds__(256) void k_topk_sigma(TopkArgs A, const T* x, T* y) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= A.namp) return;
  const Dims& d = A.d;
  const int no = d.no, nv = d.nv, N = d.n;
  int h[3], p[3], nh, set, box;
  if (!topk_decode(A, g, h, p, nh, set, box)) { y[g] = T(0); return; }
  const double* F = A.Ft;
  double diag = -A.omega;
  for (int q = 0; q < nh; ++q) diag += F[(p[q] % N) * (N + 1)] - F[(h[q] % N) * (N + 1)];
  double acc = diag * (double)A.s0[g] * own_amp(A, x, g);
  auto term = [&](const int* h2, const int* p2, int nh2, int u, int v) {
    const double c = det_coeff(A, x, h2, p2, nh2);
    if (c != 0.0) {
      const int e = nbelow(v, h, p, nh, no, N) - (u < v) + nbelow(u, h, p, nh, no, N);
      acc += F[(u % N) * N + (v % N)] * ((e & 1) ? -c : c);
    }
  };
  int h2[3], p2[3];
  for (int j = 0; j < nh; ++j) {
    // hole j refilled, occupied m (same spin, not a hole) emptied
    const int sp = h[j] / N;
    for (int m = 0; m < no; ++m) {
      const int mm = sp * N + m;
      if (holds(h, nh, mm)) continue;
      for (int q = 0; q < nh; ++q) { h2[q] = h[q]; p2[q] = p[q]; }
      h2[j] = mm;
      term(h2, p2, nh, mm, h[j]);
    }
    // particle j moved to virtual e (same spin, not a particle)
    const int spp = p[j] / N;
    for (int a = 0; a < nv; ++a) {
      const int ee = spp * N + no + a;
      if (holds(p, nh, ee)) continue;
      for (int q = 0; q < nh; ++q) { h2[q] = h[q]; p2[q] = p[q]; }
      p2[j] = ee;
      term(h2, p2, nh, p[j], ee);
    }
  }
  if (nh == 3) {
    // a particle de-excited into a hole of the same spin: a double
    for (int j = 0; j < 3; ++j)
      for (int i = 0; i < 3; ++i) {
        if (p[j] / N != h[i] / N) continue;
        int n2 = 0;
        for (int q = 0; q < 3; ++q)
          if (q != i) h2[n2++] = h[q];
        n2 = 0;
        for (int q = 0; q < 3; ++q)
          if (q != j) p2[n2++] = p[q];
        term(h2, p2, 2, p[j], h[i]);
      }
  } else {
    // a double excited into a triple holding a large TOP s: an occupied q (not a
    // hole) emptied, a virtual v (not a particle) filled, same spin; the
    // candidates are restricted by what the double already holds of TOP s, and a
    // triple holding a larger TOP r < s is left to r
    for (int s = 0; s < A.k; ++s) {
      bool hs = false, ps = false;
      for (int q = 0; q < 2; ++q) { hs |= (h[q] % N) == s; ps |= (p[q] % N) == no + s; }
      const int m0 = hs ? 0 : s, m1 = hs ? no : s + 1;
      const int a0 = ps ? 0 : s, a1 = ps ? nv : s + 1;
      for (int sp = 0; sp < 2; ++sp)
        for (int m = m0; m < m1; ++m) {
          const int qq = sp * N + m;
          if (holds(h, 2, qq)) continue;
          for (int a = a0; a < a1; ++a) {
            const int vv = sp * N + no + a;
            if (holds(p, 2, vv)) continue;
            h2[0] = h[0]; h2[1] = h[1]; h2[2] = qq;
            p2[0] = p[0]; p2[1] = p[1]; p2[2] = vv;
            bool larger = false;
            for (int r = 0; r < s; ++r) {
              bool hr = false, pr = false;
              for (int q = 0; q < 3; ++q) { hr |= (h2[q] % N) == r; pr |= (p2[q] % N) == no + r; }
              larger |= hr && pr;
            }
            if (larger) continue;
            term(h2, p2, 3, qq, vv);
          }
        }
    }
  }
  y[g] = T((double)A.s0[g] * acc);
}

template __global__ void k_topk_sigma<double>(TopkArgs, const double*, double*);
template __global__ void k_topk_sigma<float>(TopkArgs, const float*, float*);

// s0[g]: canonical phase of element g's operator string (the one-TOP layout's
// string with the set's relabelling); 0 for a masked slot
__global__ __launch_bounds__(256) void k_topk_phase(TopkArgs A, signed char* s0) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= A.namp) return;
  const Dims& d = A.d;
  int h[3], p[3], nh, set, box;
  if (!topk_decode(A, g, h, p, nh, set, box)) { s0[g] = 0; return; }
  const int64_t g1 = g < d.off[2] ? g : d.off[2] + (g - d.off[2]) % A.L1;
  const int loc = (int)(g1 - d.off[box]);
  Op ops[6];
  int64_t partner = g1;
  const int n = amp_ops(d, g1, box, loc, ops, &partner);
  for (int q = 0; q < n; ++q) {
    const int o = ops[q].orb;
    ops[q].orb = o < d.no ? relab(o, set) : d.no + relab(o - d.no, set);
  }
  int hh[3], pp[3], a, b;
  s0[g] = (signed char)apply_ops(ops, n, d.no, d.n, false, hh, a, pp, b);
}

// Jacobi diagonal of TOP(k) (FP32 preconditioner 1/D, 0 on masked slots) and
// per-workgroup minima of D over the live slots
__global__ __launch_bounds__(256) void k_topk_diag(TopkArgs A, float* dinv, double* blockmin) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double mn = 1e300;
  if (g < A.namp) {
    int h[3], p[3], nh, set, box;
    const int N = A.d.n;
    if (topk_decode(A, g, h, p, nh, set, box)) {
      double D = -A.omega;
      for (int q = 0; q < nh; ++q) D += A.Ft[(p[q] % N) * (N + 1)] - A.Ft[(h[q] % N) * (N + 1)];
      dinv[g] = (float)(1.0 / D);
      mn = D;
    } else {
      dinv[g] = 0.f;
    }
  }
  for (int o = 32; o > 0; o >>= 1) mn = fmin(mn, __shfl_xor(mn, o));
  __shared__ double ws[4];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = mn;
  __syncthreads();
  if (threadIdx.x == 0) blockmin[blockIdx.x] = fmin(fmin(ws[0], ws[1]), fmin(ws[2], ws[3]));
}

// b of set `set` from the one-TOP right-hand side of the relabelled problem
// (bs, one-TOP layout): set 0 takes every element, a set s >= 1 its L-boxes;
// masked slots are zero
__global__ __launch_bounds__(256) void k_topk_bset(TopkArgs A, int set, const double* bs, double* b) {
  const Dims& d = A.d;
  const int64_t first = set == 0 ? 0 : d.off[2] + (int64_t)set * A.L1;
  const int64_t cnt = set == 0 ? d.off[7] : A.L1;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cnt) return;
  const int64_t g = first + e;
  b[g] = A.s0[g] != 0 ? bs[set == 0 ? e : d.off[2] + e] : 0.0;
}

// partials of sum over the live L-triples of sets s >= 1 of 2 b^2 / D: the
// TOP(1) S-triples that TOP(k) moves into L
__global__ __launch_bounds__(256) void k_topk_e2s(TopkArgs A, const double* b, double* partial) {
  const Dims& d = A.d;
  const int N = d.n;
  double acc = 0.0;
  const int64_t first = d.off[2] + A.L1;
  for (int64_t g = first + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < A.namp;
       g += (int64_t)gridDim.x * blockDim.x) {
    int h[3], p[3], nh, set, box;
    if (!topk_decode(A, g, h, p, nh, set, box)) continue;
    double D = -A.omega;
    for (int q = 0; q < nh; ++q) D += A.Ft[(p[q] % N) * (N + 1)] - A.Ft[(h[q] % N) * (N + 1)];
    acc += 2.0 * b[g] * b[g] / D;
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// the one-TOP right-hand side's inputs with TOP s renamed to TOP 0 (orbitals 0
// and s swapped in both spaces)
__global__ void k_topk_permute(int s, int no, int nv, int naux, const double* Ft, const double* Bov,
                               const double* Bvt, const double* Boo, const double* lam, double* Ft_s, double* Bov_s,
                               double* Bvt_s, double* Boo_s, double* lam_s) {
  const int n = no + nv;
  const int64_t tot = (int64_t)n * n + (int64_t)naux * no * nv * 2 + (int64_t)naux * no * no + no;
  auto po = [&](int i) { return relab(i, s); };
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = e;
    if (r < (int64_t)n * n) {
      const int pq = (int)(r / n), q = (int)(r % n);
      const int P = pq < no ? po(pq) : no + po(pq - no), Qo = q < no ? po(q) : no + po(q - no);
      Ft_s[r] = Ft[(int64_t)P * n + Qo];
      continue;
    }
    r -= (int64_t)n * n;
    if (r < (int64_t)naux * no * nv) {
      const int Q = (int)(r / (no * nv)), i = (int)(r % (no * nv)) / nv, a = (int)(r % nv);
      Bov_s[r] = Bov[((int64_t)Q * no + po(i)) * nv + po(a)];
      continue;
    }
    r -= (int64_t)naux * no * nv;
    if (r < (int64_t)naux * nv * no) {
      const int Q = (int)(r / (nv * no)), a = (int)(r % (nv * no)) / no, l = (int)(r % no);
      Bvt_s[r] = Bvt[((int64_t)Q * nv + po(a)) * no + po(l)];
      continue;
    }
    r -= (int64_t)naux * nv * no;
    if (r < (int64_t)naux * no * no) {
      const int Q = (int)(r / (no * no)), i = (int)(r % (no * no)) / no, j = (int)(r % no);
      Boo_s[r] = Boo[((int64_t)Q * no + po(i)) * no + po(j)];
      continue;
    }
    r -= (int64_t)naux * no * no;
    lam_s[r] = lam[po((int)r)];
  }
}

// determinant export of TOP(k) amplitudes: own determinant of every live
// element at g, the spin-flip partner of every live element outside S2 at
// namp + (index among the elements outside S2); masked slots: key -1, 0
__global__ __launch_bounds__(256) void k_topk_export(TopkArgs A, const double* x, double* coeff, int64_t* key) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= A.namp) return;
  const Dims& d = A.d;
  const int N = d.n;
  const int64_t ns2 = d.off[B_S2 + 1] - d.off[B_S2];
  const bool s2 = g >= d.off[B_S2] && g < d.off[B_S2 + 1];
  const int64_t f = A.namp + (g < d.off[B_S2] ? g : g - ns2);
  int h[3], p[3], nh, set, box;
  if (!topk_decode(A, g, h, p, nh, set, box)) {
    key[g] = -1; coeff[g] = 0.0;
    if (!s2) { key[f] = -1; coeff[f] = 0.0; }
    return;
  }
  auto mk = [&](const int* hh, const int* pp) {
    int x[3] = {1023, 1023, 1023}, y[3] = {1023, 1023, 1023};
    for (int q = 0; q < nh; ++q) { x[q] = hh[q]; y[q] = pp[q]; }
    for (int i = 1; i < 3; ++i)
      for (int j = i; j > 0 && x[j - 1] > x[j]; --j) { const int t = x[j]; x[j] = x[j - 1]; x[j - 1] = t; }
    for (int i = 1; i < 3; ++i)
      for (int j = i; j > 0 && y[j - 1] > y[j]; --j) { const int t = y[j]; y[j] = y[j - 1]; y[j - 1] = t; }
    int64_t k = 0;
    for (int q = 0; q < 3; ++q) { k |= (int64_t)x[q] << (10 * q); k |= (int64_t)y[q] << (30 + 10 * q); }
    return k;
  };
  const double c = (double)A.s0[g] * own_amp(A, x, g);
  key[g] = mk(h, p);
  coeff[g] = c;
  if (s2) return;
  int hf[3], pf[3];
  for (int q = 0; q < nh; ++q) { hf[q] = h[q] < N ? h[q] + N : h[q] - N; pf[q] = p[q] < N ? p[q] + N : p[q] - N; }
  key[f] = mk(hf, pf);
  coeff[f] = A.sg * c;
}

}  // namespace esmp2
