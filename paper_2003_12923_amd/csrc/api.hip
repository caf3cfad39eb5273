// C ABI of libesmp2 (see include/esmp2.h).  Host orchestration: validation,
// buffer ownership, and the stream-ordered sequence of kernel launches.
#include "common.h"
#include "sigma.h"
#include "pcg.h"
#include <math.h>
#include <string.h>
#include <vector>
#include <new>
#include <algorithm>
#include <type_traits>
#include <atomic>
#include <thread>
#include <map>
#include <mutex>
#include <set>
#include <tuple>

// Kernels come from the other sources of the same translation unit (esmp2_all.hip).

using namespace esmp2;

static constexpr int E2S_CAP = 3 * 1024;   // E2_S partial sums: three grids of at most 1024 workgroups

// ---------------------------------------------------------------------------
// small helper kernels local to the orchestration
// ---------------------------------------------------------------------------
__global__ void k_finite(const double* v, int64_t n, int* bad) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(v[g])) bad[0] = 1;
}

__global__ void k_add_to(double* dst, const double* src) {
  if (threadIdx.x == 0) dst[0] += src[0];
}

__global__ void k_sub_identity(double* E, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) E[(int64_t)i * n + i] -= 1.0;
}

// TOP-basis Fock blocks, orbital energies, omega / kappa / E0 and the shifted,
// padded virtual blocks used by the Sylvester kernel.
//   sc[0] = omega = sum_l lam_l^2 (f_l'l' - f_ll), sc[1] = kappa = f_t't' - f_tt - omega,
//   sc[2] = E0 = 2 sum_i f_ii + omega
__global__ void k_topfock(const double* Ft, const double* lam, int no, int nv, int mv, double* fo, double* fv,
                          double* fov, double* eo, double* ev, double* Fd, double* Fl, double* sc) {
  const int n = no + nv;
  double om = 0.0, tr = 0.0;
  for (int l = 0; l < no; ++l) {
    om += lam[l] * lam[l] * (Ft[(no + l) * n + no + l] - Ft[l * n + l]);
    tr += Ft[l * n + l];
  }
  const double ka = Ft[no * n + no] - Ft[0] - om;
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g == 0) { sc[0] = om; sc[1] = ka; sc[2] = 2.0 * tr + om; }
  if (g < (int64_t)mv * mv) {
    int a = g / mv, b = g % mv;
    // symmetric to the last bit (the Sylvester kernel reads F' by rows for both of its operands)
    double v = (a < nv && b < nv) ? 0.5 * (Ft[(no + a) * n + no + b] + Ft[(no + b) * n + no + a]) : 0.0;
    Fd[g] = v + ((a == b && a < nv) ? -0.5 * om : 0.0);
    Fl[g] = v + ((a == b && a < nv) ? 0.5 * ka : 0.0);
    if (a < nv && b < nv) fv[a * nv + b] = v;
  }
  if (g < no * no) fo[g] = Ft[(g / no) * n + g % no];
  if (g < no * nv) fov[g] = Ft[(g / nv) * n + no + g % nv];
  if (g < no) eo[g] = Ft[g * n + g];
  if (g < nv) ev[g] = Ft[(no + g) * n + no + g];
}

// ---------------------------------------------------------------------------
// handle
// ---------------------------------------------------------------------------
// Page-locked host block of one handle: every scalar the host reads back from
// the device lands here.  A copy into it is DMA into memory the handle owns,
// so no call leaves a device-to-host copy pending into pageable or stack
// memory, on any return path.
// return the status of a call that fails
#define ESMP2_TRY(call)                          \
  do {                                           \
    esmp2_status st_ = (call);                   \
    if (st_ != ESMP2_OK) return st_;             \
  } while (0)

struct PinnedScalars {
  double sc[SC_N];       // conjugate-gradient scalars (SC_* slots)
  double rot[4];         // omega, kappa, E0 of the rotation
  double lam[64];        // singular values (n_occ <= 64)
  double tmp[4];
  double e2s;
  int info[4];
  int bad[4];
  int active[2];         // batched solve: states still iterating, two iterations in flight
  CgCtl cg[2];           // device-stopped solve: the control word after iteration i, slot i % 2
};

struct esmp2_handle_ {
  int device = 0;
  PinnedScalars* pin = nullptr;
  hipStream_t stream = nullptr;
  std::string err = "no error";
  int state = 0;                 // 0 empty, 1 problem set, 2 rotated, 3 rhs built
  bool top_given = false;        // the problem was stated in the TOP basis (no rotation)
  double* gws = nullptr;         // workspace of the gradient (allocated on first use)
  size_t gws_n = 0;
  Dims d{};
  int ntop = 1;                  // large TOPs (ESMP2-TOP(k)); k > 1: the TOP(k) layout and operator
  int64_t namp = 0;              // amplitudes: off[7] for one large TOP, off[2] + k (off[7] - off[2]) for k
  signed char* s0 = nullptr;     // TOP(k): canonical phase of every element's operator string (0: masked slot)
  double *Ft_s = nullptr, *Bov_s = nullptr, *Bvt_s = nullptr, *Boo_s = nullptr, *lam_s = nullptr;   // relabelled inputs
  double* btmp = nullptr;        // TOP(k): one-TOP right-hand side of one relabelled problem
  std::vector<void*> allocs;     // everything owned, freed at reset/destroy
  // inputs
  double *F = nullptr, *B = nullptr, *C = nullptr;
  // rotation
  double *lam, *U, *V, *rs, *evals, *R, *avo, *Ft, *T, *Bov, *Bvt, *Boo;
  int* iinfo;
  double *fo, *fv, *fov, *eo, *ev, *Fd, *Fl, *sc_rot;
  double omega = 0, kappa = 0, e0 = 0, e2s = 0;
  int svd_sweeps = 0;
  // rhs
  double *fphi, *fphi_part, *X, *Vint, *Mint, *b, *blockmin, *partial, *sc;
  bool have_rhs = false;
  bool sc_vir_early = false;    // launch_sc_vir_early has queued the virtual eigenproblem
  bool b_top_pending = false;   // build_rhs left the TOP-basis b, M and 1/D for ensure_b_top
  // sigma scratch
  double *S, *side, *side_tr;
  int2* jobs = nullptr;
  int njobs = 0;
  int4* jobs4 = nullptr;
  int njobs4 = 0;
  int* pairs = nullptr;          // (p << 16) | q tables: virtual pairs, shifted virtual, occupied, shifted occupied
  int4* chunks = nullptr;        // coupling kernel work: (box, batch, first inner index or S2 tile, (p << 16) | q)
  int nchunks = 0;
  double* pq_part = nullptr;     // per-chunk parts of <p, Ap>_W (2 nchunks: also the fused CG start's two dots)
  bool sc_init_ready = false;    // rhs_semican left the CG start from x = 0 in p and pq_part
  // Krylov vectors
  double *x, *r, *p, *q;
  // FP32 operator (Fock blocks rounded from the FP64 ones, work buffers) and
  // the FP32 vectors of the inner solves of the mixed-precision refinement
  float *Fd32, *Fl32, *fo32, *fv32, *fov32, *S32, *side32, *side_tr32;
  float *d32, *r32, *p32, *q32;
  float* dinv32;                 // Jacobi preconditioner (FP32, for the FP64 and the FP32 solves)
  // pinned-semicanonical basis: rotations (t and t' fixed), operator blocks, rotated rhs,
  // Jacobi diagonal, dense scratch of the amplitude rotation
  bool have_sc_op = false;       // the operator blocks of the pinned-semicanonical basis are built
  bool have_sc = false;          // ... and the right-hand side is rotated into that basis
  // side stream: the semicanonical eigenproblems run there while the main
  // stream builds the right-hand side (default priority, non-blocking)
  hipStream_t aux = nullptr;
  hipEvent_t ev_fock_ready = nullptr, ev_sc_eig = nullptr;
  bool sc_pending = false;       // eigenproblems queued on the side stream, not yet joined
  // E2_S (S-triples, inverted directly) also runs on the side stream, beside the
  // solve: partials, then the sum at e2s_part[E2S_CAP]
  double* e2s_part = nullptr;
  hipEvent_t ev_rhs_ready = nullptr, ev_e2s = nullptr;
  hipEvent_t ev_cg[2] = {nullptr, nullptr};   // device-stopped solve: control word of iteration i copied (i % 2)
  hipEvent_t ev_bz = nullptr;                 // side stream: B_vv V of the rotation done
  double* Tz = nullptr;                       // B[Q][vir, vir] V, n_aux x n_vir x n_occ
  double* cgctl = nullptr;                    // its control word (a CgCtl)
  bool e2s_pending = false;      // queued on the side stream, not yet joined by the main stream
  bool e2s_dev = false;          // the sum is on the device, not yet read into e2s
  bool sc_eig = false;           // To, Tv hold the rotation of the current TOP basis
  double *To, *Tv, *Tsc, *Fh, *fo_sc, *fv_sc, *fov_sc, *eo_sc, *ev_sc, *Fd_sc, *Fl_sc, *b_sc;
  float *Fd32_sc, *Fl32_sc, *fo32_sc, *fv32_sc, *fov32_sc, *dinv32_sc;
  double *dense0, *dense1;       // two n_occ^2 n_vir^2 halves of one allocation
  double* rs2;            // scratch of the side stream's virtual eigenproblem (10 nv^2 + 8 nv)
  double* rsc;            // right-hand side in the pinned-semicanonical basis: C, fphi, Bov, X, one intermediate
  double* gv;                    // row/column GEMVs of the arrow-shaped Fock blocks (FP64 or FP32 use)
  // opt-in timing of the virtual-pair kernel with HIP events on the handle's stream,
  // per operator precision (index = esmp2_precision)
  int vv_variant[3] = {-1, -1, -1};   // Sylvester variant per esmp2_precision, -1: automatic
  bool prof = false;
  struct Ev { hipEvent_t a, b; int prec; };
  std::vector<Ev> ev_vv;
  double vv_ms[3] = {0.0, 0.0, 0.0};
  int64_t vv_launches[3] = {0, 0, 0};
};

static esmp2_status fail(esmp2_handle h, esmp2_status s, const std::string& msg) {
  if (h) h->err = msg;
  return s;
}

static void drain_events(esmp2_handle h) {
  for (auto& e : h->ev_vv) {
    float ms = 0.f;
    if (hipEventSynchronize(e.b) == hipSuccess && hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) {
      h->vv_ms[e.prec] += ms;
      h->vv_launches[e.prec] += 1;
    }
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  h->ev_vv.clear();
}

static void release(esmp2_handle h) {
  if (h->aux) (void)hipStreamSynchronize(h->aux);      // side-stream work may still read these buffers
  if (!h->allocs.empty()) (void)hipStreamSynchronize(h->stream);
  for (void* p : h->allocs) (void)hipFree(p);
  h->allocs.clear();
  h->state = 0;
  h->have_rhs = false;
  h->have_sc = false;
  h->sc_init_ready = false;
  h->have_sc_op = false;
  h->sc_pending = false;
  h->sc_eig = false;
  h->e2s_pending = false;
  h->e2s_dev = false;
  h->gws = nullptr;
  h->gws_n = 0;
}

// The main stream waits for E2_S queued on the side stream; with read, its
// value is also copied into h->e2s (a synchronous point).
static esmp2_status join_e2s(esmp2_handle h, bool read) {
  if (h->e2s_pending) {
    ESMP2_HIP(hipStreamWaitEvent(h->stream, h->ev_e2s, 0));
    h->e2s_pending = false;
  }
  if (read && h->e2s_dev) {
    ESMP2_HIP(hipMemcpyAsync(&h->pin->e2s, h->e2s_part + E2S_CAP, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    ESMP2_HIP(hipStreamSynchronize(h->stream));
    h->e2s = h->pin->e2s;
    h->e2s_dev = false;
  }
  return ESMP2_OK;
}

template <class T>
static bool dalloc(esmp2_handle h, T** p, size_t count) {
  void* ptr = nullptr;
  if (count == 0) count = 1;
  if (hipMalloc(&ptr, count * sizeof(T)) != hipSuccess) return false;
  h->allocs.push_back(ptr);
  *p = (T*)ptr;
  return true;
}

static inline unsigned nblk(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }
// workgroups of the grid-stride Jacobi-diagonal kernel (<= nblk(n): blockmin holds one entry per workgroup)
static inline unsigned diag_grid(int64_t n) { return std::min<unsigned>(nblk(n), (unsigned)DIAG_BLOCKS); }

// The Jacobi diagonal of a TOP(1) operator and its per-workgroup minima: by the
// coupling chunks where the table exists.  Returns the number of minima written.
static unsigned launch_diag(esmp2_handle h, const DiagArgs& da) {
  if (h->nchunks > 0) {
    const Dims& d = h->d;
    const int* pv = h->pairs;
    const PairTables pt{pv, pv + d.npv, pv + d.npv + d.npv1, pv + d.npv + d.npv1 + d.npo};
    const unsigned g = std::min<unsigned>((unsigned)((h->nchunks + DIAG_UNROLL - 1) / DIAG_UNROLL), diag_grid(h->namp));
    hipLaunchKernelGGL(k_diag_chunks, dim3(g), dim3(256), 0, h->stream, da, pt, (const int4*)h->chunks, h->nchunks);
    return g;
  }
  hipLaunchKernelGGL(k_diag, dim3(diag_grid(h->namp)), dim3(256), 0, h->stream, da);
  return diag_grid(h->namp);
}

// The right-hand side kernel: by the coupling chunks where the table exists
// (one large TOP), else one thread per flat position.
template <bool GEN>
static void launch_rhs(esmp2_handle h, const RhsArgs& ra, hipStream_t s) {
  const Dims& d = h->d;
  if (h->ntop == 1 && h->nchunks > 0) {
    const int* pv = h->pairs;
    const PairTables pt{pv, pv + d.npv, pv + d.npv + d.npv1, pv + d.npv + d.npv1 + d.npo};
    hipLaunchKernelGGL(k_rhs_chunks<GEN>, dim3(h->nchunks), dim3(256), 0, s, ra, pt, (const int4*)h->chunks);
  } else {
    hipLaunchKernelGGL(k_rhs<GEN>, dim3(nblk(d.off[7])), dim3(256), 0, s, ra);
  }
}

// Eigenpairs of a symmetric m x m matrix A (device, contiguous) by the
// tridiagonal route of the AVO step: evals ascending, Y[i*m + k] = component i
// of eigenvector k.  Scratch ws: 2 m^2 + 3 m doubles (m <= TRI_MAX).
// Raise a kernel's dynamic-LDS limit to what the device allows, once per
// process and device, before its first launch.  The limit is process-wide
// state of the function: setting it per launch, with sizes that differ
// between the host threads of a batched solve, would race with their launches.
static hipError_t allow_device_lds(const void* fn) {
  static std::mutex mu;
  static std::set<std::pair<const void*, int>> done;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(mu);
  if (done.count({fn, dev})) return hipSuccess;
  int per_block = 0;
  if ((e = hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev)) != hipSuccess) return e;
  hipFuncAttributes fa{};
  if ((e = hipFuncGetAttributes(&fa, fn)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, per_block - (int)fa.sharedSizeBytes)) !=
      hipSuccess)
    return e;
  done.insert({fn, dev});
  return hipSuccess;
}

static esmp2_status sym_eig(esmp2_handle h, hipStream_t s, const double* A, int m, double* evals, double* Y,
                            double* ws) {
  if (m <= 0) return ESMP2_OK;
  double* refl = ws;
  double* Zt = refl + (size_t)m * m;        // eigenvectors of the tridiagonal, one per row
  double* vec = Zt + (size_t)m * m;         // rbeta, d, e
  if (m == 1) {
    hipLaunchKernelGGL(k_eig1, dim3(1), dim3(1), 0, s, A, evals, Y);
    return ESMP2_OK;
  }
  if (m > TRI_MAX) return fail(h, ESMP2_UNSUPPORTED, "eigenproblem order beyond the tridiagonal solver's limit");
  size_t lt = sizeof(double) * (size_t)m * (m + 1) / 2;
  ESMP2_HIP(allow_device_lds((const void*)k_tridiag));
  hipLaunchKernelGGL(k_tridiag, dim3(1), dim3(1024), lt, s, A, m, refl, vec, vec + m, vec + 2 * m);
  hipLaunchKernelGGL(k_tri_eig, dim3(m), dim3(64), 0, s, vec + m, vec + 2 * m, m, evals, Zt);
  hipLaunchKernelGGL(k_cluster_mgs, dim3(1), dim3(64), 0, s, evals, m, Zt);
  hipLaunchKernelGGL(k_backtransform, dim3(m), dim3(64), 0, s, refl, vec, m, Zt, Y);
  ESMP2_HIP(hipGetLastError());
  return ESMP2_OK;
}


// The virtual eigenproblem of the pinned-semicanonical rotation, queued on the
// side stream right after the SVD, beside the AVO eigenproblem of the main
// stream: virtuals 1.. of that basis span the complement of t' (virtual TOP
// vector 0), whatever basis the AVO step picks inside it, so they are the
// eigenvectors of F_vv on that complement, S = Q' Y' (Q' from one Householder
// reflector of t').  launch_semican_eig takes them into the TOP basis once W
// exists.  Scratch: rs2 = [Q' | Tt | Fa | Y' | S | ws (2 m^2 + 3 m) | refl | t' | evals].
static esmp2_status launch_sc_vir_early(esmp2_handle h) {
  const Dims& d = h->d;
  const int no = d.no, nv = d.nv, n = d.n, m = nv - 1;
  hipStream_t s = h->aux;
  ESMP2_HIP(hipEventRecord(h->ev_fock_ready, h->stream));
  ESMP2_HIP(hipStreamWaitEvent(s, h->ev_fock_ready, 0));
  const size_t v2 = (size_t)nv * nv;
  double* Qp = h->rs2;             // nv x m
  double* Tt = Qp + v2;            // nv x m
  double* Fa = Tt + v2;            // m x m
  double* Yp = Fa + v2;            // m x m
  double* S = Yp + v2;             // nv x m
  double* ws = S + v2;             // 2 m^2 + 3 m
  double* refl = ws + 3 * v2;      // nv + 1
  double* tp = refl + 2 * nv;      // nv
  double* evals = tp + 2 * nv;     // m
  // the rotation's B_vv V (the TOP virtuals V from the SVD; the AVOs are not
  // needed): Tz[Q] = B[Q][vir, vir] V, first on the side stream
  {
    GemmArgs g{};
    const int64_t nn = (int64_t)n * n;
    g.A = h->B + (int64_t)no * n + no; g.B = h->V; g.C = h->Tz; g.M = nv; g.N = no; g.K = nv;
    g.sAb = nn; g.sAi = n; g.sAk = 1; g.sBb = 0; g.sBk = no; g.sBj = 1; g.sCb = (int64_t)nv * no; g.sCi = no; g.sCj = 1;
    g.alpha = 1; g.beta = 0;
    ESMP2_HIP(gemm(s, d.naux, g));
    ESMP2_HIP(hipEventRecord(h->ev_bz, s));
  }
  hipLaunchKernelGGL(k_take_column, dim3(nblk(nv)), dim3(256), 0, s, (const double*)h->V, no, nv, tp);
  ESMP2_HIP(allow_device_lds((const void*)k_complement_qr));
  hipLaunchKernelGGL(k_complement_qr, dim3(1), dim3(1024), sizeof(double) * 3 * (size_t)nv, s, (const double*)tp, nv,
                     1, refl);
  hipLaunchKernelGGL(k_complement_apply, dim3(m), dim3(64), 0, s, (const double*)refl, nv, 1, Qp);
  GemmArgs g{};
  g.A = h->F + (int64_t)no * n + no; g.B = Qp; g.C = Tt; g.M = nv; g.N = m; g.K = nv;
  g.sAi = n; g.sAk = 1; g.sBk = m; g.sBj = 1; g.sCi = m; g.sCj = 1; g.alpha = 1; g.beta = 0;
  ESMP2_HIP(gemm(s, 1, g));
  g = GemmArgs{};
  g.A = Qp; g.B = Tt; g.C = Fa; g.M = m; g.N = m; g.K = nv;
  g.sAi = 1; g.sAk = m; g.sBk = m; g.sBj = 1; g.sCi = m; g.sCj = 1; g.alpha = 1; g.beta = 0;
  ESMP2_HIP(gemm(s, 1, g));
  const esmp2_status st = sym_eig(h, s, Fa, m, evals, Yp, ws);
  if (st != ESMP2_OK) return st;
  g = GemmArgs{};
  g.A = Qp; g.B = Yp; g.C = S; g.M = nv; g.N = m; g.K = m;
  g.sAi = m; g.sAk = 1; g.sBk = m; g.sBj = 1; g.sCi = m; g.sCj = 1; g.alpha = 1; g.beta = 0;
  ESMP2_HIP(gemm(s, 1, g));
  ESMP2_HIP(hipGetLastError());
  h->sc_vir_early = true;
  return ESMP2_OK;
}

// The two eigenproblems of the pinned-semicanonical rotation (F~_oo[1:,1:],
// F~_vv[1:,1:]), queued on the side stream as soon as F~ exists; semican_setup
// joins them.  The virtual one, when launch_sc_vir_early has solved it in the
// original basis, only needs its vectors taken into the TOP basis: W[:, 1:]^T S.
// Scratch: rs.
static esmp2_status launch_semican_eig(esmp2_handle h) {
  const Dims& d = h->d;
  const int no = d.no, nv = d.nv, n = d.n;
  hipStream_t s = h->aux;
  ESMP2_HIP(hipEventRecord(h->ev_fock_ready, h->stream));
  ESMP2_HIP(hipStreamWaitEvent(s, h->ev_fock_ready, 0));
  double* A = h->rs;                                   // (nv-1)^2 block copy
  double* evals = A + (size_t)nv * nv;
  double* Y = evals + nv;
  double* ws = Y + (size_t)nv * nv;                    // 2 nv^2 + 3 nv  (rs holds 11 nv^2)
  hipLaunchKernelGGL(k_block_copy, dim3(64), dim3(256), 0, s, (const double*)h->Ft, (int64_t)n + 1, n, no - 1, A);
  esmp2_status st = sym_eig(h, s, A, no - 1, evals, Y, ws);
  if (st != ESMP2_OK) return st;
  hipLaunchKernelGGL(k_embed_rotation, dim3(no), dim3(64), 0, s, (const double*)Y, no, h->To);
  if (h->sc_vir_early) {
    // Y[a-1][A-1] = sum_k W[k][a] S[k][A-1], a >= 1 (W = R[no:, no:])
    const int m = nv - 1;
    GemmArgs g{};
    g.A = h->R + (int64_t)no * n + no + 1; g.B = h->rs2 + 4 * (size_t)nv * nv; g.C = Y; g.M = m; g.N = m; g.K = nv;
    g.sAi = 1; g.sAk = n; g.sBk = m; g.sBj = 1; g.sCi = m; g.sCj = 1; g.alpha = 1; g.beta = 0;
    ESMP2_HIP(gemm(s, 1, g));
    h->sc_vir_early = false;
  } else {
    hipLaunchKernelGGL(k_block_copy, dim3(256), dim3(256), 0, s, (const double*)h->Ft, (int64_t)(no + 1) * n + no + 1,
                       n, nv - 1, A);
    st = sym_eig(h, s, A, nv - 1, evals, Y, ws);
    if (st != ESMP2_OK) return st;
  }
  hipLaunchKernelGGL(k_embed_rotation, dim3(nv), dim3(64), 0, s, (const double*)Y, nv, h->Tv);
  ESMP2_HIP(hipGetLastError());
  ESMP2_HIP(hipEventRecord(h->ev_sc_eig, s));
  h->sc_pending = true;
  return ESMP2_OK;
}

static esmp2_status scratch_address(esmp2_handle h, double** out);

extern "C" {

esmp2_status esmp2_create(esmp2_handle* out, int device, void* stream) {
  if (!out) return ESMP2_INVALID_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return ESMP2_INVALID_ARG;
  esmp2_handle h = new (std::nothrow) esmp2_handle_();
  if (!h) return ESMP2_OOM;
  h->device = device;
  h->stream = (hipStream_t)stream;
  if (hipSetDevice(device) != hipSuccess || hipHostMalloc((void**)&h->pin, sizeof(PinnedScalars), 0) != hipSuccess ||
      hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_fock_ready, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_sc_eig, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_rhs_ready, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_e2s, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_cg[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_cg[1], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_bz, hipEventDisableTiming) != hipSuccess) {
    if (h->aux) (void)hipStreamDestroy(h->aux);
    if (h->ev_cg[0]) (void)hipEventDestroy(h->ev_cg[0]);
    if (h->ev_cg[1]) (void)hipEventDestroy(h->ev_cg[1]);
    if (h->ev_bz) (void)hipEventDestroy(h->ev_bz);
    if (h->ev_fock_ready) (void)hipEventDestroy(h->ev_fock_ready);
    if (h->ev_sc_eig) (void)hipEventDestroy(h->ev_sc_eig);
    if (h->ev_rhs_ready) (void)hipEventDestroy(h->ev_rhs_ready);
    if (h->ev_e2s) (void)hipEventDestroy(h->ev_e2s);
    if (h->pin) (void)hipHostFree(h->pin);
    delete h;
    return ESMP2_HIP_ERROR;
  }
  {
    double* ws = nullptr;   // the allocation-free entry point's workspace on this device
    if (scratch_address(h, &ws) != ESMP2_OK) {
      (void)hipStreamDestroy(h->aux);
      (void)hipEventDestroy(h->ev_fock_ready);
      (void)hipEventDestroy(h->ev_sc_eig);
      (void)hipEventDestroy(h->ev_rhs_ready);
      (void)hipEventDestroy(h->ev_e2s);
      (void)hipEventDestroy(h->ev_cg[0]);
      (void)hipEventDestroy(h->ev_cg[1]);
      (void)hipEventDestroy(h->ev_bz);
      (void)hipHostFree(h->pin);
      delete h;
      return ESMP2_HIP_ERROR;
    }
  }
  *out = h;
  return ESMP2_OK;
}

esmp2_status esmp2_destroy(esmp2_handle h) {
  if (!h) return ESMP2_OK;
  (void)hipSetDevice(h->device);
  (void)hipStreamSynchronize(h->stream);
  (void)hipStreamSynchronize(h->aux);
  drain_events(h);
  release(h);
  (void)hipStreamDestroy(h->aux);
  (void)hipEventDestroy(h->ev_fock_ready);
  (void)hipEventDestroy(h->ev_sc_eig);
  (void)hipEventDestroy(h->ev_rhs_ready);
  (void)hipEventDestroy(h->ev_e2s);
  (void)hipEventDestroy(h->ev_cg[0]);
  (void)hipEventDestroy(h->ev_cg[1]);
  (void)hipEventDestroy(h->ev_bz);
  (void)hipHostFree(h->pin);
  delete h;
  return ESMP2_OK;
}

const char* esmp2_last_error(esmp2_handle h) { return h ? h->err.c_str() : "null handle"; }

esmp2_status esmp2_profile(esmp2_handle h, int enable, double* vv_ms, int64_t* vv_launches) {
  if (!h) return ESMP2_INVALID_ARG;
  ESMP2_HIP(hipSetDevice(h->device));
  drain_events(h);
  for (int k = 0; k < 3; ++k) {
    if (vv_ms) vv_ms[k] = h->vv_ms[k];
    if (vv_launches) vv_launches[k] = h->vv_launches[k];
    h->vv_ms[k] = 0.0;
    h->vv_launches[k] = 0;
  }
  h->prof = enable != 0;
  return ESMP2_OK;
}

esmp2_status esmp2_gemm_f64(esmp2_handle h, int m, int n, int k, const double* A, const double* B, double* C) {
  if (!h) return ESMP2_INVALID_ARG;
  if (m < 0 || n < 0 || k < 0 || (!A && m * k) || (!B && k * n) || (!C && m * n))
    return fail(h, ESMP2_INVALID_ARG, "bad gemm arguments");
  ESMP2_HIP(hipSetDevice(h->device));
  GemmArgs g{};
  g.A = A; g.B = B; g.C = C; g.M = m; g.N = n; g.K = k;
  g.sAi = k; g.sAk = 1; g.sBk = n; g.sBj = 1; g.sCi = n; g.sCj = 1; g.alpha = 1.0; g.beta = 0.0;
  ESMP2_HIP(gemm(h->stream, 1, g));
  return ESMP2_OK;
}

// kernel arguments of the TOP(k) path
static TopkArgs topk_args(esmp2_handle h) {
  TopkArgs a{};
  a.d = h->d;
  a.k = h->ntop;
  a.L1 = h->d.off[7] - h->d.off[2];
  a.namp = h->namp;
  a.Ft = h->Ft;
  a.omega = h->omega;
  a.sg = h->d.sg;
  a.s0 = h->s0;
  return a;
}

static esmp2_status check_sizes(esmp2_handle h, int n_occ, int n_vir, int n_aux) {
  if (n_occ < 2 || n_vir < n_occ || n_aux < 1)
    return fail(h, ESMP2_INVALID_ARG, "need 2 <= n_occ <= n_vir and n_aux >= 1");
  if (n_occ > 64 || (int64_t)n_occ * n_vir > 8192 || n_vir > 192)
    return fail(h, ESMP2_UNSUPPORTED, "sizes beyond n_occ <= 64, n_occ*n_vir <= 8192, n_vir <= 192");
  return ESMP2_OK;
}

// Allocation, tables and input copies shared by both ways of stating a problem:
// either C (the ESMF singles, rotated to the TOP basis later) or, for a problem
// already in the TOP basis, its singular values lam.
static esmp2_status setup_problem(esmp2_handle h, int n_occ, int n_vir, int n_aux, const double* F,
                                  const double* B, const double* C, const double* lam, int spin, int n_top) {
  ESMP2_HIP(hipSetDevice(h->device));
  ESMP2_HIP(hipStreamSynchronize(h->stream));
  release(h);
  Dims d = make_dims(n_occ, n_vir, n_aux);
  d.sg = spin ? -1 : 1;
  h->d = d;
  const int no = n_occ, nv = n_vir, n = d.n, na = n_aux, mv = d.mv;
  h->ntop = n_top;
  h->namp = d.off[2] + (int64_t)n_top * (d.off[7] - d.off[2]);
  const int64_t namp = h->namp;
  bool ok = dalloc(h, &h->F, (size_t)n * n) && dalloc(h, &h->B, (size_t)na * n * n) &&
            dalloc(h, &h->C, (size_t)no * nv) && dalloc(h, &h->lam, no) && dalloc(h, &h->U, no * no) &&
            dalloc(h, &h->V, (size_t)nv * no) && dalloc(h, &h->rs, (size_t)11 * nv * nv) &&
            dalloc(h, &h->evals, nv) && dalloc(h, &h->R, (size_t)n * n) &&
            dalloc(h, &h->avo, nv) && dalloc(h, &h->Ft, (size_t)n * n) &&
            dalloc(h, &h->T, std::max((size_t)na * no * nv, (size_t)n * n)) &&
            dalloc(h, &h->Tz, (size_t)na * nv * no) &&
            dalloc(h, &h->Bov, 2 * (size_t)na * no * nv) && dalloc(h, &h->Bvt, (size_t)na * nv * no) &&
            dalloc(h, &h->Boo, (size_t)na * no * no) && dalloc(h, &h->iinfo, 8) && dalloc(h, &h->fo, no * no) &&
            dalloc(h, &h->fv, (size_t)nv * nv) && dalloc(h, &h->fov, (size_t)no * nv) && dalloc(h, &h->eo, no) &&
            dalloc(h, &h->ev, nv) && dalloc(h, &h->Fd, (size_t)mv * mv) && dalloc(h, &h->Fl, (size_t)mv * mv) &&
            dalloc(h, &h->sc_rot, 8) && dalloc(h, &h->fphi, (size_t)no * nv) &&
            dalloc(h, &h->fphi_part, (size_t)FPHI_QCHUNKS * no * nv + na) &&
            dalloc(h, &h->Vint, (size_t)no * nv * no * nv) &&
            dalloc(h, &h->Mint, (size_t)no * nv * no * nv) && dalloc(h, &h->b, namp) &&
            dalloc(h, &h->blockmin, nblk(namp)) &&
            dalloc(h, &h->partial, (size_t)4 * PCG_BLOCKS) && dalloc(h, &h->sc, SC_N) &&
            dalloc(h, &h->e2s_part, (size_t)E2S_CAP + 2) &&
            dalloc(h, &h->S, (size_t)no * no * nv * nv) &&
            dalloc(h, &h->side, (size_t)nv * (3 * d.npo1 + 2 * d.npo + 3 * d.npo + 5 * (no - 1) * (no - 1))) &&
            dalloc(h, &h->side_tr, (size_t)nv * (d.npo + (no - 1) * (no - 1))) &&
            dalloc(h, &h->x, namp) && dalloc(h, &h->r, namp) && dalloc(h, &h->p, namp) && dalloc(h, &h->q, namp);
  ok = ok && dalloc(h, &h->Fd32, (size_t)mv * mv) && dalloc(h, &h->Fl32, (size_t)mv * mv) &&
       dalloc(h, &h->fo32, no * no) && dalloc(h, &h->fv32, (size_t)nv * nv) && dalloc(h, &h->fov32, (size_t)no * nv) &&
       dalloc(h, &h->S32, (size_t)no * no * nv * nv) &&
       dalloc(h, &h->side32, (size_t)nv * (3 * d.npo1 + 2 * d.npo + 3 * d.npo + 5 * (no - 1) * (no - 1))) &&
       dalloc(h, &h->side_tr32, (size_t)nv * (d.npo + (no - 1) * (no - 1))) && dalloc(h, &h->d32, namp) &&
       dalloc(h, &h->r32, namp) && dalloc(h, &h->p32, namp) && dalloc(h, &h->q32, namp) &&
       dalloc(h, &h->dinv32, namp);
  const size_t dense = (size_t)no * no * nv * nv;
  ok = ok && dalloc(h, &h->To, no * no) && dalloc(h, &h->Tv, (size_t)nv * nv) && dalloc(h, &h->Tsc, (size_t)n * n) &&
       dalloc(h, &h->Fh, (size_t)n * n) && dalloc(h, &h->fo_sc, no * no) && dalloc(h, &h->fv_sc, (size_t)nv * nv) &&
       dalloc(h, &h->fov_sc, (size_t)no * nv) && dalloc(h, &h->eo_sc, no) && dalloc(h, &h->ev_sc, nv) &&
       dalloc(h, &h->Fd_sc, (size_t)mv * mv) && dalloc(h, &h->Fl_sc, (size_t)mv * mv) &&
       dalloc(h, &h->b_sc, namp) && dalloc(h, &h->Fd32_sc, (size_t)mv * mv) &&
       dalloc(h, &h->Fl32_sc, (size_t)mv * mv) && dalloc(h, &h->fo32_sc, no * no) &&
       dalloc(h, &h->fv32_sc, (size_t)nv * nv) && dalloc(h, &h->fov32_sc, (size_t)no * nv) &&
       dalloc(h, &h->dinv32_sc, namp) && dalloc(h, &h->dense0, 2 * dense) &&
       dalloc(h, &h->rsc, (size_t)no * nv * (2 + 4 * (size_t)na)) &&
       dalloc(h, &h->rs2, (size_t)10 * nv * nv + 8 * (size_t)nv) && dalloc(h, &h->cgctl, 4) &&
       dalloc(h, &h->gv, (size_t)nv * (2 * d.npo + 2 * no * no + (no - 1) * (no - 1)));
  if (n_top > 1)
    ok = ok && dalloc(h, &h->s0, namp) && dalloc(h, &h->Ft_s, (size_t)n * n) &&
         dalloc(h, &h->Bov_s, (size_t)na * no * nv) && dalloc(h, &h->Bvt_s, (size_t)na * nv * no) &&
         dalloc(h, &h->Boo_s, (size_t)na * no * no) && dalloc(h, &h->lam_s, no) && dalloc(h, &h->btmp, d.off[7]);
  if (ok) h->dense1 = h->dense0 + dense;        // the second half of one allocation
  if (ok) h->X = h->Bov + (size_t)na * no * nv;  // right after Bov: the two are rotated as one stack
  if (!ok) { release(h); return fail(h, ESMP2_OOM, "device allocation failed"); }
  // vv job table
  std::vector<int2> jobs;
  int nbat[7] = {d.npo, no * no, d.npo1, d.npo, d.npo, (no - 1) * (no - 1), (no - 1) * (no - 1)};
  for (int bx = 0; bx < 7; ++bx)
    for (int k = 0; k < nbat[bx]; ++k) jobs.push_back(make_int2(bx, k));
  h->njobs = (int)jobs.size();
  // k_vv2 jobs: dense-output work first (heaviest), then triangular outputs
  std::vector<int4> j4;
  // (box, batch or i, storage/output format code of k_vv3, j)
  for (int k = 0; k < (no - 1) * (no - 1); ++k) j4.push_back(make_int4(B_H22, k, 2, 0));
  for (int k = 0; k < d.npo; ++k) j4.push_back(make_int4(B_H12, k, 2, 0));
  for (int i = 0; i < no; ++i)
    for (int j = i + 1; j < no; ++j) j4.push_back(make_int4(B_S2, i, 3, j));
  for (int k = 0; k < (no - 1) * (no - 1); ++k) j4.push_back(make_int4(B_H21, k, 0, 0));
  for (int k = 0; k < d.npo; ++k) j4.push_back(make_int4(B_H11, k, 0, 0));
  for (int k = 0; k < d.npo; ++k) j4.push_back(make_int4(B_T2, k, 0, 0));
  for (int k = 0; k < d.npo1; ++k) j4.push_back(make_int4(B_T3, k, 1, 0));
  for (int i = 0; i < no; ++i) j4.push_back(make_int4(B_S2, i, 4, i));
  h->njobs4 = (int)j4.size();
  std::vector<int> pairs;
  auto add_pairs = [&](int m) {
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) pairs.push_back((p << 16) | q);
  };
  add_pairs(nv); add_pairs(nv - 1); add_pairs(no); add_pairs(no - 1);
  std::vector<int4> chunks;
  {
    const int inner[7] = {d.npv, nv * nv, d.npv1, d.npv, (nv - 1) * (nv - 1), d.npv, (nv - 1) * (nv - 1)};
    for (int bx = 0; bx < 7; ++bx)
      for (int k = 0; k < nbat[bx]; ++k) {
        int p = 0, q = 0;
        if (bx == B_T2 || bx == B_H11 || bx == B_H12 || bx == B_T3) {
          const int m = bx == B_T3 ? no - 1 : no;
          int r = k;
          while (r >= m - 1 - p) { r -= m - 1 - p; ++p; }
          q = p + 1 + r;
          if (bx == B_T3) { ++p; ++q; }
        } else if (bx == B_S2) {
          p = k / no; q = k % no;
        } else {
          p = k / (no - 1) + 1; q = k % (no - 1) + 1;
        }
        if (bx == B_S2) {             // 16 x 16 tiles of (a, b), row-major
          const int nt = (nv + 15) / 16;
          for (int ta = 0; ta < nt; ++ta)
            for (int tb = 0; tb < nt; ++tb) chunks.push_back(make_int4(bx, k, (ta << 16) | tb, (p << 16) | q));
        } else {
          for (int v0 = 0; v0 < inner[bx]; v0 += 256) chunks.push_back(make_int4(bx, k, v0, (p << 16) | q));
        }
      }
  }
  h->nchunks = (int)chunks.size();
  if (!dalloc(h, &h->jobs, jobs.size()) || !dalloc(h, &h->jobs4, j4.size()) || !dalloc(h, &h->pairs, pairs.size()) ||
      !dalloc(h, &h->chunks, chunks.size()) || !dalloc(h, &h->pq_part, 2 * chunks.size())) {
    release(h);
    return fail(h, ESMP2_OOM, "device allocation failed");
  }
  if (!pairs.empty())
    ESMP2_HIP(hipMemcpyAsync(h->pairs, pairs.data(), pairs.size() * sizeof(int), hipMemcpyHostToDevice, h->stream));
  if (!chunks.empty())
    ESMP2_HIP(hipMemcpyAsync(h->chunks, chunks.data(), chunks.size() * sizeof(int4), hipMemcpyHostToDevice, h->stream));
  ESMP2_HIP(hipMemcpyAsync(h->jobs4, j4.data(), j4.size() * sizeof(int4), hipMemcpyHostToDevice, h->stream));
  ESMP2_HIP(hipMemcpyAsync(h->jobs, jobs.data(), jobs.size() * sizeof(int2), hipMemcpyHostToDevice, h->stream));
  ESMP2_HIP(hipMemcpyAsync(h->F, F, sizeof(double) * n * n, hipMemcpyDefault, h->stream));
  ESMP2_HIP(hipMemcpyAsync(h->B, B, sizeof(double) * (size_t)na * n * n, hipMemcpyDefault, h->stream));
  if (C) ESMP2_HIP(hipMemcpyAsync(h->C, C, sizeof(double) * no * nv, hipMemcpyDefault, h->stream));
  else ESMP2_HIP(hipMemcpyAsync(h->lam, lam, sizeof(double) * no, hipMemcpyDefault, h->stream));
  // NaN / Inf check
  int* bad = h->iinfo;
  ESMP2_HIP(hipMemsetAsync(bad, 0, sizeof(int), h->stream));
  hipLaunchKernelGGL(k_finite, dim3(256), dim3(256), 0, h->stream, h->F, (int64_t)n * n, bad);
  hipLaunchKernelGGL(k_finite, dim3(1024), dim3(256), 0, h->stream, h->B, (int64_t)na * n * n, bad);
  if (C) hipLaunchKernelGGL(k_finite, dim3(64), dim3(256), 0, h->stream, h->C, (int64_t)no * nv, bad);
  else hipLaunchKernelGGL(k_finite, dim3(1), dim3(64), 0, h->stream, h->lam, (int64_t)no, bad);
  ESMP2_HIP(hipMemcpyAsync(h->pin->bad, bad, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  ESMP2_HIP(hipStreamSynchronize(h->stream));
  if (h->pin->bad[0]) { release(h); return fail(h, ESMP2_INVALID_ARG, C ? "NaN or Inf in F, B or C" : "NaN or Inf in F, B or lam"); }
  h->top_given = (C == nullptr);
  if (n_top > 1) {
    const TopkArgs ta = topk_args(h);
    hipLaunchKernelGGL(k_topk_phase, dim3(nblk(namp)), dim3(256), 0, h->stream, ta, h->s0);
    ESMP2_HIP(hipGetLastError());
  }
  h->state = 1;
  return ESMP2_OK;
}

esmp2_status esmp2_set_problem(esmp2_handle h, int n_occ, int n_vir, int n_aux, const double* F,
                               const double* B, const double* C, int spin, int n_top) {
  if (!h) return ESMP2_INVALID_ARG;
  if (!F || !B || !C) return fail(h, ESMP2_INVALID_ARG, "null input pointer");
  esmp2_status st = check_sizes(h, n_occ, n_vir, n_aux);
  if (st != ESMP2_OK) return st;
  if (spin != 0 && spin != 1) return fail(h, ESMP2_INVALID_ARG, "spin must be 0 (singlet) or 1 (triplet)");
  if (n_top < 1 || n_top > n_occ) return fail(h, ESMP2_INVALID_ARG, "n_top must lie in [1, n_occ]");
  return setup_problem(h, n_occ, n_vir, n_aux, F, B, C, nullptr, spin, n_top);
}

esmp2_status esmp2_set_problem_top(esmp2_handle h, int n_occ, int n_vir, int n_aux, const double* Ft,
                                   const double* Bt, const double* lam, int spin) {
  if (!h) return ESMP2_INVALID_ARG;
  if (!Ft || !Bt || !lam) return fail(h, ESMP2_INVALID_ARG, "null input pointer");
  if (spin != 0 && spin != 1) return fail(h, ESMP2_INVALID_ARG, "spin must be 0 (singlet) or 1 (triplet)");
  esmp2_status st = check_sizes(h, n_occ, n_vir, n_aux);
  if (st != ESMP2_OK) return st;
  std::vector<double> l(n_occ);
  ESMP2_HIP(hipSetDevice(h->device));
  ESMP2_HIP(hipMemcpy(l.data(), lam, sizeof(double) * n_occ, hipMemcpyDefault));
  double s2 = 0.0;
  for (int k = 0; k < n_occ; ++k) {
    if (!(l[k] >= 0.0) || !(l[k] <= l[0])) return fail(h, ESMP2_INVALID_ARG, "lam must be >= 0 with lam[0] the largest");
    s2 += l[k] * l[k];
  }
  if (!(fabs(s2 - 1.0) <= 1e-10)) return fail(h, ESMP2_INVALID_ARG, "sum of lam^2 must be 1 (normalised reference)");
  return setup_problem(h, n_occ, n_vir, n_aux, Ft, Bt, nullptr, lam, spin, 1);
}

esmp2_status esmp2_rotate_top(esmp2_handle h, double* lambda_out) {
  if (!h) return ESMP2_INVALID_ARG;
  if (h->state < 1) return fail(h, ESMP2_BAD_ORDER, "esmp2_set_problem first");
  ESMP2_HIP(hipSetDevice(h->device));
  const Dims& d = h->d;
  const int no = d.no, nv = d.nv, n = d.n, na = d.naux, mv = d.mv;
  hipStream_t s = h->stream;
  // side-stream work of a previous rotation shares the scratch, and E2_S reads
  // what the rotation rewrites: order after both
  {
    const esmp2_status st = join_e2s(h, false);
    if (st != ESMP2_OK) return st;
  }
  if (h->sc_pending) {
    ESMP2_HIP(hipStreamWaitEvent(s, h->ev_sc_eig, 0));
    h->sc_pending = false;
  }
  h->sc_eig = false;
  GemmArgs g{};
  if (!h->top_given) {
    // SVD of C
    size_t lds = sizeof(double) * (no * nv + no * no);
    ESMP2_HIP(allow_device_lds((const void*)k_svd_jacobi));
    hipLaunchKernelGGL(k_svd_jacobi, dim3(1), dim3(512), lds, s, h->C, no, nv, h->lam, h->U, h->V, h->iinfo);
    {
      const esmp2_status st = launch_sc_vir_early(h);
      if (st != ESMP2_OK) return st;
    }
    // semicanonical AVOs: complement of the TOP virtuals, F restricted to it,
    // tridiagonal eigensolver, back-transformation, Loewdin re-orthonormalisation
    {
      const int m = nv - no;
      double* Q2 = h->rs;                                 // nv x m
      double* Tt = Q2 + (size_t)nv * nv;                  // nv x m
      double* Fa = Tt + (size_t)nv * nv;                  // m x m
      double* refl = Fa + (size_t)nv * nv;                // complement reflectors (nv x nv)
      double* Ym = refl + (size_t)nv * nv;                // m x m
      double* AV = Ym + (size_t)nv * nv;                  // nv x m; with AV2.. the eigensolver's scratch
      double* AV2 = AV + (size_t)nv * nv;                 // nv x m  (rs holds 11 nv^2)
      size_t lc = sizeof(double) * (size_t)nv * (2 * no + 1);    // padded working copy + reflectors
      if (m > 0) {   // n_vir == n_occ: no AVOs
      ESMP2_HIP(allow_device_lds((const void*)k_complement_qr));
      hipLaunchKernelGGL(k_complement_qr, dim3(1), dim3(1024), lc, s, (const double*)h->V, nv, no, refl);
      if (m > 0) hipLaunchKernelGGL(k_complement_apply, dim3(m), dim3(64), 0, s, (const double*)refl, nv, no, Q2);
      GemmArgs g{};
      g.A = h->F + (int64_t)no * n + no; g.B = Q2; g.C = Tt; g.M = nv; g.N = m; g.K = nv;
      g.sAi = n; g.sAk = 1; g.sBk = m; g.sBj = 1; g.sCi = m; g.sCj = 1; g.alpha = 1; g.beta = 0;
      ESMP2_HIP(gemm(s, 1, g));
      g = GemmArgs{};
      g.A = Q2; g.B = Tt; g.C = Fa; g.M = m; g.N = m; g.K = nv;
      g.sAi = 1; g.sAk = m; g.sBk = m; g.sBj = 1; g.sCi = m; g.sCj = 1; g.alpha = 1; g.beta = 0;
      ESMP2_HIP(gemm(s, 1, g));
      {
        const esmp2_status st = sym_eig(h, s, Fa, m, h->evals, Ym, AV);   // 2 m^2 + 3 m <= 6 nv^2 free from AV on
        if (st != ESMP2_OK) return st;
      }
      g = GemmArgs{};
      g.A = Q2; g.B = Ym; g.C = AV; g.M = nv; g.N = m; g.K = m;
      g.sAi = m; g.sAk = 1; g.sBk = m; g.sBj = 1; g.sCi = m; g.sCj = 1; g.alpha = 1; g.beta = 0;
      ESMP2_HIP(gemm(s, 1, g));
      // one first-order Loewdin step: AV <- AV - AV (AV^T AV - 1) / 2
      g = GemmArgs{};
      g.A = AV; g.B = AV; g.C = Fa; g.M = m; g.N = m; g.K = nv;
      g.sAi = 1; g.sAk = m; g.sBk = m; g.sBj = 1; g.sCi = m; g.sCj = 1; g.alpha = 1; g.beta = 0;
      ESMP2_HIP(gemm(s, 1, g));
      hipLaunchKernelGGL(k_sub_identity, dim3(nblk(m)), dim3(256), 0, s, Fa, m);
      ESMP2_HIP(hipMemcpyAsync(AV2, AV, sizeof(double) * nv * m, hipMemcpyDeviceToDevice, s));
      g = GemmArgs{};
      g.A = AV; g.B = Fa; g.C = AV2; g.M = nv; g.N = m; g.K = m;
      g.sAi = m; g.sAk = 1; g.sBk = m; g.sBj = 1; g.sCi = m; g.sCj = 1; g.alpha = -0.5; g.beta = 1.0;
      ESMP2_HIP(gemm(s, 1, g));
      }
      hipLaunchKernelGGL(k_assemble_r2, dim3(n), dim3(64), 0, s, h->U, h->V, AV2, h->evals, no, nv, h->R, h->avo);
    }
    // F~ = R^T F R
    g = GemmArgs{};
    g.A = h->F; g.B = h->R; g.C = h->T; g.M = n; g.N = n; g.K = n;
    g.sAi = n; g.sAk = 1; g.sBk = n; g.sBj = 1; g.sCi = n; g.sCj = 1; g.alpha = 1; g.beta = 0;
    ESMP2_HIP(gemm(s, 1, g));   // T = F R
    g = GemmArgs{};
    g.A = h->R; g.B = h->T; g.C = h->Ft; g.M = n; g.N = n; g.K = n;
    g.sAi = 1; g.sAk = n; g.sBk = n; g.sBj = 1; g.sCi = n; g.sCj = 1; g.alpha = 1; g.beta = 0;
    ESMP2_HIP(gemm(s, 1, g));   // Ft = R^T T
  } else {
    // stated in the TOP basis: the rotation is the identity
    ESMP2_HIP(hipMemcpyAsync(h->Ft, h->F, sizeof(double) * n * n, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_identity, dim3(nblk((int64_t)n * n)), dim3(256), 0, s, h->R, n);
    ESMP2_HIP(hipMemsetAsync(h->iinfo, 0, sizeof(int), s));
  }
  hipLaunchKernelGGL(k_topfock, dim3(nblk((int64_t)mv * mv > n * n ? (int64_t)mv * mv : (int64_t)n * n)), dim3(256),
                     0, s, h->Ft, h->lam, no, nv, mv, h->fo, h->fv, h->fov, h->eo, h->ev, h->Fd, h->Fl, h->sc_rot);
  // the FP32 operator's Fock blocks, rounded from the FP64 ones
  {
    const ToF32Set t{{h->Fd, h->Fl, h->fo, h->fv, h->fov}, {h->Fd32, h->Fl32, h->fo32, h->fv32, h->fov32},
                     {(int64_t)mv * mv, (int64_t)mv * mv, (int64_t)no * no, (int64_t)nv * nv, (int64_t)no * nv}};
    hipLaunchKernelGGL(k_to_f32_set, dim3(nblk((int64_t)mv * mv)), dim3(256), 0, s, t);
  }
  {
    esmp2_status st = launch_semican_eig(h);
    if (st != ESMP2_OK) return st;
  }
  if (!h->top_given) {
    // B~ blocks: Bov = U^T B_ov W, Bvt = W^T B_vv W[:, :no], Boo = U^T B_oo U
    const int64_t nn = (int64_t)n * n;
    // T[Q] (no x nv) = B[Q][occ, vir] W
    g = GemmArgs{};
    g.A = h->B + no; g.B = h->R + (int64_t)no * n + no; g.C = h->T; g.M = no; g.N = nv; g.K = nv;
    g.sAb = nn; g.sAi = n; g.sAk = 1; g.sBb = 0; g.sBk = n; g.sBj = 1; g.sCb = (int64_t)no * nv; g.sCi = nv; g.sCj = 1;
    g.alpha = 1; g.beta = 0;
    ESMP2_HIP(gemm(s, na, g));
    g = GemmArgs{};
    g.A = h->R; g.B = h->T; g.C = h->Bov; g.M = no; g.N = nv; g.K = no;
    g.sAb = 0; g.sAi = 1; g.sAk = n; g.sBb = (int64_t)no * nv; g.sBk = nv; g.sBj = 1;
    g.sCb = (int64_t)no * nv; g.sCi = nv; g.sCj = 1; g.alpha = 1; g.beta = 0;
    ESMP2_HIP(gemm(s, na, g));
    // Tz[Q] = B[Q][vir, vir] W[:, :no] came from the side stream (W[:, :no] = V)
    ESMP2_HIP(hipStreamWaitEvent(s, h->ev_bz, 0));
    g = GemmArgs{};
    g.A = h->R + (int64_t)no * n + no; g.B = h->Tz; g.C = h->Bvt; g.M = nv; g.N = no; g.K = nv;
    g.sAb = 0; g.sAi = 1; g.sAk = n; g.sBb = (int64_t)nv * no; g.sBk = no; g.sBj = 1;
    g.sCb = (int64_t)nv * no; g.sCi = no; g.sCj = 1; g.alpha = 1; g.beta = 0;
    ESMP2_HIP(gemm(s, na, g));
    // T[Q] (no x no) = B[Q][occ, occ] U ; Boo = U^T T
    g = GemmArgs{};
    g.A = h->B; g.B = h->R; g.C = h->T; g.M = no; g.N = no; g.K = no;
    g.sAb = nn; g.sAi = n; g.sAk = 1; g.sBb = 0; g.sBk = n; g.sBj = 1; g.sCb = (int64_t)no * no; g.sCi = no; g.sCj = 1;
    g.alpha = 1; g.beta = 0;
    ESMP2_HIP(gemm(s, na, g));
    g = GemmArgs{};
    g.A = h->R; g.B = h->T; g.C = h->Boo; g.M = no; g.N = no; g.K = no;
    g.sAb = 0; g.sAi = 1; g.sAk = n; g.sBb = (int64_t)no * no; g.sBk = no; g.sBj = 1;
    g.sCb = (int64_t)no * no; g.sCi = no; g.sCj = 1; g.alpha = 1; g.beta = 0;
    ESMP2_HIP(gemm(s, na, g));
  } else {
    // the factor is given in the TOP basis: its blocks are read off directly
    hipLaunchKernelGGL(k_extract_blocks, dim3(1024), dim3(256), 0, s, (const double*)h->B, no, nv, na, h->Bov,
                       h->Bvt, h->Boo);
  }
  PinnedScalars* pin = h->pin;
  ESMP2_HIP(hipMemcpyAsync(pin->rot, h->sc_rot, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  ESMP2_HIP(hipMemcpyAsync(pin->info, h->iinfo, sizeof(int), hipMemcpyDeviceToHost, s));
  if (lambda_out) ESMP2_HIP(hipMemcpyAsync(pin->lam, h->lam, no * sizeof(double), hipMemcpyDeviceToHost, s));
  ESMP2_HIP(hipStreamSynchronize(s));
  ESMP2_HIP(hipGetLastError());
  if (lambda_out) memcpy(lambda_out, pin->lam, no * sizeof(double));
  h->omega = pin->rot[0]; h->kappa = pin->rot[1]; h->e0 = pin->rot[2];
  h->svd_sweeps = pin->info[0];
  h->state = 2;
  h->have_rhs = false;
  h->have_sc = false;
  h->sc_init_ready = false;
  h->have_sc_op = false;
  return ESMP2_OK;
}

esmp2_status esmp2_space(esmp2_handle h, int64_t* n_amp, int64_t* box_offsets) {
  if (!h) return ESMP2_INVALID_ARG;
  if (h->state < 1) return fail(h, ESMP2_BAD_ORDER, "esmp2_set_problem first");
  if (n_amp) *n_amp = h->namp;
  if (box_offsets) for (int k = 0; k < 8; ++k) box_offsets[k] = h->d.off[k];
  return ESMP2_OK;
}

// The one-TOP right-hand side b_mu = <mu|H|Psi0> of the problem given by its
// TOP-basis blocks (Ft, Bov, Bvt, Boo, lam) into b (one-TOP layout); scratch:
// fphi, X, Vint, Mint.
static esmp2_status rhs_core(esmp2_handle h, const double* Ft, const double* Bov, const double* Bvt,
                             const double* Boo, const double* lam, double* b, bool defer_b = false) {
  const Dims& d = h->d;
  const int no = d.no, nv = d.nv, na = d.naux, nov = no * nv;
  hipStream_t s = h->stream;
  double* dq = h->fphi_part + (size_t)FPHI_QCHUNKS * nov;
  hipLaunchKernelGGL(k_fphi_dq, dim3(nblk(na)), dim3(256), 0, s, Bvt, Boo, lam, no, nv, na, dq);
  hipLaunchKernelGGL(k_fphi_part, dim3(FPHI_QCHUNKS, no), dim3(256), 0, s, Bov, Bvt, Boo, lam, (const double*)dq, no,
                     nv, na, h->fphi_part);
  hipLaunchKernelGGL(k_fphi_sum, dim3(nblk(nov)), dim3(256), 0, s, Ft, (const double*)h->fphi_part, no, nv,
                     FPHI_QCHUNKS, h->fphi);
  hipLaunchKernelGGL(k_make_x, dim3(nblk((int64_t)na * nov)), dim3(256), 0, s, Bvt, Boo, lam, no, nv, na, h->X);
  GemmArgs g{};
  // V[(ia),(jb)] = sum_Q Bov[Q][(ia)] Bov[Q][(jb)]
  g.A = Bov; g.B = Bov; g.C = h->Vint; g.M = nov; g.N = nov; g.K = na;
  g.sAi = 1; g.sAk = nov; g.sBk = nov; g.sBj = 1; g.sCi = nov; g.sCj = 1; g.alpha = 1; g.beta = 0;
  ESMP2_HIP(gemm(s, 1, g));
  if (defer_b) return ESMP2_OK;
  g.A = h->X; g.C = h->Mint;
  ESMP2_HIP(gemm(s, 1, g));
  RhsArgs ra{d, h->Vint, h->Mint, h->fphi, lam, b, nullptr};
  launch_rhs<false>(h, ra, s);
  ESMP2_HIP(hipGetLastError());
  return ESMP2_OK;
}

// The one-TOP right-hand side and Jacobi diagonal in the TOP basis, left for
// later by build_rhs (a solve in the pinned-semicanonical basis builds its own
// and never reads these): M = X^T Bov, b from V, M, f^Phi, and 1/D.
static esmp2_status ensure_b_top(esmp2_handle h) {
  if (!h->b_top_pending) return ESMP2_OK;
  const Dims& d = h->d;
  const int nov = d.no * d.nv;
  GemmArgs g{};
  g.A = h->X; g.B = h->Bov; g.C = h->Mint; g.M = nov; g.N = nov; g.K = d.naux;
  g.sAi = 1; g.sAk = nov; g.sBk = nov; g.sBj = 1; g.sCi = nov; g.sCj = 1; g.alpha = 1; g.beta = 0;
  ESMP2_HIP(gemm(h->stream, 1, g));
  RhsArgs ra{d, h->Vint, h->Mint, h->fphi, h->lam, h->b, nullptr};
  launch_rhs<false>(h, ra, h->stream);
  DiagArgs da{d, h->eo, h->ev, h->omega, h->dinv32, h->blockmin};
  (void)launch_diag(h, da);
  ESMP2_HIP(hipGetLastError());
  h->b_top_pending = false;
  return ESMP2_OK;
}

static esmp2_status build_rhs(esmp2_handle h) {
  {
    const esmp2_status st = join_e2s(h, false);   // the previous E2_S still reads Vint and e2s_part
    if (st != ESMP2_OK) return st;
  }
  const Dims& d = h->d;
  const int no = d.no, nv = d.nv;
  const int64_t namp = h->namp;
  hipStream_t s = h->stream;
  {
    h->b_top_pending = false;
    const esmp2_status st = rhs_core(h, h->Ft, h->Bov, h->Bvt, h->Boo, h->lam, h->ntop > 1 ? h->btmp : h->b,
                                     h->ntop == 1);
    if (st != ESMP2_OK) return st;
    h->b_top_pending = h->ntop == 1;
  }
  if (h->ntop == 1) {
    // the smallest denominator from the orbital energies; the TOP-basis
    // diagonal itself waits for ensure_b_top with b
    hipLaunchKernelGGL(k_diag_min, dim3(1), dim3(64), 0, s, d, (const double*)h->eo, (const double*)h->ev, h->omega,
                       h->sc + SC_TMP);
  } else {
    const TopkArgs ta = topk_args(h);
    hipLaunchKernelGGL(k_topk_bset, dim3(nblk(d.off[7])), dim3(256), 0, s, ta, 0, (const double*)h->btmp, h->b);
    hipLaunchKernelGGL(k_topk_diag, dim3(nblk(namp)), dim3(256), 0, s, ta, h->dinv32, h->blockmin);
    hipLaunchKernelGGL(k_min_reduce, dim3(1), dim3(1024), 0, s, h->blockmin, (int64_t)nblk(namp), h->sc + SC_TMP);
  }
  // E2_S on the side stream (after the eigenproblems queued there), beside the
  // solve: it reads Vint, lam, eo, ev, omega and the pair tables, which the
  // next rotation or right-hand side rewrites only after joining it.  Grids of
  // at most 1024 blocks each; partials laid out one kernel after the other.
  ESMP2_HIP(hipEventRecord(h->ev_rhs_ready, s));
  ESMP2_HIP(hipStreamWaitEvent(h->aux, h->ev_rhs_ready, 0));
  const int* pv = h->pairs;
  E2sArgs ea{d, h->Vint, h->lam, h->eo, h->ev, h->omega, h->e2s_part, pv, pv + d.npv, pv + d.npv + d.npv1,
             pv + d.npv + d.npv1 + d.npo};
  const int y1 = std::max(1, no - 1), x1 = std::max(1, 1024 / y1);
  const int y3 = std::min(1024, no * nv), x3 = std::max(1, 1024 / y3);
  const int nb1 = x1 * y1, nb3 = x3 * y3;
  if (2 * nb1 + nb3 > E2S_CAP) return fail(h, ESMP2_HIP_ERROR, "internal: E2_S partials beyond their buffer");
  hipLaunchKernelGGL(k_e2s_same, dim3(x1, y1), dim3(256), 0, h->aux, ea);
  ea.partial = h->e2s_part + nb1;
  hipLaunchKernelGGL(k_e2s_mixed_a, dim3(x1, y1), dim3(256), 0, h->aux, ea);
  ea.partial = h->e2s_part + 2 * nb1;
  hipLaunchKernelGGL(k_e2s_mixed_b, dim3(x3, y3), dim3(256), 0, h->aux, ea);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, h->aux, (const double*)h->e2s_part, 2 * nb1 + nb3,
                     h->e2s_part + E2S_CAP, -1.0);
  ESMP2_HIP(hipEventRecord(h->ev_e2s, h->aux));
  h->e2s_pending = true;
  h->e2s_dev = true;
  if (h->ntop > 1) {
    // the other large TOPs: the one-TOP right-hand side of each relabelled
    // problem (after E2_S has read Vint), its L-boxes into set s; then the
    // S-triples that TOP(k) moves into L leave E2_S
    const esmp2_status st0 = join_e2s(h, false);
    if (st0 != ESMP2_OK) return st0;
    const TopkArgs ta = topk_args(h);
    for (int t = 1; t < h->ntop; ++t) {
      hipLaunchKernelGGL(k_topk_permute, dim3(1024), dim3(256), 0, s, t, no, nv, d.naux, (const double*)h->Ft,
                         (const double*)h->Bov, (const double*)h->Bvt, (const double*)h->Boo, (const double*)h->lam,
                         h->Ft_s, h->Bov_s, h->Bvt_s, h->Boo_s, h->lam_s);
      const esmp2_status st = rhs_core(h, h->Ft_s, h->Bov_s, h->Bvt_s, h->Boo_s, h->lam_s, h->btmp);
      if (st != ESMP2_OK) return st;
      hipLaunchKernelGGL(k_topk_bset, dim3(nblk(d.off[7] - d.off[2])), dim3(256), 0, s, ta, t,
                         (const double*)h->btmp, h->b);
    }
    hipLaunchKernelGGL(k_topk_e2s, dim3(PCG_BLOCKS), dim3(256), 0, s, ta, (const double*)h->b, h->partial);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, s, (const double*)h->partial, (int)PCG_BLOCKS,
                       h->e2s_part + E2S_CAP + 1, 1.0);
    hipLaunchKernelGGL(k_add_to, dim3(1), dim3(64), 0, s, h->e2s_part + E2S_CAP, (const double*)h->e2s_part + E2S_CAP + 1);
    ESMP2_HIP(hipGetLastError());
  }
  ESMP2_HIP(hipMemcpyAsync(h->pin->tmp, h->sc + SC_TMP, sizeof(double), hipMemcpyDeviceToHost, s));
  ESMP2_HIP(hipStreamSynchronize(s));
  ESMP2_HIP(hipGetLastError());
  if (!(h->pin->tmp[0] > 0.0)) return fail(h, ESMP2_NOT_SPD, "a diagonal denominator of the first-order space is <= 0");
  h->have_rhs = true;
  h->have_sc = false;
  h->sc_init_ready = false;
  h->state = 3;
  return ESMP2_OK;
}

esmp2_status esmp2_build_rhs(esmp2_handle h, double* b_out, double* e0, double* e2_s) {
  if (!h) return ESMP2_INVALID_ARG;
  if (h->state < 2) return fail(h, ESMP2_BAD_ORDER, "esmp2_rotate_top first");
  ESMP2_HIP(hipSetDevice(h->device));
  esmp2_status st = build_rhs(h);
  if (st != ESMP2_OK) return st;
  if (b_out) {
    st = ensure_b_top(h);
    if (st != ESMP2_OK) return st;
    ESMP2_HIP(hipMemcpyAsync(b_out, h->b, sizeof(double) * h->namp, hipMemcpyDeviceToDevice, h->stream));
  }
  if (e0) *e0 = h->e0;
  if (e2_s) {
    st = join_e2s(h, true);
    if (st != ESMP2_OK) return st;
    *e2_s = h->e2s;
  }
  return ESMP2_OK;
}

}  // extern "C"

// Operator data of one precision
template <class T>
struct SigmaBufs {
  const T *Fd, *Fl, *fo, *fv, *fov;
  T *S, *side, *side_tr;
  int prec;
};

static SigmaBufs<double> bufs64(esmp2_handle h) {
  return SigmaBufs<double>{h->Fd, h->Fl, h->fo, h->fv, h->fov, h->S, h->side, h->side_tr, ESMP2_FP64};
}

static SigmaBufs<float> bufs32(esmp2_handle h) {
  return SigmaBufs<float>{h->Fd32, h->Fl32, h->fo32, h->fv32, h->fov32, h->S32, h->side32, h->side_tr32, ESMP2_FP32};
}

// y = A x in the precision of T, all on the handle's stream:
// S~ (flip-symmetrised S2) -> side contractions -> virtual-pair Sylvester
// products (y = ...) -> couplings (y += ...) -> occupied-index action (y += ...)
// S~ and the per-batch side contractions with f_ov; returns the argument
// block of the coupling terms.
template <class T>
struct PrologueArgs {
  GemvArgs<T> gv;
  GatherArgs<T> ga;
  int jobs;       // workgroups of the GEMV launch
};

// the argument blocks of the prologue's kernels and of the coupling terms
// (pointer arithmetic only; nothing is launched)
template <class T>
static PrologueArgs<T> prologue_args(esmp2_handle h, const SigmaBufs<T>& w, const T* x, T* y, bool arrow) {
  const Dims& d = h->d;
  const int no = d.no, nv = d.nv;
  SideArgs<T> sa{};
  sa.d = d; sa.x = x; sa.fov = w.fov;
  T* p = w.side;
  auto take = [&](int64_t rows) { T* r = p; p += rows * nv; return r; };
  sa.t3_t = take(d.npo1); sa.t3_p1 = take(d.npo1); sa.t3_p2 = take(d.npo1);
  sa.h11_p1 = take(d.npo); sa.h11_p2 = take(d.npo);
  sa.h12_t = take(d.npo); sa.h12_u1 = take(d.npo); sa.h12_u2 = take(d.npo);
  const int n2 = (no - 1) * (no - 1);
  sa.h21_t = take(n2); sa.h21_k = take(n2);
  sa.h22_ut = take(n2); sa.h22_i = take(n2); sa.h22_uk = take(n2);
  PrologueArgs<T> r{};
  // per-batch GEMVs: the side contractions, and with the arrow-shaped Fock blocks
  // also the t'-row products (T2 and S2 batches join the job list)
  r.gv = GemvArgs<T>{sa, w.S, w.fv, (T*)h->gv, w.side_tr, arrow ? 1 : 0};
  r.jobs = d.npo1 + 2 * d.npo + 2 * n2 + (arrow ? d.npo + no * no : 0);
  GatherArgs<T>& ga = r.ga;
  ga.d = d; ga.x = x; ga.S = w.S; ga.y = y; ga.fo = w.fo; ga.fv = w.fv; ga.fov = w.fov; ga.side_tr = w.side_tr;
  ga.t3_t = sa.t3_t; ga.t3_p1 = sa.t3_p1; ga.t3_p2 = sa.t3_p2; ga.h11_p1 = sa.h11_p1; ga.h11_p2 = sa.h11_p2;
  ga.h12_t = sa.h12_t; ga.h12_u1 = sa.h12_u1; ga.h12_u2 = sa.h12_u2; ga.h21_t = sa.h21_t; ga.h21_k = sa.h21_k;
  ga.h22_ut = sa.h22_ut; ga.h22_i = sa.h22_i; ga.h22_uk = sa.h22_uk;
  return r;
}

template <class T>
static GatherArgs<T> sigma_prologue(esmp2_handle h, const SigmaBufs<T>& w, const T* x, T* y, bool arrow = false) {
  const Dims& d = h->d;
  hipStream_t s = h->stream;
  hipLaunchKernelGGL(k_sym_s2<T>, dim3(sym_s2_blocks(d)), dim3(256), 0, s, d, x, w.S);
  const PrologueArgs<T> r = prologue_args(h, w, x, y, arrow);
  if (d.nv <= 160)
    hipLaunchKernelGGL((k_gemv<T, 160>), dim3(r.jobs), dim3(256), 0, s, r.gv);
  else
    hipLaunchKernelGGL((k_gemv<T, 192>), dim3(r.jobs), dim3(256), 0, s, r.gv);
  return r.ga;
}

// Sylvester-product variants: 0 = the specialised kernel (padded virtual
// dimension 80, 112 or 160; BF16 operands only there), 1..5 = the generic
// kernel with 32 TW x 32 TW output blocks per workgroup, TW = variant.
constexpr int VV_VARIANTS = 6;

static bool vv_specialised(const Dims& d) { return d.mv == 160 || d.mv == 112 || d.mv == 80; }

static bool vv_variant_ok(const Dims& d, int prec, int v) {
  if (prec == ESMP2_BF16) return v == 0 && vv_specialised(d);
  return v == 0 ? vv_specialised(d) : (v >= 1 && v < VV_VARIANTS);
}

// Choices of esmp2_autotune, shared by every handle of the process (key: n_occ, n_vir, precision)
static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int>, int> g_tune;

static int vv_variant(esmp2_handle h, int prec) {
  const Dims& d = h->d;
  if (h->vv_variant[prec] >= 0 && vv_variant_ok(d, prec, h->vv_variant[prec])) return h->vv_variant[prec];
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(std::make_tuple(d.no, d.nv, prec));
    if (it != g_tune.end() && vv_variant_ok(d, prec, it->second)) return it->second;
  }
  if (vv_specialised(d)) return 0;
  return std::min((d.mv / 16 + 1) / 2, 5);
}

template <class T>
static void launch_vv(esmp2_handle h, const VVArgs<T>& va, int prec, int variant, hipStream_t s) {
  const Dims& d = h->d;
  if (variant == 0) {
    if (prec == ESMP2_BF16) {
      if constexpr (std::is_same<T, float>::value) {
        if (d.mv == 160) hipLaunchKernelGGL((k_vv3b<10>), dim3(h->njobs4), dim3(V3_THREADS), 0, s, va);
        else if (d.mv == 112) hipLaunchKernelGGL((k_vv3b<7>), dim3(h->njobs4), dim3(V3_THREADS), 0, s, va);
        else hipLaunchKernelGGL((k_vv3b<5>), dim3(h->njobs4), dim3(V3_THREADS), 0, s, va);
      }
    } else if (d.mv == 160) {
      hipLaunchKernelGGL((k_vv3<T, 10>), dim3(h->njobs4), dim3(V3_THREADS), 0, s, va);
    } else if (d.mv == 112) {
      hipLaunchKernelGGL((k_vv3<T, 7>), dim3(h->njobs4), dim3(V3_THREADS), 0, s, va);
    } else {
      hipLaunchKernelGGL((k_vv3<T, 5>), dim3(h->njobs4), dim3(V3_THREADS), 0, s, va);
    }
    return;
  }
  const int nb = (d.mv + 32 * variant - 1) / (32 * variant);
  const dim3 grid(h->njobs, nb, nb);
  switch (variant) {
    case 1: hipLaunchKernelGGL((k_vv<T, 1>), grid, dim3(256), 0, s, va); break;
    case 2: hipLaunchKernelGGL((k_vv<T, 2>), grid, dim3(256), 0, s, va); break;
    case 3: hipLaunchKernelGGL((k_vv<T, 3>), grid, dim3(256), 0, s, va); break;
    case 4: hipLaunchKernelGGL((k_vv<T, 4>), grid, dim3(256), 0, s, va); break;
    default: hipLaunchKernelGGL((k_vv<T, 5>), grid, dim3(256), 0, s, va); break;
  }
}

template <class T>
static esmp2_status sigma_t(esmp2_handle h, const SigmaBufs<T>& w, const T* x, T* y) {
  const Dims& d = h->d;
  const int no = d.no, nv = d.nv;
  hipStream_t s = h->stream;
  GatherArgs<T> ga = sigma_prologue(h, w, x, y);
  // tile prefix sums per box for the occupied-index kernel
  const int inner[7] = {d.npv, nv * nv, d.npv1, d.npv, (nv - 1) * (nv - 1), d.npv, (nv - 1) * (nv - 1)};
  const int nbat[7] = {d.npo, no * no, d.npo1, d.npo, d.npo, (no - 1) * (no - 1), (no - 1) * (no - 1)};
  int maxb = 1;
  for (int k = 0; k < 7; ++k)
    if (nbat[k] > 0 && inner[k] > 0) maxb = std::max(maxb, nbat[k]);
  const size_t lds_oo = sizeof(T) * (size_t)2 * maxb * (GO + 1) + 256 * sizeof(int);
  // occupied-index action on the matrix cores when the occupied range fits one 16x16 tile
  const bool oo_mfma = no <= 16 && lds_oo <= 160 * 1024 - 2048;
  // virtual-pair Sylvester products (+ the diagonal constants folded into F')
  VVArgs<T> va{d, x, w.S, y, w.Fd, w.Fl, w.side_tr, h->jobs, h->jobs4};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (h->prof) {
    if (h->ev_vv.size() >= 4096) drain_events(h);
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
      (void)hipEventRecord(e0, s);
    } else {
      e0 = e1 = nullptr;
    }
  }
  launch_vv(h, va, w.prec, vv_variant(h, w.prec), s);
  if (e0) {
    (void)hipEventRecord(e1, s);
    h->ev_vv.push_back({e0, e1, w.prec});
  }
  const int* pv = h->pairs;
  PairTables pt{pv, pv + d.npv, pv + d.npv + d.npv1, pv + d.npv + d.npv1 + d.npo};
  if (h->nchunks > 0)
    hipLaunchKernelGGL(k_couple<T>, dim3(h->nchunks), dim3(256), 0, s, ga, pt, (const int4*)h->chunks);
  if (oo_mfma) {
    int pre[8] = {0};
    for (int k = 0; k < 7; ++k) {
      int nt = (nbat[k] > 0 && inner[k] > 0) ? (inner[k] + GO - 1) / GO : 0;
      pre[k + 1] = pre[k] + nt;
    }
    ESMP2_HIP(allow_device_lds((const void*)k_oo<T>));
    hipLaunchKernelGGL(k_oo<T>, dim3(pre[7]), dim3(256), lds_oo, s, ga, make_int4(pre[1], pre[2], pre[3], pre[4]),
                       make_int4(pre[5], pre[6], pre[7], 0));
  } else {
    hipLaunchKernelGGL(k_oo_plain<T>, dim3(nblk(d.off[7])), dim3(256), 0, s, ga);
  }
  ESMP2_HIP(hipGetLastError());
  return ESMP2_OK;
}

// sigma in the pinned-semicanonical basis, where the non-pinned Fock blocks
// are diagonal: O(N_o^2 N_v^2) arrow kernels instead of the Sylvester products
// pq != nullptr: also the per-workgroup parts of <x, y>_W (h->nchunks of them)
template <class T>
static esmp2_status sigma_arrow(esmp2_handle h, const SigmaBufs<T>& w, const T* x, T* y, double* pq = nullptr) {
  const Dims& d = h->d;
  const int no = d.no;
  hipStream_t s = h->stream;
  GatherArgs<T> ga = sigma_prologue(h, w, x, y, true);
  ArrowArgs<T> aa{ga, w.Fd, w.Fl, w.side_tr, (T*)h->gv};
  const int* pv = h->pairs;
  PairTables pt{pv, pv + d.npv, pv + d.npv + d.npv1, pv + d.npv + d.npv1 + d.npo};
  if (h->nchunks > 0)
    hipLaunchKernelGGL(k_arrow<T>, dim3(h->nchunks), dim3(256), 0, s, aa, pt, (const int4*)h->chunks, pq);
  ESMP2_HIP(hipGetLastError());
  return ESMP2_OK;
}

static esmp2_status sigma64(esmp2_handle h, const double* x, double* y) { return sigma_t(h, bufs64(h), x, y); }
static esmp2_status sigma32(esmp2_handle h, const float* x, float* y) { return sigma_t(h, bufs32(h), x, y); }
// the FP32 operator with BF16 operands in the Sylvester products
static SigmaBufs<float> bufs_bf16(esmp2_handle h) {
  SigmaBufs<float> w = bufs32(h);
  w.prec = ESMP2_BF16;
  return w;
}
// padded virtual dimensions with a BF16 Sylvester kernel
static bool bf16_supported(const Dims& d) { return d.mv == 160 || d.mv == 112 || d.mv == 80; }

// ---------------------------------------------------------------------------
// pinned-semicanonical basis
// ---------------------------------------------------------------------------
// Contract index `which` (0: P, 1: Q, 2: A, 3: B) of dense[P][Q][A][B]
// (ranges ro, ro, rv, rv) with G: out[..c'..] = sum_c G(c, c') in[..c..],
// G(c, c') = Gm[c*sr + c'*sc].
static hipError_t contract_index(hipStream_t s, int which, int ro, int rv, const double* Gm, int64_t sr,
                                 int64_t sc, const double* in, double* out) {
  GemmArgs g{};
  g.alpha = 1; g.beta = 0;
  const int64_t v2 = (int64_t)rv * rv;
  if (which == 3) {                 // out[R][B'] = sum_B in[R][B] G(B, B')
    g.A = in; g.B = Gm; g.C = out; g.M = ro * ro * rv; g.N = rv; g.K = rv;
    g.sAi = rv; g.sAk = 1; g.sBk = sr; g.sBj = sc; g.sCi = rv; g.sCj = 1;
    return gemm(s, 1, g);
  }
  if (which == 2) {                 // out[PQ][A'][B] = sum_A G(A, A') in[PQ][A][B]
    g.A = Gm; g.B = in; g.C = out; g.M = rv; g.N = rv; g.K = rv;
    g.sAb = 0; g.sAi = sc; g.sAk = sr; g.sBb = v2; g.sBk = rv; g.sBj = 1; g.sCb = v2; g.sCi = rv; g.sCj = 1;
    return gemm(s, ro * ro, g);
  }
  if (which == 0) {                 // out[P'][rest] = sum_P G(P, P') in[P][rest]
    g.A = Gm; g.B = in; g.C = out; g.M = ro; g.N = (int)(ro * v2); g.K = ro;
    g.sAi = sc; g.sAk = sr; g.sBk = ro * v2; g.sBj = 1; g.sCi = ro * v2; g.sCj = 1;
    return gemm(s, 1, g);
  }
  // out[P][Q'][AB] = sum_Q G(Q, Q') in[P][Q][AB]
  g.A = Gm; g.B = in; g.C = out; g.M = ro; g.N = (int)v2; g.K = ro;
  g.sAb = 0; g.sAi = sc; g.sAk = sr; g.sBb = ro * v2; g.sBk = v2; g.sBj = 1; g.sCb = ro * v2; g.sCi = v2; g.sCj = 1;
  return gemm(s, ro, g);
}

// y = rotation of the amplitude vector x: forward (TOP basis -> pinned
// semicanonical basis) contracts every free index with the rotation block,
// G = T; backward with its transpose.  x and y must not overlap.
static esmp2_status rotate_amplitudes(esmp2_handle h, const double* x, double* y, bool forward) {
  const Dims& d = h->d;
  hipStream_t s = h->stream;
  for (int box = 0; box < 7; ++box) {
    if (d.off[box + 1] == d.off[box]) continue;
    int lo_o, lo_v;
    box_ranges(box, lo_o, lo_v);
    const int ro = d.no - lo_o, rv = d.nv - lo_v;
    const double* Go = h->To + lo_o * d.no + lo_o;
    const double* Gv = h->Tv + lo_v * d.nv + lo_v;
    const int64_t sro = forward ? d.no : 1, sco = forward ? 1 : d.no;
    const int64_t srv = forward ? d.nv : 1, scv = forward ? 1 : d.nv;
    const int64_t nd = (int64_t)ro * ro * rv * rv;
    // S2 and H2P2 are stored dense in exactly the [P][Q][A][B] order: read from
    // x and written to y in place of the unpack and pack passes
    const bool dense_box = box == B_S2 || box == B_H22;
    if (!dense_box) hipLaunchKernelGGL(k_unpack_box, dim3(nblk(nd)), dim3(256), 0, s, d, box, x, h->dense0);
    ESMP2_HIP(contract_index(s, 3, ro, rv, Gv, srv, scv, dense_box ? x + d.off[box] : h->dense0, h->dense1));
    ESMP2_HIP(contract_index(s, 2, ro, rv, Gv, srv, scv, h->dense1, h->dense0));
    const int64_t v2 = (int64_t)rv * rv;
    dim3 grid_o((unsigned)((v2 + 255) / 256), (unsigned)ro);
    auto rot_occ = [&](const double* in, double* out, int which) {
      if (ro <= 16)
        hipLaunchKernelGGL(k_rot_occ<16>, grid_o, dim3(256), 0, s, in, out, Go, sro, sco, ro, v2, which);
      else if (ro <= 32)
        hipLaunchKernelGGL(k_rot_occ<32>, grid_o, dim3(256), 0, s, in, out, Go, sro, sco, ro, v2, which);
      else
        hipLaunchKernelGGL(k_rot_occ<64>, grid_o, dim3(256), 0, s, in, out, Go, sro, sco, ro, v2, which);
    };
    rot_occ(h->dense0, h->dense1, 0);
    rot_occ(h->dense1, dense_box ? y + d.off[box] : h->dense0, 1);
    if (!dense_box)
      hipLaunchKernelGGL(k_pack_box, dim3(nblk(d.off[box + 1] - d.off[box])), dim3(256), 0, s, d, box,
                         (const double*)h->dense0, y);
  }
  ESMP2_HIP(hipGetLastError());
  return ESMP2_OK;
}

// Rotation diagonalising F~_oo[1:,1:] and F~_vv[1:,1:], the operator blocks in
// the new basis (TOP-basis omega and kappa) and its Jacobi diagonal (unless the
// right-hand side kernel that follows forms it: diag = false).  Requires the
// rotation to the TOP basis.
static esmp2_status semican_operator(esmp2_handle h, bool diag = true) {
  const Dims& d = h->d;
  const int no = d.no, nv = d.nv, n = d.n, mv = d.mv;
  const int64_t namp = d.off[7];
  hipStream_t s = h->stream;
  // the rotation's eigenproblems, queued on the side stream by esmp2_rotate_top
  if (h->sc_pending) {
    ESMP2_HIP(hipStreamWaitEvent(s, h->ev_sc_eig, 0));
    h->sc_pending = false;
    h->sc_eig = true;
  }
  if (!h->sc_eig) return fail(h, ESMP2_BAD_ORDER, "esmp2_rotate_top first");
  // Fh = T^T F~ T
  hipLaunchKernelGGL(k_blkdiag, dim3(nblk((int64_t)n * n)), dim3(256), 0, s, (const double*)h->To,
                     (const double*)h->Tv, no, nv, h->Tsc);
  GemmArgs g{};
  g.A = h->Ft; g.B = h->Tsc; g.C = h->T; g.M = n; g.N = n; g.K = n;
  g.sAi = n; g.sAk = 1; g.sBk = n; g.sBj = 1; g.sCi = n; g.sCj = 1; g.alpha = 1; g.beta = 0;
  ESMP2_HIP(gemm(s, 1, g));
  g = GemmArgs{};
  g.A = h->Tsc; g.B = h->T; g.C = h->Fh; g.M = n; g.N = n; g.K = n;
  g.sAi = 1; g.sAk = n; g.sBk = n; g.sBj = 1; g.sCi = n; g.sCj = 1; g.alpha = 1; g.beta = 0;
  ESMP2_HIP(gemm(s, 1, g));
  hipLaunchKernelGGL(k_fock_blocks, dim3(nblk((int64_t)mv * mv > n * n ? (int64_t)mv * mv : (int64_t)n * n)),
                     dim3(256), 0, s, (const double*)h->Fh, no, nv, mv, h->omega, h->kappa, h->fo_sc, h->fv_sc,
                     h->fov_sc, h->eo_sc, h->ev_sc, h->Fd_sc, h->Fl_sc);
  {
    const ToF32Set t{{h->Fd_sc, h->Fl_sc, h->fo_sc, h->fv_sc, h->fov_sc},
                     {h->Fd32_sc, h->Fl32_sc, h->fo32_sc, h->fv32_sc, h->fov32_sc},
                     {(int64_t)mv * mv, (int64_t)mv * mv, (int64_t)no * no, (int64_t)nv * nv, (int64_t)no * nv}};
    hipLaunchKernelGGL(k_to_f32_set, dim3(nblk((int64_t)mv * mv)), dim3(256), 0, s, t);
  }
  if (diag) {
    DiagArgs da{d, h->eo_sc, h->ev_sc, h->omega, h->dinv32_sc, h->blockmin};
    launch_diag(h, da);
  }
  ESMP2_HIP(hipGetLastError());
  h->have_sc_op = true;
  return ESMP2_OK;
}

// Y[q] = To^T X[q] Tv for nq stacked no x nv matrices (a tensor in (i, a)
// taken into the pinned-semicanonical basis); Y[q] starts at Y + q * ldy;
// tmp holds nq * no * nv.
static hipError_t rotate_ov(esmp2_handle h, int nq, const double* X, double* tmp, double* Y, int64_t ldy) {
  const int no = h->d.no, nv = h->d.nv;
  GemmArgs g{};
  g.alpha = 1; g.beta = 0;
  // tmp[(q,i)][A] = sum_a X[(q,i)][a] Tv[a][A]
  g.A = X; g.B = h->Tv; g.C = tmp; g.M = nq * no; g.N = nv; g.K = nv;
  g.sAi = nv; g.sAk = 1; g.sBk = nv; g.sBj = 1; g.sCi = nv; g.sCj = 1;
  hipError_t e = gemm(h->stream, 1, g);
  if (e != hipSuccess) return e;
  // Y[q][I][A] = sum_i To[i][I] tmp[q][i][A]
  g = GemmArgs{};
  g.alpha = 1; g.beta = 0;
  g.A = h->To; g.B = tmp; g.C = Y; g.M = no; g.N = nv; g.K = no;
  g.sAb = 0; g.sAi = 1; g.sAk = no; g.sBb = (int64_t)no * nv; g.sBk = nv; g.sBj = 1;
  g.sCb = ldy; g.sCi = nv; g.sCj = 1;
  return gemm(h->stream, nq, g);
}

// The right-hand side built in the pinned-semicanonical basis instead of
// rotating the TOP-basis one (a four-index rotation of every box): V, M and
// f^Phi are tensors in their (i, a) index pairs, so the three-index factors
// Bov and X and f^Phi are rotated (To^T . Tv) and V, M rebuilt from them; the
// singles amplitudes of Psi0, diagonal in the TOP basis, become the matrix
// C = To^T diag(c) Tv.  Requires the TOP-basis right-hand side's Bov, X and
// f^Phi (esmp2_build_rhs) and the rotation (semican_operator).  V and M go to
// the dense scratch buffers (n_occ^2 n_vir^2 each): the TOP-basis V stays for
// E2_S on the side stream.
// With init, the kernel of b also forms the Jacobi diagonal and starts the FP64
// conjugate gradient from x = 0 (p and the parts of its two dots, for solve64).
static esmp2_status rhs_semican(esmp2_handle h, bool init) {
  const Dims& d = h->d;
  const int no = d.no, nv = d.nv, na = d.naux, nov = no * nv;
  hipStream_t s = h->stream;
  double* Cs = h->rsc;
  double* fphi = Cs + nov;
  double* W = fphi + nov;                       // [Bov; X] rotated: 2 na nov
  double* tmp = W + 2 * (size_t)na * nov;       // 2 na nov
  hipLaunchKernelGGL(k_singles_sc, dim3(nblk(nov)), dim3(256), 0, s, (const double*)h->To, (const double*)h->Tv,
                     (const double*)h->lam, no, nv, Cs);
  ESMP2_HIP(rotate_ov(h, 1, h->fphi, tmp, fphi, nov));
  // X = Bov + na nov: both factors rotated as one stack of 2 na matrices
  ESMP2_HIP(rotate_ov(h, 2 * na, h->Bov, tmp, W, nov));
  // [V; M] = [Bov | X]^T Bov, two products in one call: V into dense0, M into dense1 = dense0 + nov^2
  GemmArgs g{};
  g.A = W; g.B = W; g.C = h->dense0; g.M = nov; g.N = nov; g.K = na;
  g.sAb = (int64_t)na * nov; g.sAi = 1; g.sAk = nov; g.sBb = 0; g.sBk = nov; g.sBj = 1;
  g.sCb = (int64_t)nov * nov; g.sCi = nov; g.sCj = 1;
  g.alpha = 1; g.beta = 0;
  ESMP2_HIP(gemm(s, 2, g));
  RhsArgs ra{d, h->dense0, h->dense1, fphi, h->lam, h->b_sc, Cs};
  const bool fused = init && h->ntop == 1 && h->nchunks > 0;     // the chunk kernel
  if (fused) {
    ra.dinv = h->dinv32_sc; ra.p = h->p; ra.part = h->pq_part;
    ra.eo = h->eo_sc; ra.ev = h->ev_sc; ra.omega = h->omega;
  }
  launch_rhs<true>(h, ra, s);
  h->sc_init_ready = fused;
  ESMP2_HIP(hipGetLastError());
  return ESMP2_OK;
}

// The operator of the pinned-semicanonical basis (if not built yet) and the
// right-hand side in it.  Requires the right-hand side.
static esmp2_status semican_setup(esmp2_handle h, bool init = false) {
  if (!h->have_sc_op) {
    // the right-hand side kernel forms the diagonal where it also starts the solve
    const esmp2_status st = semican_operator(h, !(init && h->ntop == 1 && h->nchunks > 0));
    if (st != ESMP2_OK) return st;
  }
  const esmp2_status st = rhs_semican(h, init);
  if (st != ESMP2_OK) return st;
  ESMP2_HIP(hipGetLastError());
  h->have_sc = true;
  return ESMP2_OK;
}

// Everything a solve needs in one basis
struct OpCtx {
  const double* b;
  const float* dinv32;
  SigmaBufs<double> s64;
  SigmaBufs<float> s32;
  bool rotated;      // pinned-semicanonical basis: x_out is rotated back
  bool arrow;        // the operator through the arrow kernels
};

// y = A x of ESMP2-TOP(k), k > 1 (FP64 or FP32 vectors)
template <class T>
static esmp2_status sigma_topk(esmp2_handle h, const T* x, T* y) {
  const TopkArgs ta = topk_args(h);
  hipLaunchKernelGGL(k_topk_sigma<T>, dim3(nblk(h->namp)), dim3(256), 0, h->stream, ta, x, y);
  ESMP2_HIP(hipGetLastError());
  return ESMP2_OK;
}

template <class T>
static esmp2_status apply_op(esmp2_handle h, const OpCtx& c, const SigmaBufs<T>& w, const T* x, T* y) {
  if (h->ntop > 1) return sigma_topk(h, x, y);
  return c.arrow ? sigma_arrow(h, w, x, y) : sigma_t(h, w, x, y);
}

template <class T>
static void wdot(esmp2_handle h, const T* x, const T* y, int slot);

// y = A x and sc[SC_PQ] = <x, y>_W (fused into the operator where it writes every element once)
template <class T>
static esmp2_status apply_op_dot(esmp2_handle h, const OpCtx& c, const SigmaBufs<T>& w, const T* x, T* y) {
  if (h->ntop > 1) {
    const esmp2_status st = sigma_topk(h, x, y);
    if (st != ESMP2_OK) return st;
    wdot(h, x, (const T*)y, SC_PQ);
    return ESMP2_OK;
  }
  if (c.arrow && h->nchunks > 0) {
    esmp2_status st = sigma_arrow(h, w, x, y, h->pq_part);
    if (st != ESMP2_OK) return st;
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, h->stream, (const double*)h->pq_part, h->nchunks, h->sc,
                       (int)SC_PQ);
    return ESMP2_OK;
  }
  esmp2_status st = sigma_t(h, w, x, y);
  if (st != ESMP2_OK) return st;
  wdot(h, x, (const T*)y, SC_PQ);
  return ESMP2_OK;
}

static OpCtx ctx_top(esmp2_handle h) { return OpCtx{h->b, h->dinv32, bufs64(h), bufs32(h), false, false}; }

static OpCtx ctx_sc(esmp2_handle h) {
  OpCtx c{h->b_sc, h->dinv32_sc, bufs64(h), bufs32(h), true, true};
  c.s64.Fd = h->Fd_sc; c.s64.Fl = h->Fl_sc; c.s64.fo = h->fo_sc; c.s64.fv = h->fv_sc; c.s64.fov = h->fov_sc;
  c.s32.Fd = h->Fd32_sc; c.s32.Fl = h->Fl32_sc; c.s32.fo = h->fo32_sc; c.s32.fv = h->fv32_sc;
  c.s32.fov = h->fov32_sc;
  return c;
}

extern "C" {

esmp2_status esmp2_sigma(esmp2_handle h, const void* x, void* y, int precision) {
  if (!h) return ESMP2_INVALID_ARG;
  if (h->state < 2) return fail(h, ESMP2_BAD_ORDER, "esmp2_rotate_top first");
  if (!x || !y) return fail(h, ESMP2_INVALID_ARG, "null vector");
  if (x == y) return fail(h, ESMP2_INVALID_ARG, "x and y must not overlap");
  ESMP2_HIP(hipSetDevice(h->device));
  if (h->ntop > 1) {
    if (precision == ESMP2_FP64) return sigma_topk(h, (const double*)x, (double*)y);
    if (precision == ESMP2_FP32) return sigma_topk(h, (const float*)x, (float*)y);
    return fail(h, ESMP2_UNSUPPORTED, "more than one large TOP: FP64 or FP32");
  }
  if (precision == ESMP2_FP64) return sigma64(h, (const double*)x, (double*)y);
  if (precision == ESMP2_FP32) return sigma32(h, (const float*)x, (float*)y);
  if (precision == ESMP2_BF16) {
    if (!bf16_supported(h->d))
      return fail(h, ESMP2_UNSUPPORTED, "BF16 Sylvester products need a padded virtual dimension of 80, 112 or 160");
    return sigma_t(h, bufs_bf16(h), (const float*)x, (float*)y);
  }
  return fail(h, ESMP2_INVALID_ARG, "unknown precision");
}

esmp2_status esmp2_sigma_basis(esmp2_handle h, const void* x, void* y, int precision, int basis) {
  if (!h) return ESMP2_INVALID_ARG;
  if (basis == ESMP2_BASIS_TOP) return esmp2_sigma(h, x, y, precision);
  if (basis != ESMP2_BASIS_SEMICANONICAL) return fail(h, ESMP2_INVALID_ARG, "unknown basis");
  if (h->state < 2) return fail(h, ESMP2_BAD_ORDER, "esmp2_rotate_top first");
  if (!x || !y) return fail(h, ESMP2_INVALID_ARG, "null vector");
  if (x == y) return fail(h, ESMP2_INVALID_ARG, "x and y must not overlap");
  if (h->ntop > 1) return fail(h, ESMP2_UNSUPPORTED, "more than one large TOP: TOP basis only");
  if (precision != ESMP2_FP64 && precision != ESMP2_FP32) {
    if (precision == ESMP2_BF16)
      return fail(h, ESMP2_UNSUPPORTED, "the pinned-semicanonical operator has no Sylvester products (no BF16 form)");
    return fail(h, ESMP2_INVALID_ARG, "unknown precision");
  }
  ESMP2_HIP(hipSetDevice(h->device));
  if (!h->have_sc_op) {
    const esmp2_status st = semican_operator(h);
    if (st != ESMP2_OK) return st;
  }
  const OpCtx c = ctx_sc(h);
  if (precision == ESMP2_FP64) return sigma_arrow(h, c.s64, (const double*)x, (double*)y);
  return sigma_arrow(h, c.s32, (const float*)x, (float*)y);
}

esmp2_status esmp2_export_determinants(esmp2_handle h, const double* x, double* coeff, int64_t* det_key,
                                       int64_t n) {
  if (!h) return ESMP2_INVALID_ARG;
  if (h->state < 1) return fail(h, ESMP2_BAD_ORDER, "esmp2_set_problem first");
  const Dims& d = h->d;
  const int64_t namp = h->namp, ndet = 2 * namp - (d.off[B_S2 + 1] - d.off[B_S2]);
  if (!x || !coeff || !det_key) return fail(h, ESMP2_INVALID_ARG, "null pointer");
  if (n < ndet) return fail(h, ESMP2_INVALID_ARG, "output arrays shorter than 2 n_amp - n_S2 determinants");
  ESMP2_HIP(hipSetDevice(h->device));
  if (h->ntop > 1) {
    const TopkArgs ta = topk_args(h);
    hipLaunchKernelGGL(k_topk_export, dim3(nblk(namp)), dim3(256), 0, h->stream, ta, x, coeff, det_key);
  } else {
    hipLaunchKernelGGL(k_export_dets, dim3(nblk(namp)), dim3(256), 0, h->stream, d, x, coeff, det_key);
  }
  ESMP2_HIP(hipGetLastError());
  return ESMP2_OK;
}

esmp2_status esmp2_set_sylvester_variant(esmp2_handle h, int precision, int variant) {
  if (!h) return ESMP2_INVALID_ARG;
  if (precision < ESMP2_FP64 || precision > ESMP2_BF16) return fail(h, ESMP2_INVALID_ARG, "unknown precision");
  if (h->state < 1) return fail(h, ESMP2_BAD_ORDER, "esmp2_set_problem first");
  if (variant != -1 && !vv_variant_ok(h->d, precision, variant))
    return fail(h, ESMP2_INVALID_ARG, "Sylvester variant not available for this size and precision");
  h->vv_variant[precision] = variant;
  return ESMP2_OK;
}

esmp2_status esmp2_autotune(esmp2_handle h, int precision, int reps, int* variant_out, double* ms_out) {
  if (!h) return ESMP2_INVALID_ARG;
  if (precision < ESMP2_FP64 || precision > ESMP2_BF16) return fail(h, ESMP2_INVALID_ARG, "unknown precision");
  if (reps < 1 || reps > 1000) return fail(h, ESMP2_INVALID_ARG, "reps must lie in [1, 1000]");
  if (h->state < 2) return fail(h, ESMP2_BAD_ORDER, "esmp2_rotate_top first");
  if (precision == ESMP2_BF16 && !vv_specialised(h->d))
    return fail(h, ESMP2_UNSUPPORTED, "BF16 Sylvester products need a padded virtual dimension of 80, 112 or 160");
  ESMP2_HIP(hipSetDevice(h->device));
  hipStream_t s = h->stream;
  const int64_t n = h->d.off[7];
  double ms[VV_VARIANTS];
  hipEvent_t a = nullptr, b = nullptr;
  ESMP2_HIP(hipEventCreate(&a));
  ESMP2_HIP(hipEventCreate(&b));
  auto time_all = [&](auto w, auto* x, auto* y) -> esmp2_status {
    ESMP2_HIP(hipMemsetAsync(x, 0, sizeof(*x) * n, s));
    VVArgs<typename std::remove_pointer<decltype(x)>::type> va{h->d, x, w.S, y, w.Fd, w.Fl, w.side_tr, h->jobs,
                                                                 h->jobs4};
    (void)sigma_prologue(h, w, x, y);       // the flip-symmetrised S2 block the kernels read
    for (int v = 0; v < VV_VARIANTS; ++v) {
      ms[v] = -1.0;
      if (!vv_variant_ok(h->d, precision, v)) continue;
      launch_vv(h, va, precision, v, s);
      ESMP2_HIP(hipEventRecord(a, s));
      for (int r = 0; r < reps; ++r) launch_vv(h, va, precision, v, s);
      ESMP2_HIP(hipEventRecord(b, s));
      ESMP2_HIP(hipEventSynchronize(b));
      float t = 0.f;
      ESMP2_HIP(hipEventElapsedTime(&t, a, b));
      ms[v] = t / reps;
    }
    return ESMP2_OK;
  };
  esmp2_status st;
  if (precision == ESMP2_FP64) st = time_all(bufs64(h), h->p, h->q);
  else if (precision == ESMP2_FP32) st = time_all(bufs32(h), h->p32, h->q32);
  else st = time_all(bufs_bf16(h), h->p32, h->q32);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (st != ESMP2_OK) return st;
  int best = -1;
  for (int v = 0; v < VV_VARIANTS; ++v)
    if (ms[v] >= 0 && (best < 0 || ms[v] < ms[best])) best = v;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[std::make_tuple(h->d.no, h->d.nv, precision)] = best;
  }
  h->vv_variant[precision] = -1;
  if (variant_out) *variant_out = best;
  if (ms_out)
    for (int v = 0; v < VV_VARIANTS; ++v) ms_out[v] = ms[v];
  return ESMP2_OK;
}

}  // extern "C"

// weighted dot product into h->sc[slot] (stream ordered)
template <class T>
static void wdot(esmp2_handle h, const T* x, const T* y, int slot) {
  const Dims& d = h->d;
  hipLaunchKernelGGL(k_dot<T>, dim3(PCG_BLOCKS), dim3(256), 0, h->stream, x, y, h->namp, d.off[1], d.off[2],
                     h->partial);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, h->stream, h->partial, PCG_BLOCKS, h->sc, slot);
}

extern "C" {

// E2 (Hylleraas form <b,x>_W - <x,r>_W, r = -b - A x) and the result record
static esmp2_status finish_solve(esmp2_handle h, const OpCtx& c, const esmp2_solve_opts* opts,
                                 esmp2_solve_result* res, double rel, int it, int outer, esmp2_status status,
                                 bool dots_ready = false) {
  const int64_t n = h->namp;
  hipStream_t s = h->stream;
  {
    const esmp2_status st = join_e2s(h, true);
    if (st != ESMP2_OK) return st;
  }
  const double* hs = h->pin->sc;
  if (!dots_ready) {
    wdot(h, c.b, (const double*)h->x, SC_BX);
    wdot(h, (const double*)h->x, (const double*)h->r, SC_XR);
  }
  ESMP2_HIP(hipMemcpyAsync(h->pin->sc, h->sc, sizeof(double) * SC_N, hipMemcpyDeviceToHost, s));
  if (opts->x_out) {
    if (c.rotated) {
      esmp2_status st = rotate_amplitudes(h, h->x, opts->x_out, false);
      if (st != ESMP2_OK) return st;
    } else {
      ESMP2_HIP(hipMemcpyAsync(opts->x_out, h->x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    }
  }
  ESMP2_HIP(hipStreamSynchronize(s));
  ESMP2_HIP(hipGetLastError());
  res->e2_dl = hs[SC_BX] - hs[SC_XR];
  res->e2_s = h->e2s;
  res->e2 = res->e2_dl + res->e2_s;
  res->e0 = h->e0;
  res->rel_resid = rel;
  res->iterations = it;
  res->outer = outer;
  res->status = status;
  return status;
}

// The FP64 iterations of solve64 in the pinned-semicanonical basis with the
// stop decided on the device (cgdev.hip): iteration i + 1 is queued before the
// host reads the control word of iteration i.  Starts from the state k_init
// (or the fused start of the right-hand side kernel) left: x = x0 or 0, r, p,
// rho, and <r, r>_W in sc; ||b||_W^2 is in sc[SC_BB] for a start from x0.
// rel0: the host's relative residual of the start, or (rel_on_device) the
// device computes it and may stop before the first iteration.
static esmp2_status solve64_dev(esmp2_handle h, const OpCtx& c, const esmp2_solve_opts* opts,
                                esmp2_solve_result* res, double rel0, bool rel_on_device) {
  const Dims& d = h->d;
  const int64_t n = h->namp;
  hipStream_t s = h->stream;
  const unsigned NB = PCG_BLOCKS;
  CgCtl* ctl = (CgCtl*)h->cgctl;
  const SigmaBufs<double>& w = c.s64;
  const PrologueArgs<double> pa = prologue_args(h, w, (const double*)h->p, h->q, true);
  const ArrowArgs<double> aa{pa.ga, w.Fd, w.Fl, w.side_tr, h->gv};
  const int* pv = h->pairs;
  const PairTables pt{pv, pv + d.npv, pv + d.npv + d.npv1, pv + d.npv + d.npv1 + d.npo};
  // a solve from x = 0 leaves r and x unwritten at the start: the first iteration reads -b for r
  const int from_zero = opts->x0 ? 0 : 1;
  // from x = 0 without x_out no x is kept: E2_DL from the iterates' scalars (cgdev.hip)
  const int no_x = (from_zero && !opts->x_out) ? 1 : 0;
  hipLaunchKernelGGL(kd_ctl_init, dim3(1), dim3(64), 0, s, ctl, h->sc, from_zero, opts->tol, rel0,
                     rel_on_device ? 1 : 0);
  auto enqueue = [&](int slot, int first) -> esmp2_status {
    hipLaunchKernelGGL(kd_sym, dim3(sym_s2_blocks(d)), dim3(256), 0, s, d, (const double*)h->p, w.S,
                       (const CgCtl*)ctl);
    if (d.nv <= 160)
      hipLaunchKernelGGL(kd_gemv<160>, dim3(pa.jobs), dim3(256), 0, s, pa.gv, (const CgCtl*)ctl);
    else
      hipLaunchKernelGGL(kd_gemv<192>, dim3(pa.jobs), dim3(256), 0, s, pa.gv, (const CgCtl*)ctl);
    hipLaunchKernelGGL(kd_arrow, dim3(h->nchunks), dim3(256), 0, s, aa, pt, (const int4*)h->chunks, h->pq_part,
                       (const CgCtl*)ctl);
    hipLaunchKernelGGL(kd_finish_pq, dim3(PQ_PARTS), dim3(1024), 0, s, (const double*)h->pq_part, h->nchunks, h->sc,
                       ctl);
    hipLaunchKernelGGL(kd_update_r, dim3(NB), dim3(256), 0, s, h->r, (const double*)h->q, c.dinv32, n, d.off[1],
                       d.off[2], (const double*)h->sc, h->partial, h->sc, (const CgCtl*)ctl, c.b, first, no_x);
    hipLaunchKernelGGL(kd_finish_r, dim3(2), dim3(1024), 0, s, (const double*)h->partial, (int)NB, h->sc, ctl,
                       opts->tol, opts->max_iter);
    ESMP2_HIP(hipMemcpyAsync(&h->pin->cg[slot], ctl, sizeof(CgCtl), hipMemcpyDeviceToHost, s));
    ESMP2_HIP(hipEventRecord(h->ev_cg[slot], s));
    hipLaunchKernelGGL(kd_update_px, dim3(NB), dim3(256), 0, s, h->x, h->p, (const double*)h->r, c.b, c.dinv32, n,
                       d.off[1], d.off[2], (const double*)h->sc, h->partial, (const CgCtl*)ctl, first, no_x);
    ESMP2_HIP(hipGetLastError());
    return ESMP2_OK;
  };
  ESMP2_TRY(enqueue(0, from_zero));
  int queued = 1;
  CgCtl last{};
  for (int i = 0;; ++i) {
    if (queued < opts->max_iter) {            // the next iteration before this one's outcome
      ESMP2_TRY(enqueue(queued & 1, 0));
      ++queued;
    }
    ESMP2_HIP(hipEventSynchronize(h->ev_cg[i & 1]));
    last = h->pin->cg[i & 1];
    if (last.status != ESMP2_NOT_SPD && opts->resid_hist && last.it >= 1) opts->resid_hist[last.it - 1] = last.rel;
    if (last.mode != CG_RUN || i + 1 >= queued) break;
  }
  esmp2_status status = (esmp2_status)last.status;
  if (last.mode == CG_RUN) {                  // not reached: the device stops at max_iter
    status = ESMP2_NOT_CONVERGED;
  }
  if (no_x) {    // sc[SC_BX] holds the sum over the iterations (0 before the first), sc[SC_XR] = 0
    if (status == ESMP2_NOT_SPD) h->err = "p.Ap <= 0 in conjugate gradient";
    else if (status == ESMP2_NOT_CONVERGED) h->err = "max_iter reached";
    return finish_solve(h, c, opts, res, last.rel, last.it, 0, status, true);
  }
  if (status == ESMP2_NOT_SPD) {
    h->err = "p.Ap <= 0 in conjugate gradient";
    if (from_zero && last.it == 0)    // stopped before the first update: x = 0, r = -b
      hipLaunchKernelGGL(k_init, dim3(NB), dim3(256), 0, s, c.b, (const double*)nullptr, h->r, h->p, c.dinv32, n,
                         d.off[1], d.off[2], h->partial, h->x);
    return finish_solve(h, c, opts, res, last.rel, last.it, 0, status);
  }
  if (last.it == 0) {                 // stopped at the start (b = 0): x = 0, r = -b
    if (from_zero)
      hipLaunchKernelGGL(k_init, dim3(NB), dim3(256), 0, s, c.b, (const double*)nullptr, h->r, h->p, c.dinv32, n,
                         d.off[1], d.off[2], h->partial, h->x);
    return finish_solve(h, c, opts, res, last.rel, 0, 0, status);
  }
  if (status == ESMP2_NOT_CONVERGED) h->err = "max_iter reached";
  // the Hylleraas dots from the parts of the last update
  hipLaunchKernelGGL(k_finish, dim3(2), dim3(1024), 0, s, (const double*)h->partial, (int)NB, h->sc, (int)SC_BX);
  return finish_solve(h, c, opts, res, last.rel, last.it, 0, status, true);
}

// Jacobi-preconditioned conjugate gradient in FP64 for A x = -b
static esmp2_status solve64(esmp2_handle h, const OpCtx& c, const esmp2_solve_opts* opts,
                            esmp2_solve_result* res) {
  const Dims& d = h->d;
  const int64_t n = h->namp;
  hipStream_t s = h->stream;
  const unsigned NB = PCG_BLOCKS;
  // the device-stopped iterations (pinned-semicanonical basis): from x = 0 the
  // start stores neither r nor x (the first iteration reads -b for r)
  const bool dev = c.arrow && h->nchunks > 0 && h->ntop == 1 && opts->max_iter > 0;
  const bool lazy = dev && !opts->x0;
  // the right-hand side kernel has started this solve (p, the parts of its two
  // dots); from x = 0 the relative residual is 1 (b != 0): no host read needed
  const bool fused = lazy && c.rotated && h->sc_init_ready && opts->tol < 1.0;
  h->sc_init_ready = false;
  if (fused) {
    hipLaunchKernelGGL(k_finish, dim3(2), dim3(1024), 0, s, (const double*)h->pq_part, h->nchunks, h->sc, SC_RHO);
    return solve64_dev(h, c, opts, res, 0.0, true);
  }
  if (opts->x0) {
    wdot(h, c.b, c.b, SC_BB);   // ||b||_W^2
    if (c.rotated) {
      esmp2_status st0 = rotate_amplitudes(h, opts->x0, h->x, true);
      if (st0 != ESMP2_OK) return st0;
    } else {
      ESMP2_HIP(hipMemcpyAsync(h->x, opts->x0, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    }
    esmp2_status st = apply_op(h, c, c.s64, (const double*)h->x, h->q);
    if (st != ESMP2_OK) return st;
    hipLaunchKernelGGL(k_init, dim3(NB), dim3(256), 0, s, c.b, h->q, h->r, h->p, c.dinv32, n, d.off[1], d.off[2],
                       h->partial, (double*)nullptr);
  } else {
    // x = 0 in the same pass; r = -b exactly, so <r, r>_W is ||b||_W^2
    hipLaunchKernelGGL(k_init, dim3(NB), dim3(256), 0, s, c.b, (const double*)nullptr, lazy ? nullptr : h->r, h->p,
                       c.dinv32, n, d.off[1], d.off[2], h->partial, lazy ? nullptr : h->x);
  }
  // rho = <r, D^-1 r> into SC_RHO and <r, r> into SC_RHO + 1 = SC_PQ
  hipLaunchKernelGGL(k_finish, dim3(2), dim3(1024), 0, s, h->partial, (int)NB, h->sc, SC_RHO);
  double* hs = h->pin->sc;
  ESMP2_HIP(hipMemcpyAsync(h->pin->sc, h->sc, sizeof(double) * SC_N, hipMemcpyDeviceToHost, s));
  ESMP2_HIP(hipStreamSynchronize(s));
  const double bn = sqrt(opts->x0 ? hs[SC_BB] : hs[SC_PQ]);
  double rel = sqrt(hs[SC_PQ]) / bn;
  if (dev && rel > opts->tol) return solve64_dev(h, c, opts, res, rel, false);
  if (lazy)      // converged at the start: x = 0 and r = -b for the Hylleraas dots
    hipLaunchKernelGGL(k_init, dim3(NB), dim3(256), 0, s, c.b, (const double*)nullptr, h->r, h->p, c.dinv32, n,
                       d.off[1], d.off[2], h->partial, h->x);
  int it = 0;
  esmp2_status status = ESMP2_OK;
  while (rel > opts->tol && it < opts->max_iter) {
    esmp2_status st = apply_op_dot(h, c, c.s64, (const double*)h->p, h->q);
    if (st != ESMP2_OK) return st;
    hipLaunchKernelGGL(k_update_r<double>, dim3(NB), dim3(256), 0, s, h->r, (const double*)h->q, c.dinv32, n,
                       d.off[1], d.off[2], (const double*)h->sc, h->partial);
    hipLaunchKernelGGL(k_finish, dim3(2), dim3(1024), 0, s, h->partial, (int)NB, h->sc, SC_RHO_NEW);  // RHO_NEW, RR
    ESMP2_HIP(hipMemcpyAsync(h->pin->sc, h->sc, sizeof(double) * SC_N, hipMemcpyDeviceToHost, s));
    ESMP2_HIP(hipStreamSynchronize(s));
    if (!(hs[SC_PQ] > 0.0)) { status = ESMP2_NOT_SPD; h->err = "p.Ap <= 0 in conjugate gradient"; break; }
    ++it;
    rel = sqrt(hs[SC_RR]) / bn;
    if (opts->resid_hist) opts->resid_hist[it - 1] = rel;
    if (rel <= opts->tol || it >= opts->max_iter) {   // last step: x += alpha p only
      hipLaunchKernelGGL(k_update_x<double>, dim3(NB), dim3(256), 0, s, h->x, (const double*)h->p, n,
                         (const double*)h->sc);
      break;
    }
    hipLaunchKernelGGL(k_update_px<double>, dim3(NB), dim3(256), 0, s, h->x, h->p, (const double*)h->r, c.dinv32, n,
                       (const double*)h->sc);
    hipLaunchKernelGGL(k_roll_rho, dim3(1), dim3(64), 0, s, h->sc);
  }
  if (status == ESMP2_OK && rel > opts->tol) { status = ESMP2_NOT_CONVERGED; h->err = "max_iter reached"; }
  return finish_solve(h, c, opts, res, rel, it, 0, status);
}

// Mixed precision: FP64 iterative refinement around FP32 inner solves.
//   r = -b - A64 x;  repeat: d = A32^-1 (r / ||r||) by FP32 Jacobi-PCG to a
//   relative reduction eta;  x += ||r|| d;  r = -b - A64 x;  until ||r||/||b|| <= tol.
// eta = max(inner_tol, tol / (2 ||r||/||b||)): the last inner solve stops as soon
// as it reaches the target; inner_tol bounds what an FP32 operator can deliver.
static esmp2_status solve_mixed(esmp2_handle h, const OpCtx& c, const esmp2_solve_opts* opts,
                                esmp2_solve_result* res) {
  h->sc_init_ready = false;
  const Dims& d = h->d;
  const int64_t n = h->namp;
  hipStream_t s = h->stream;
  const unsigned NB = PCG_BLOCKS;
  // an operator with BF16 operands is accurate to ~1e-3 relative: ask its inner
  // solves for two digits and let the FP64 refinement do the rest
  const double floor_eta = opts->inner_tol > 0 ? opts->inner_tol : (c.s32.prec == ESMP2_BF16 ? 1e-2 : 1e-5);
  wdot(h, c.b, c.b, SC_BB);
  if (opts->x0) {
    if (c.rotated) {
      esmp2_status st0 = rotate_amplitudes(h, opts->x0, h->x, true);
      if (st0 != ESMP2_OK) return st0;
    } else {
      ESMP2_HIP(hipMemcpyAsync(h->x, opts->x0, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    }
    esmp2_status st = apply_op(h, c, c.s64, (const double*)h->x, h->q);
    if (st != ESMP2_OK) return st;
    hipLaunchKernelGGL(k_resid, dim3(NB), dim3(256), 0, s, c.b, (const double*)h->q, h->r, n, d.off[1], d.off[2],
                       h->partial);
  } else {
    ESMP2_HIP(hipMemsetAsync(h->x, 0, sizeof(double) * n, s));
    hipLaunchKernelGGL(k_resid, dim3(NB), dim3(256), 0, s, c.b, (const double*)nullptr, h->r, n, d.off[1],
                       d.off[2], h->partial);
  }
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, h->partial, (int)NB, h->sc, SC_RR);
  double* hs = h->pin->sc;
  ESMP2_HIP(hipMemcpyAsync(h->pin->sc, h->sc, sizeof(double) * SC_N, hipMemcpyDeviceToHost, s));
  ESMP2_HIP(hipStreamSynchronize(s));
  const double bn = sqrt(hs[SC_BB]);
  double rel = sqrt(hs[SC_RR]) / bn;
  int it = 0, outer = 0;
  esmp2_status status = ESMP2_OK;
  while (rel > opts->tol && it < opts->max_iter && status == ESMP2_OK) {
    ++outer;
    const double scale = rel * bn;
    const double eta = std::max(floor_eta, 0.5 * opts->tol / rel);
    hipLaunchKernelGGL(k_init_inner, dim3(NB), dim3(256), 0, s, (const double*)h->r, scale, h->r32, h->p32, h->d32,
                       c.dinv32, n, d.off[1], d.off[2], h->partial);
    hipLaunchKernelGGL(k_finish, dim3(2), dim3(1024), 0, s, h->partial, (int)NB, h->sc, SC_RHO);  // RHO, rr0
    ESMP2_HIP(hipMemcpyAsync(h->pin->sc, h->sc, sizeof(double) * SC_N, hipMemcpyDeviceToHost, s));
    ESMP2_HIP(hipStreamSynchronize(s));
    const double rr0 = hs[SC_PQ];
    while (it < opts->max_iter) {
      esmp2_status st = apply_op_dot(h, c, c.s32, (const float*)h->p32, h->q32);
      if (st != ESMP2_OK) return st;
      hipLaunchKernelGGL(k_update_r<float>, dim3(NB), dim3(256), 0, s, h->r32, (const float*)h->q32, c.dinv32, n,
                         d.off[1], d.off[2], (const double*)h->sc, h->partial);
      hipLaunchKernelGGL(k_finish, dim3(2), dim3(1024), 0, s, h->partial, (int)NB, h->sc, SC_RHO_NEW);
      ESMP2_HIP(hipMemcpyAsync(h->pin->sc, h->sc, sizeof(double) * SC_N, hipMemcpyDeviceToHost, s));
      ESMP2_HIP(hipStreamSynchronize(s));
      if (!(hs[SC_PQ] > 0.0)) { status = ESMP2_NOT_SPD; h->err = "p.Ap <= 0 in conjugate gradient"; break; }
      ++it;
      const double irel = sqrt(hs[SC_RR] / rr0);
      if (opts->resid_hist) opts->resid_hist[it - 1] = irel * rel;   // estimate of the FP64 residual
      if (irel <= eta || it >= opts->max_iter) {   // last step of this inner solve: d += alpha p only
        hipLaunchKernelGGL(k_update_x<float>, dim3(NB), dim3(256), 0, s, h->d32, (const float*)h->p32, n,
                           (const double*)h->sc);
        break;
      }
      hipLaunchKernelGGL(k_update_px<float>, dim3(NB), dim3(256), 0, s, h->d32, h->p32, (const float*)h->r32,
                         c.dinv32, n, (const double*)h->sc);
      hipLaunchKernelGGL(k_roll_rho, dim3(1), dim3(64), 0, s, h->sc);
    }
    if (status != ESMP2_OK) break;
    hipLaunchKernelGGL(k_refine, dim3(NB), dim3(256), 0, s, h->x, (const float*)h->d32, scale, n);
    esmp2_status st = apply_op(h, c, c.s64, (const double*)h->x, h->q);
    if (st != ESMP2_OK) return st;
    hipLaunchKernelGGL(k_resid, dim3(NB), dim3(256), 0, s, c.b, (const double*)h->q, h->r, n, d.off[1], d.off[2],
                       h->partial);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, h->partial, (int)NB, h->sc, SC_RR);
    ESMP2_HIP(hipMemcpyAsync(h->pin->sc, h->sc, sizeof(double) * SC_N, hipMemcpyDeviceToHost, s));
    ESMP2_HIP(hipStreamSynchronize(s));
    rel = sqrt(hs[SC_RR]) / bn;
  }
  if (status == ESMP2_OK && rel > opts->tol) { status = ESMP2_NOT_CONVERGED; h->err = "max_iter reached"; }
  return finish_solve(h, c, opts, res, rel, it, outer, status);
}

esmp2_status esmp2_solve(esmp2_handle h, const esmp2_solve_opts* opts, esmp2_solve_result* res) {
  if (!h) return ESMP2_INVALID_ARG;
  if (!opts || !res) return fail(h, ESMP2_INVALID_ARG, "null opts/result");
  if (h->state < 2) return fail(h, ESMP2_BAD_ORDER, "esmp2_rotate_top first");
  if (!(opts->tol > 0) || opts->max_iter < 1) return fail(h, ESMP2_INVALID_ARG, "tol > 0 and max_iter >= 1");
  if (opts->precision != ESMP2_FP64 && opts->precision != ESMP2_FP32 && opts->precision != ESMP2_BF16)
    return fail(h, ESMP2_INVALID_ARG, "unknown precision");
  if (opts->precision == ESMP2_BF16 && (opts->basis != ESMP2_BASIS_TOP || !bf16_supported(h->d)))
    return fail(h, ESMP2_UNSUPPORTED,
                "BF16 applies to the Sylvester products of the TOP-basis operator, padded virtual dimension 80, 112 "
                "or 160");
  if (opts->basis != ESMP2_BASIS_TOP && opts->basis != ESMP2_BASIS_SEMICANONICAL)
    return fail(h, ESMP2_INVALID_ARG, "unknown basis");
  if (opts->precision != ESMP2_FP64 && !(opts->inner_tol >= 0 && opts->inner_tol < 1))
    return fail(h, ESMP2_INVALID_ARG, "inner_tol must lie in [0, 1)");
  if (h->ntop > 1 && (opts->precision == ESMP2_BF16 || opts->basis != ESMP2_BASIS_TOP))
    return fail(h, ESMP2_UNSUPPORTED, "more than one large TOP: FP64 or FP32-refined solve in the TOP basis only");
  ESMP2_HIP(hipSetDevice(h->device));
  memset(res, 0, sizeof(*res));
  if (!h->have_rhs) {
    esmp2_status st = build_rhs(h);
    if (st != ESMP2_OK) { res->status = st; return st; }
  }
  if (opts->basis == ESMP2_BASIS_TOP) {
    esmp2_status st = ensure_b_top(h);
    if (st != ESMP2_OK) { res->status = st; return st; }
  }
  OpCtx c = ctx_top(h);
  if (opts->basis == ESMP2_BASIS_SEMICANONICAL) {
    if (!h->have_sc) {
      esmp2_status st = semican_setup(h, opts->precision == ESMP2_FP64 && !opts->x0);
      if (st != ESMP2_OK) { res->status = st; return st; }
    }
    c = ctx_sc(h);
  }
  if (opts->precision == ESMP2_BF16) c.s32.prec = ESMP2_BF16;
  return opts->precision == ESMP2_FP64 ? solve64(h, c, opts, res) : solve_mixed(h, c, opts, res);
}

}  // extern "C"

// The batched FP64 conjugate gradient of many one-TOP states in the
// pinned-semicanonical basis (set up, with their right-hand sides, beforehand):
// every step is one launch for all states (see batch.hip), each state's
// scalars, convergence test and stop live on the device, and the host polls the
// number of states still iterating one iteration behind the launches, so the
// device never waits for the host between iterations.
static esmp2_status solve_batch_sc64(esmp2_handle* hs, int n, const esmp2_solve_opts* opts,
                                     esmp2_solve_result* res) {
  esmp2_handle h0 = hs[0];
  hipStream_t s = h0->stream;
  std::vector<BState> st(n);
  std::vector<int> first[3];
  int64_t tot[3] = {0, 0, 0};
  for (int k = 0; k < 3; ++k) first[k].resize(n + 1);
  for (int i = 0; i < n; ++i) {
    esmp2_handle h = hs[i];
    const OpCtx c = ctx_sc(h);
    const PrologueArgs<double> pa = prologue_args(h, c.s64, (const double*)h->p, h->q, true);
    BState& B = st[i];
    memset(&B, 0, sizeof(B));
    B.d = h->d;
    B.gv = pa.gv;
    B.aa = ArrowArgs<double>{pa.ga, c.s64.Fd, c.s64.Fl, c.s64.side_tr, h->gv};
    const int* pv = h->pairs;
    const Dims& d = h->d;
    B.pt = PairTables{pv, pv + d.npv, pv + d.npv + d.npv1, pv + d.npv + d.npv1 + d.npo};
    B.chunks = (const int4*)h->chunks;
    B.nsym = (int)sym_s2_blocks(d);
    B.ngemv = pa.jobs;
    B.nchunks = h->nchunks;
    B.r = h->r; B.p = h->p; B.q = h->q; B.sc = h->sc; B.partial = h->partial; B.pq = h->pq_part;
    B.S = c.s64.S;
    B.b = c.b;
    B.dinv = c.dinv32;
    B.n = h->namp;
    B.mode = BS_DONE;
    const int cnt[3] = {B.nsym, B.ngemv, B.nchunks};
    for (int k = 0; k < 3; ++k) {
      first[k][i] = (int)tot[k];
      tot[k] += cnt[k];
    }
  }
  for (int k = 0; k < 3; ++k) {
    if (tot[k] <= 0 || tot[k] >= (int64_t)INT32_MAX) return fail(h0, ESMP2_INVALID_ARG, "batch too large");
    first[k][n] = (int)tot[k];
  }
  if ((int64_t)n * 2 * BATCH_CG_BLOCKS >= (int64_t)INT32_MAX) return fail(h0, ESMP2_INVALID_ARG, "batch too large");
  // device copies of the state records, the first-block tables and the counter
  BState* dS = nullptr;
  int* dfirst = nullptr;
  int* dact = nullptr;
  auto cleanup = [&]() {
    if (dS) (void)hipFree(dS);
    if (dfirst) (void)hipFree(dfirst);
    if (dact) (void)hipFree(dact);
  };
  if (hipMalloc(&dS, sizeof(BState) * n) != hipSuccess || hipMalloc(&dfirst, sizeof(int) * 3 * (n + 1)) != hipSuccess ||
      hipMalloc(&dact, sizeof(int)) != hipSuccess) {
    cleanup();
    return fail(h0, ESMP2_OOM, "device allocation of the batch records");
  }
  std::vector<int> fcat;
  for (int k = 0; k < 3; ++k) fcat.insert(fcat.end(), first[k].begin(), first[k].end());
  hipError_t e = hipMemcpyAsync(dS, st.data(), sizeof(BState) * n, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dfirst, fcat.data(), sizeof(int) * fcat.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);    // the host vectors go out of scope with this call
  if (e != hipSuccess) { cleanup(); return fail(h0, ESMP2_HIP_ERROR, hipGetErrorString(e)); }
  const int* f_sym = dfirst;
  const int* f_gemv = dfirst + (n + 1);
  const int* f_arrow = dfirst + 2 * (n + 1);
  const unsigned NBV = (unsigned)(n * BATCH_CG_BLOCKS);
  int nv_max = 0;                  // the LDS arrays of the GEMV kernel hold the largest virtual dimension
  for (int i = 0; i < n; ++i) nv_max = std::max(nv_max, hs[i]->d.nv);
  const unsigned nsmall = (unsigned)((n + 63) / 64);
  volatile int* act = h0->pin->active;
  hipEvent_t ev[2] = {nullptr, nullptr};
  auto fin = [&](esmp2_status r, const char* msg) {
    for (auto& v : ev)
      if (v) (void)hipEventDestroy(v);
    cleanup();
    return msg ? fail(h0, r, msg) : r;
  };
  for (auto& v : ev)
    if (hipEventCreateWithFlags(&v, hipEventDisableTiming) != hipSuccess) return fin(ESMP2_HIP_ERROR, "event");
  // start from x = 0: r = -b, p = M r, <b, b>, then the states converged already drop out
  hipLaunchKernelGGL(kb_init, dim3(NBV), dim3(256), 0, s, dS);
  hipLaunchKernelGGL(kb_dot_bb, dim3(NBV), dim3(256), 0, s, dS);
  hipLaunchKernelGGL(kb_finish_init, dim3(3 * n), dim3(1024), 0, s, dS);
  hipLaunchKernelGGL(kb_zero, dim3(1), dim3(64), 0, s, dact);
  hipLaunchKernelGGL(kb_start, dim3(nsmall), dim3(64), 0, s, dS, n, opts->tol, dact);
  act[0] = act[1] = -1;
  if (hipMemcpyAsync((void*)&act[0], dact, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipEventRecord(ev[0], s) != hipSuccess)
    return fin(ESMP2_HIP_ERROR, "enqueue of the batched start");
  // iterations: launch iteration k + 1, then read the count left by iteration k
  for (int k = 0;; ++k) {
    if (k > opts->max_iter + 1) return fin(ESMP2_HIP_ERROR, "internal: batched iteration count exceeded");
    hipLaunchKernelGGL(kb_sym, dim3((unsigned)tot[0]), dim3(256), 0, s, (const BState*)dS, f_sym, n);
    if (nv_max <= 160)
      hipLaunchKernelGGL(kb_gemv<160>, dim3((unsigned)tot[1]), dim3(256), 0, s, (const BState*)dS, f_gemv, n);
    else
      hipLaunchKernelGGL(kb_gemv<192>, dim3((unsigned)tot[1]), dim3(256), 0, s, (const BState*)dS, f_gemv, n);
    hipLaunchKernelGGL(kb_arrow, dim3((unsigned)tot[2]), dim3(256), 0, s, (const BState*)dS, f_arrow, n);
    hipLaunchKernelGGL(kb_finish_pq, dim3(n), dim3(1024), 0, s, dS);
    hipLaunchKernelGGL(kb_update_r, dim3(NBV), dim3(256), 0, s, dS);
    hipLaunchKernelGGL(kb_finish_r, dim3(2 * n), dim3(1024), 0, s, dS);
    hipLaunchKernelGGL(kb_zero, dim3(1), dim3(64), 0, s, dact);
    hipLaunchKernelGGL(kb_check, dim3(nsmall), dim3(64), 0, s, dS, n, opts->tol, opts->max_iter, dact);
    hipLaunchKernelGGL(kb_update, dim3(NBV), dim3(256), 0, s, dS);
    hipLaunchKernelGGL(kb_roll, dim3(nsmall), dim3(64), 0, s, dS, n);
    const int nx = (k + 1) & 1;
    if (hipEventSynchronize(ev[nx]) != hipSuccess) return fin(ESMP2_HIP_ERROR, "batched iteration");
    act[nx] = -1;
    if (hipMemcpyAsync((void*)&act[nx], dact, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipEventRecord(ev[nx], s) != hipSuccess)
      return fin(ESMP2_HIP_ERROR, "enqueue of a batched iteration");
    if (hipEventSynchronize(ev[k & 1]) != hipSuccess) return fin(ESMP2_HIP_ERROR, "batched iteration");
    if (act[k & 1] == 0) break;     // the iteration just launched finds every state stopped
  }
  // E2 = -sum_i alpha_i rho_i (in sc, batch.hip) and E2_S, for every state, then one wait
  for (int i = 0; i < n; ++i) {
    esmp2_handle h = hs[i];
    if (h->e2s_pending) {
      if (hipStreamWaitEvent(s, h->ev_e2s, 0) != hipSuccess) return fin(ESMP2_HIP_ERROR, "E2_S join");
      h->e2s_pending = false;
    }
  }
  e = hipMemcpyAsync(st.data(), dS, sizeof(BState) * n, hipMemcpyDeviceToHost, s);
  for (int i = 0; i < n && e == hipSuccess; ++i) {
    esmp2_handle h = hs[i];
    e = hipMemcpyAsync(h->pin->sc, h->sc, sizeof(double) * SC_N, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && h->e2s_dev)
      e = hipMemcpyAsync(&h->pin->e2s, h->e2s_part + E2S_CAP, sizeof(double), hipMemcpyDeviceToHost, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return fin(ESMP2_HIP_ERROR, hipGetErrorString(e));
  esmp2_status ret = ESMP2_OK;
  for (int i = 0; i < n; ++i) {
    esmp2_handle h = hs[i];
    if (h->e2s_dev) { h->e2s = h->pin->e2s; h->e2s_dev = false; }
    const double* sc = h->pin->sc;
    esmp2_solve_result& r = res[i];
    const BState& B = st[i];
    r.e2_dl = sc[SC_BX] - sc[SC_XR];
    r.e2_s = h->e2s;
    r.e2 = r.e2_dl + r.e2_s;
    r.e0 = h->e0;
    r.rel_resid = B.rel;
    r.iterations = B.it;
    r.outer = 0;
    r.status = (esmp2_status)B.status;
    if (B.status == ESMP2_NOT_SPD) h->err = "p.Ap <= 0 in conjugate gradient";
    if (B.status == ESMP2_NOT_CONVERGED) h->err = "max_iter reached";
    if (B.status != ESMP2_OK && ret == ESMP2_OK) ret = (esmp2_status)B.status;
  }
  return fin(ret, nullptr);
}

extern "C" {

esmp2_status esmp2_solve_batch(esmp2_handle* hs, int n, const esmp2_solve_opts* opts, esmp2_solve_result* res,
                               int n_threads) {
  if (n < 0 || (n > 0 && (!hs || !res)) || !opts) return ESMP2_INVALID_ARG;
  for (int i = 0; i < n; ++i) {
    if (!hs[i]) return ESMP2_INVALID_ARG;
    if (opts->x0 || opts->x_out || opts->resid_hist)
      return fail(hs[i], ESMP2_INVALID_ARG, "x0, x_out and resid_hist are per-state: use esmp2_solve");
    if (hs[i]->state < 1) return fail(hs[i], ESMP2_BAD_ORDER, "esmp2_set_problem first");
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return fail(hs[i], ESMP2_INVALID_ARG, "a handle appears twice in the batch");
  }
  if (n == 0) return ESMP2_OK;
  // one launch per step for all states: FP64, pinned-semicanonical basis, one
  // large TOP, every state on one device; otherwise one solve per state
  bool together = opts->precision == ESMP2_FP64 && opts->basis == ESMP2_BASIS_SEMICANONICAL &&
                  opts->tol > 0 && opts->max_iter >= 1;
  for (int i = 0; i < n; ++i)
    together = together && hs[i]->ntop == 1 && hs[i]->device == hs[0]->device;
  const int nt = std::max(1, std::min(n, n_threads > 0 ? n_threads : 8));
  std::vector<esmp2_status> st(n, ESMP2_OK);
  std::atomic<int> next{0};
  auto work = [&]() {
    for (int i = next++; i < n; i = next++) {
      esmp2_handle h = hs[i];
      memset(&res[i], 0, sizeof(res[i]));
      esmp2_status s = esmp2_rotate_top(h, nullptr);
      if (s == ESMP2_OK) s = esmp2_build_rhs(h, nullptr, nullptr, nullptr);
      if (together) {
        // set-up only: the operator blocks and right-hand side of the basis
        if (s == ESMP2_OK && hipSetDevice(h->device) != hipSuccess) s = fail(h, ESMP2_HIP_ERROR, "hipSetDevice");
        if (s == ESMP2_OK && !h->have_sc) s = semican_setup(h);
        if (s == ESMP2_OK && hipStreamSynchronize(h->stream) != hipSuccess) s = fail(h, ESMP2_HIP_ERROR, "set-up");
        if (s == ESMP2_OK && h->nchunks <= 0) s = fail(h, ESMP2_UNSUPPORTED, "internal: no coupling chunks");
        res[i].status = s;
      } else if (s == ESMP2_OK) {
        s = esmp2_solve(h, opts, &res[i]);
      } else {
        res[i].status = s;
      }
      st[i] = s;
    }
  };
  std::vector<std::thread> pool;
  try {
    for (int t = 1; t < nt; ++t) pool.emplace_back(work);
  } catch (...) {
    // fewer host threads than asked: the remaining ones (and this one) take the states
  }
  work();
  for (auto& t : pool) t.join();
  for (int i = 0; i < n; ++i)
    if (st[i] != ESMP2_OK) return st[i];
  if (together) {
    esmp2_handle h = hs[0];
    ESMP2_HIP(hipSetDevice(h->device));
    return solve_batch_sc64(hs, n, opts, res);
  }
  return ESMP2_OK;
}

// ---------------------------------------------------------------------------
// dE2/dF~ and dE2/dB~ (rotation held fixed)
// ---------------------------------------------------------------------------
// npart_cap: size of the partials buffer; lenA, lenB, lenOut: element counts of the
// operands and the output; every index the launch can form is checked against them
// on the host first.
static esmp2_status contract(esmp2_handle h, double* part, int64_t npart_cap, const Contr& c, int64_t lenA,
                             int64_t lenB, double alpha, double* out, int64_t lenOut, int64_t dst, int64_t so0,
                             int64_t so1) {
  const int64_t ncon = (int64_t)c.nC[0] * c.nC[1] * c.nC[2] * c.nC[3];
  const int nout = c.nE[0] * c.nE[1];
  if (nout <= 0 || ncon <= 0) return ESMP2_OK;
  int64_t hiA = c.oA, hiB = c.oB, hiO = dst + (c.nE[0] - 1) * so0 + (c.nE[1] - 1) * so1;
  for (int k = 0; k < 2; ++k) { hiA += (c.nE[k] - 1) * c.aE[k]; hiB += (c.nE[k] - 1) * c.bE[k]; }
  for (int k = 0; k < 4; ++k) { hiA += (c.nC[k] - 1) * c.aC[k]; hiB += (c.nC[k] - 1) * c.bC[k]; }
  if (c.oA < 0 || c.oB < 0 || dst < 0 || hiA >= lenA || hiB >= lenB || hiO >= lenOut)
    return fail(h, ESMP2_HIP_ERROR, "internal: gradient contraction out of range");
  const int64_t cap = std::max<int64_t>(1, std::min<int64_t>(1024, npart_cap / nout));
  const int nsplit = (int)std::min<int64_t>(cap, std::max<int64_t>(1, ncon / 4096));
  hipLaunchKernelGGL(k_contract, dim3(nout, nsplit), dim3(256), 0, h->stream, c, part);
  hipLaunchKernelGGL(k_contract_fin, dim3(nblk(nout)), dim3(256), 0, h->stream, (const double*)part, c.nE[0],
                     c.nE[1], nsplit, alpha, out, dst, so0, so1);
  ESMP2_HIP(hipGetLastError());
  return ESMP2_OK;
}

// G[i * ld + j] += alpha * sum_b sum_k X[b*sb + i*si + k*sk] X[b*sb + j*si + k*sk]   (i, j < m)
static esmp2_status gram(esmp2_handle h, const double* X, int nb, int64_t sb, int m, int64_t si, int K, int64_t sk,
                         double alpha, double* G, int ld, double* tmp) {
  if (nb <= 0 || m <= 0 || K <= 0) return ESMP2_OK;
  GemmArgs g{};
  g.A = X; g.B = X; g.C = tmp; g.M = m; g.N = m; g.K = K;
  g.sAb = sb; g.sAi = si; g.sAk = sk; g.sBb = sb; g.sBk = sk; g.sBj = si;
  g.sCb = (int64_t)m * m; g.sCi = m; g.sCj = 1; g.alpha = 1.0; g.beta = 0.0;
  ESMP2_HIP(gemm(h->stream, nb, g));
  const int ny = std::max(1, std::min(nb / 8, 2048 / (int)nblk((int64_t)m * m)));   // batch split
  hipLaunchKernelGGL(k_batch_sum_acc, dim3(nblk((int64_t)m * m), ny), dim3(256), 0, h->stream, (const double*)tmp,
                     nb, m, m, alpha, G, ld);
  ESMP2_HIP(hipGetLastError());
  return ESMP2_OK;
}


esmp2_status esmp2_gradient(esmp2_handle h, const double* x, double* dF, double* dB) {
  if (!h) return ESMP2_INVALID_ARG;
  if (h->state < 3) return fail(h, ESMP2_BAD_ORDER, "esmp2_build_rhs (and a solve for x) first");
  if (!x || (!dF && !dB)) return fail(h, ESMP2_INVALID_ARG, "x and at least one of dF, dB are required");
  if (h->ntop > 1) return fail(h, ESMP2_UNSUPPORTED, "gradient with more than one large TOP");
  ESMP2_HIP(hipSetDevice(h->device));
  ESMP2_TRY(ensure_b_top(h));
  const Dims& d = h->d;
  const int no = d.no, nv = d.nv, n = d.n, na = d.naux, nov = no * nv;
  const int o1 = no - 1, v1 = nv - 1;
  hipStream_t s = h->stream;
  // ---- workspace
  const int64_t nd = (int64_t)no * no * nv * nv;
  const int64_t dsz[7] = {nd, nd, (int64_t)o1 * o1 * v1 * v1, nd, (int64_t)no * no * v1 * v1,
                          (int64_t)o1 * o1 * nv * nv, (int64_t)o1 * o1 * v1 * v1};
  constexpr int NB_NORM = 256;
  int64_t need = nd;                                           // swap
  for (int k = 0; k < 7; ++k) need += dsz[k];
  const int64_t ntmp = nd + (int64_t)no * no * no * nv;      // per-batch Gram blocks (summed afterwards)
  const int64_t npart = (int64_t)64 * nov;
  need += ntmp + (int64_t)n * n + 2 * (int64_t)nov * nov + nov + nv + no + 8 + npart + 7 * NB_NORM + 8 +
          2 * (int64_t)na * nov + (int64_t)na * nv * no + (int64_t)na * no * no;
  if (h->gws_n < (size_t)need) {
    if (!dalloc(h, &h->gws, (size_t)need)) return fail(h, ESMP2_OOM, "gradient workspace allocation failed");
    h->gws_n = (size_t)need;
  }
  double* w = h->gws;
  double* dn[7];
  for (int k = 0; k < 7; ++k) { dn[k] = w; w += dsz[k]; }
  double* swp = w; w += nd;
  double* tmp = w; w += ntmp;
  double* G = w; w += (int64_t)n * n;
  double* GV = w; w += (int64_t)nov * nov;
  double* GM = w; w += (int64_t)nov * nov;
  double* Gf = w; w += nov;
  double* Gev = w; w += nv;
  double* Geo = w; w += no;
  double* scal = w; w += 8;
  double* part = w; w += npart;
  double* npt = w; w += 7 * NB_NORM;
  double* sbox = w; w += 8;
  double* dBov = w; w += (int64_t)na * nov;
  double* dX = w; w += (int64_t)na * nov;
  double* dBvt = w; w += (int64_t)na * nv * no;
  double* dBoo = w; w += (int64_t)na * no * no;
  // everything accumulated into starts at zero (one contiguous range from G to sbox)
  ESMP2_HIP(hipMemsetAsync(G, 0, sizeof(double) * (size_t)(sbox - G), s));
  ESMP2_HIP(hipMemsetAsync(dBov, 0, sizeof(double) * (size_t)(w - dBov), s));
  // box scales s = W / (copies of a stored amplitude in the dense tensor)
  const double sb_h[8] = {0.5, 1.0, 0.5, 0.5, 1.0, 1.0, 2.0, 0.0};
  ESMP2_HIP(hipMemcpyAsync(sbox, sb_h, sizeof(sb_h), hipMemcpyHostToDevice, s));
  // ---- 1. dense boxes (S2 flip-symmetrised)
  for (int k = 0; k < 7; ++k) {
    if (k == B_S2) hipLaunchKernelGGL(k_sym_s2<double>, dim3(sym_s2_blocks(d)), dim3(256), 0, s, d, x, dn[k]);
    else hipLaunchKernelGGL(k_unpack_box, dim3(1024), dim3(256), 0, s, d, k, x, dn[k]);
  }
  ESMP2_HIP(hipGetLastError());
  // ---- 2a. Fock blocks on the free indices: Gram matrices of the batch matrices
  for (int k = 0; k < 7; ++k) {
    int lo_o, lo_v;
    box_ranges(k, lo_o, lo_v);
    const int ro = no - lo_o, rv = nv - lo_v;
    const double sc = sb_h[k];
    const int64_t v2 = (int64_t)rv * rv;
    double* Gv = G + (int64_t)(no + lo_v) * n + no + lo_v;
    double* Go = G + (int64_t)lo_o * n + lo_o;
    // Gram blocks per batch (summed afterwards), batches small enough to fill the chip.
    // Virtual slots: sum over (P, Q, c) of X[P][Q][c][a] X[P][Q][c][e] (left slot, one batch
    // per (P, Q)); the right slot equals it for virtual-antisymmetric boxes and S~, else it
    // comes from the transposed copy.
    const bool vir_dense = (k == B_H12 || k == B_H22);
    ESMP2_TRY(gram(h, dn[k], ro * ro, v2, rv, 1, rv, rv, vir_dense ? sc : 2.0 * sc, Gv, n, tmp));
    if (vir_dense) {
      hipLaunchKernelGGL(k_swap_mid, dim3(1024), dim3(256), 0, s, (const double*)dn[k], swp, (int64_t)ro * ro, rv,
                         rv, (int64_t)1);
      ESMP2_TRY(gram(h, swp, ro * ro, v2, rv, 1, rv, rv, sc, Gv, n, tmp));
    }
    // Occupied slots: -sum over (k, A, B) of X[i][k][AB] X[m][k][AB] (first slot, one batch
    // per (k, A)); the second equals it for occupied-antisymmetric boxes and S~, else it
    // comes from the transposed copy.
    const bool occ_dense = (k == B_H21 || k == B_H22);
    ESMP2_TRY(gram(h, dn[k], ro * rv, rv, ro, ro * v2, rv, 1, occ_dense ? -sc : -2.0 * sc, Go, n, tmp));
    if (occ_dense) {
      hipLaunchKernelGGL(k_swap_mid, dim3(1024), dim3(256), 0, s, (const double*)dn[k], swp, (int64_t)1, ro, ro, v2);
      ESMP2_TRY(gram(h, swp, ro * rv, rv, ro, ro * v2, rv, 1, -sc, Go, n, tmp));
    }
    hipLaunchKernelGGL(k_sumsq, dim3(NB_NORM), dim3(256), 0, s, (const double*)dn[k], dsz[k], npt + k * NB_NORM);
  }
  hipLaunchKernelGGL(k_norm_scalars, dim3(1), dim3(64), 0, s, (const double*)npt, NB_NORM, (const double*)sbox, scal);
  ESMP2_HIP(hipGetLastError());
  // ---- 2b. pinned-row transfers and f_ov couplings (strided contractions)
  {
    const double *T2 = dn[B_T2], *St = dn[B_S2], *T3 = dn[B_T3], *H11 = dn[B_H11], *H12 = dn[B_H12],
                 *H21 = dn[B_H21], *H22 = dn[B_H22];
    const int64_t N = n;
    // tensor strides (dims d0 d1 d2 d3 -> d1 d2 d3, d2 d3, d3, 1)
    const int64_t sT2[4] = {(int64_t)no * nv * nv, (int64_t)nv * nv, nv, 1};            // also St, H11
    const int64_t sT3[4] = {(int64_t)o1 * v1 * v1, (int64_t)v1 * v1, v1, 1};
    const int64_t sH12[4] = {(int64_t)no * v1 * v1, (int64_t)v1 * v1, v1, 1};
    const int64_t sH21[4] = {(int64_t)o1 * nv * nv, (int64_t)nv * nv, nv, 1};
    const int64_t sH22[4] = {(int64_t)o1 * v1 * v1, (int64_t)v1 * v1, v1, 1};
    auto C = [&](const double* A, int64_t oA, const double* B, int64_t oB) {
      Contr c{};
      c.A = A; c.B = B; c.oA = oA; c.oB = oB;
      c.nE[0] = c.nE[1] = 1;
      c.nC[0] = c.nC[1] = c.nC[2] = c.nC[3] = 1;
      return c;
    };
    auto E = [](Contr& c, int slot, int nE, int64_t a, int64_t b) { c.nE[slot] = nE; c.aE[slot] = a; c.bE[slot] = b; };
    auto len = [&](const double* p) -> int64_t {
      for (int k = 0; k < 7; ++k) if (p == dn[k]) return dsz[k];
      return 0;
    };
    auto K = [](Contr& c, int slot, int nC, int64_t a, int64_t b) { c.nC[slot] = nC; c.aC[slot] = a; c.bC[slot] = b; };
    Contr c;
    // transfers through the t' row of F_vv: G[t'][e], e >= 1
    c = C(H11, 1, H12, 0); E(c, 0, v1, 0, v1);
    K(c, 0, no, sT2[0], sH12[0]); K(c, 1, no, sT2[1], sH12[1]); K(c, 2, v1, 1, 1);
    ESMP2_TRY(contract(h, part, npart, c, len(c.A), len(c.B), 2.0, G, N * N, N * no + no + 1, 1, 0));
    c = C(H21, 1, H22, 0); E(c, 0, v1, 0, v1);
    K(c, 0, o1, sH21[0], sH22[0]); K(c, 1, o1, sH21[1], sH22[1]); K(c, 2, v1, 1, 1);
    ESMP2_TRY(contract(h, part, npart, c, len(c.A), len(c.B), 4.0, G, N * N, N * no + no + 1, 1, 0));
    // transfers through the t column of F_oo: G[m][t], m >= 1
    c = C(H11, (int64_t)nv * nv, H21, 0); E(c, 0, o1, 0, sH21[0]);
    K(c, 0, o1, sT2[1], sH21[1]); K(c, 1, nv * nv, 1, 1);
    ESMP2_TRY(contract(h, part, npart, c, len(c.A), len(c.B), -2.0, G, N * N, N, N, 0));
    c = C(H12, (int64_t)v1 * v1, H22, 0); E(c, 0, o1, 0, sH22[0]);
    K(c, 0, o1, sH12[1], sH22[1]); K(c, 1, v1 * v1, 1, 1);
    ESMP2_TRY(contract(h, part, npart, c, len(c.A), len(c.B), -4.0, G, N * N, N, N, 0));
    // f_ov couplings (doubles -> L-triples; the de-excitation doubles them): G[i][n_occ + a]
    const int64_t ov = no;     // column offset of the virtual block
    // L-triples <- T2
    c = C(T3, 0, T2, sT2[0] + sT2[1] + sT2[2] + 1);
    K(c, 0, o1, sT3[0], sT2[0]); K(c, 1, o1, sT3[1], sT2[1]); K(c, 2, v1, sT3[2], sT2[2]); K(c, 3, v1, 1, 1);
    ESMP2_TRY(contract(h, part, npart, c, len(c.A), len(c.B), 1.0, G, N * N, ov, 0, 0));
    c = C(T3, 0, T2, sT2[1] + sT2[2] + 1); E(c, 0, o1, sT3[0], 0);
    K(c, 0, o1, sT3[1], sT2[1]); K(c, 1, v1, sT3[2], sT2[2]); K(c, 2, v1, 1, 1);
    ESMP2_TRY(contract(h, part, npart, c, len(c.A), len(c.B), -2.0, G, N * N, N + ov, N, 0));
    c = C(T3, 0, T2, sT2[0] + sT2[1] + 1); E(c, 0, v1, sT3[2], 0);
    K(c, 0, o1, sT3[0], sT2[0]); K(c, 1, o1, sT3[1], sT2[1]); K(c, 2, v1, 1, 1);
    ESMP2_TRY(contract(h, part, npart, c, len(c.A), len(c.B), -2.0, G, N * N, ov + 1, 1, 0));
    c = C(T3, 0, T2, sT2[1] + 1); E(c, 0, o1, sT3[0], 0); E(c, 1, v1, sT3[2], 0);
    K(c, 0, o1, sT3[1], sT2[1]); K(c, 1, v1, 1, 1);
    ESMP2_TRY(contract(h, part, npart, c, len(c.A), len(c.B), 4.0, G, N * N, N + ov + 1, N, 1));
    // S3 boxes <- T2 (through the flip partner of T2: sg)
    const double sg = (double)d.sg;
    c = C(H11, 0, T2, 0); K(c, 0, (int)nd, 1, 1);
    ESMP2_TRY(contract(h, part, npart, c, len(c.A), len(c.B), sg * 1.0, G, N * N, ov, 0, 0));
    c = C(H12, 0, T2, 1); E(c, 0, v1, v1, 0);
    K(c, 0, no, sH12[0], sT2[0]); K(c, 1, no, sH12[1], sT2[1]); K(c, 2, v1, 1, 1);
    ESMP2_TRY(contract(h, part, npart, c, len(c.A), len(c.B), sg * 2.0, G, N * N, ov + 1, 1, 0));
    c = C(H21, 0, T2, sT2[1]); E(c, 0, o1, sH21[0], 0);
    K(c, 0, o1, sH21[1], sT2[1]); K(c, 1, nv * nv, 1, 1);
    ESMP2_TRY(contract(h, part, npart, c, len(c.A), len(c.B), sg * 2.0, G, N * N, N + ov, N, 0));
    c = C(H22, 0, T2, sT2[1] + 1); E(c, 0, o1, sH22[0], 0); E(c, 1, v1, v1, 0);
    K(c, 0, o1, sH22[1], sT2[1]); K(c, 1, v1, 1, 1);
    ESMP2_TRY(contract(h, part, npart, c, len(c.A), len(c.B), sg * 4.0, G, N * N, N + ov + 1, N, 1));
    // S3 boxes <- S~
    c = C(H11, 0, St, 0); E(c, 0, no, sT2[0], 0); E(c, 1, nv, nv, 0);
    K(c, 0, no, sT2[1], sT2[1]); K(c, 1, nv, 1, 1);
    ESMP2_TRY(contract(h, part, npart, c, len(c.A), len(c.B), 4.0, G, N * N, ov, N, 1));
    c = C(H12, 0, St, nv + 1); E(c, 0, no, sH12[0], 0);
    K(c, 0, no, sH12[1], sT2[1]); K(c, 1, v1, v1, nv); K(c, 2, v1, 1, 1);
    ESMP2_TRY(contract(h, part, npart, c, len(c.A), len(c.B), 4.0, G, N * N, ov, N, 0));
    c = C(H12, 0, St, nv); E(c, 0, no, sH12[0], 0); E(c, 1, v1, 1, 0);
    K(c, 0, no, sH12[1], sT2[1]); K(c, 1, v1, v1, nv);
    ESMP2_TRY(contract(h, part, npart, c, len(c.A), len(c.B), -4.0, G, N * N, ov + 1, N, 1));
    c = C(H21, 0, St, sT2[0] + sT2[1]); E(c, 0, nv, nv, 0);
    K(c, 0, o1, sH21[0], sT2[0]); K(c, 1, o1, sH21[1], sT2[1]); K(c, 2, nv, 1, 1);
    ESMP2_TRY(contract(h, part, npart, c, len(c.A), len(c.B), 4.0, G, N * N, ov, 1, 0));
    c = C(H21, 0, St, sT2[0]); E(c, 0, o1, sH21[1], 0); E(c, 1, nv, nv, 0);
    K(c, 0, o1, sH21[0], sT2[0]); K(c, 1, nv, 1, 1);
    ESMP2_TRY(contract(h, part, npart, c, len(c.A), len(c.B), -4.0, G, N * N, N + ov, N, 1));
    c = C(H22, 0, St, sT2[0] + sT2[1] + nv + 1);
    K(c, 0, o1, sH22[0], sT2[0]); K(c, 1, o1, sH22[1], sT2[1]); K(c, 2, v1, v1, nv); K(c, 3, v1, 1, 1);
    ESMP2_TRY(contract(h, part, npart, c, len(c.A), len(c.B), 4.0, G, N * N, ov, 0, 0));
    c = C(H22, 0, St, sT2[0] + nv + 1); E(c, 0, o1, sH22[1], 0);
    K(c, 0, o1, sH22[0], sT2[0]); K(c, 1, v1, v1, nv); K(c, 2, v1, 1, 1);
    ESMP2_TRY(contract(h, part, npart, c, len(c.A), len(c.B), -4.0, G, N * N, N + ov, N, 0));
    c = C(H22, 0, St, sT2[0] + sT2[1] + nv); E(c, 0, v1, 1, 0);
    K(c, 0, o1, sH22[0], sT2[0]); K(c, 1, o1, sH22[1], sT2[1]); K(c, 2, v1, v1, nv);
    ESMP2_TRY(contract(h, part, npart, c, len(c.A), len(c.B), -4.0, G, N * N, ov + 1, 1, 0));
    c = C(H22, 0, St, sT2[0] + nv); E(c, 0, o1, sH22[1], 0); E(c, 1, v1, 1, 0);
    K(c, 0, o1, sH22[0], sT2[0]); K(c, 1, v1, v1, nv);
    ESMP2_TRY(contract(h, part, npart, c, len(c.A), len(c.B), 4.0, G, N * N, N + ov + 1, N, 1));
  }
  // ---- 3. transposes of the right-hand side and of E2_S
  RhsAdjArgs ra{d, x, h->lam, GV, GM, Gf};
  hipLaunchKernelGGL(k_rhs_adj, dim3(nblk(d.off[7])), dim3(256), 0, s, ra);
  {
    const int* pv = h->pairs;
    E2sAdjArgs ea{d, h->Vint, h->lam, h->eo, h->ev, h->omega, pv, pv + d.npv, pv + d.npv + d.npv1,
                  pv + d.npv + d.npv1 + d.npo, GV, Gev, Geo, scal + 2};
    const int y1 = std::max(1, no - 1), x1 = std::max(1, 1024 / y1);
    const int y3 = std::min(1024, no * nv), x3 = std::max(1, 1024 / y3);
    hipLaunchKernelGGL(k_e2s_same_adj, dim3(x1, y1), dim3(256), 0, s, ea);
    hipLaunchKernelGGL(k_e2s_mixed_a_adj, dim3(x1, y1), dim3(256), 0, s, ea);
    hipLaunchKernelGGL(k_e2s_mixed_b_adj, dim3(x3, y3), dim3(256), 0, s, ea);
  }
  ESMP2_HIP(hipGetLastError());
  // ---- 4. chain to the factor blocks
  if (dB) {
    GemmArgs g{};
    // dBov = Bov (GV + GV^T)
    g.A = h->Bov; g.B = GV; g.C = dBov; g.M = na; g.N = nov; g.K = nov;
    g.sAi = nov; g.sAk = 1; g.sBk = nov; g.sBj = 1; g.sCi = nov; g.sCj = 1; g.alpha = 1.0; g.beta = 1.0;
    ESMP2_HIP(gemm(s, 1, g));
    g.sBk = 1; g.sBj = nov;
    ESMP2_HIP(gemm(s, 1, g));
    // dBov += X GM ; dX = Bov GM^T
    g.A = h->X; g.B = GM; g.sBk = nov; g.sBj = 1;
    ESMP2_HIP(gemm(s, 1, g));
    g.A = h->Bov; g.C = dX; g.sBk = 1; g.sBj = nov; g.beta = 0.0;
    ESMP2_HIP(gemm(s, 1, g));
    hipLaunchKernelGGL(k_make_x_adj, dim3(nblk((int64_t)na * nov)), dim3(256), 0, s, (const double*)dX,
                       (const double*)h->lam, no, nv, na, dBvt, dBoo);
    hipLaunchKernelGGL(k_fphi_adj, dim3(na), dim3(256), 0, s, (const double*)h->Bov, (const double*)h->Bvt,
                       (const double*)h->Boo, (const double*)h->lam, (const double*)Gf, no, nv, dBov, dBvt, dBoo);
    hipLaunchKernelGGL(k_grad_b_assemble, dim3(2048), dim3(256), 0, s, (const double*)dBov, (const double*)dBvt,
                       (const double*)dBoo, no, nv, na, dB);
  }
  // ---- 5. the Fock gradient
  if (dF)
    hipLaunchKernelGGL(k_grad_f_finish, dim3(nblk((int64_t)n * n)), dim3(256), 0, s, G, (const double*)h->lam,
                       (const double*)Gf, (const double*)Gev, (const double*)Geo, (const double*)scal, no, nv, dF);
  ESMP2_HIP(hipGetLastError());
  return ESMP2_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free variant of esmp2_fock_from_core: its intermediates live in
// one static device array per GPU.  Layout (doubles, n = n_occ + n_vir):
// gamma (n^2), K (n^2), the Coulomb weights d (n_aux), then the per-chunk
// GEMM intermediate T[p][Q][r] of FOCK_QCHUNK auxiliary indices (FOCK_QCHUNK n^2).
// ---------------------------------------------------------------------------
constexpr int FOCK_NMAX = 256, FOCK_AUXMAX = 16384, FOCK_QCHUNK = 16;
constexpr size_t FOCK_SCRATCH_DOUBLES =
    (size_t)2 * FOCK_NMAX * FOCK_NMAX + FOCK_AUXMAX + (size_t)FOCK_QCHUNK * FOCK_NMAX * FOCK_NMAX;   // 9.57 MB
static __device__ __align__(256) double scratch[FOCK_SCRATCH_DOUBLES];

// Device address of this GPU's copy of `scratch`, looked up once per device
// with that device current (the array's host-side name is not a device address).
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[64] = {};

static esmp2_status scratch_address(esmp2_handle h, double** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (h->device < 0 || h->device >= 64) return fail(h, ESMP2_INVALID_ARG, "device ordinal beyond 63");
  if (!g_scratch_ptr[h->device]) {
    void* p = nullptr;
    ESMP2_HIP(hipSetDevice(h->device));
    ESMP2_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[h->device] = (double*)p;
  }
  *out = g_scratch_ptr[h->device];
  return ESMP2_OK;
}

extern "C" {

esmp2_status esmp2_fock_from_core_noalloc(esmp2_handle h, int n_occ, int n_vir, int n_aux, const double* hcore,
                                          const double* B, const double* C, double* F_out) {
  if (!h) return ESMP2_INVALID_ARG;
  if (!hcore || !B || !C || !F_out) return fail(h, ESMP2_INVALID_ARG, "null pointer");
  if (n_occ < 1 || n_vir < n_occ || n_aux < 1)
    return fail(h, ESMP2_INVALID_ARG, "need 1 <= n_occ <= n_vir and n_aux >= 1");
  if (n_occ + n_vir > FOCK_NMAX || n_aux > FOCK_AUXMAX)
    return fail(h, ESMP2_INVALID_ARG, "sizes beyond the static workspace: n_occ + n_vir <= 256, n_aux <= 16384");
  ESMP2_HIP(hipSetDevice(h->device));
  double* ws = nullptr;
  {
    const esmp2_status st = scratch_address(h, &ws);
    if (st != ESMP2_OK) return st;
  }
  const int n = n_occ + n_vir;
  const int64_t nn = (int64_t)n * n;
  hipStream_t s = h->stream;
  double* gam = ws;
  double* K = gam + nn;
  double* d = K + nn;
  double* T = d + n_aux;
  hipLaunchKernelGGL(k_ref_density, dim3(nblk(nn)), dim3(256), 0, s, C, n_occ, n_vir, gam);
  hipLaunchKernelGGL(k_coulomb_weights, dim3(n_aux), dim3(256), 0, s, B, (const double*)gam, n, d);
  // K[p][q] = sum_Q sum_r (B[Q] gamma)[p][r] B[Q][r][q], FOCK_QCHUNK auxiliary
  // indices at a time; the first chunk writes K (beta = 0), so nothing in the
  // workspace needs clearing
  for (int q0 = 0; q0 < n_aux; q0 += FOCK_QCHUNK) {
    const int qc = std::min(FOCK_QCHUNK, n_aux - q0);
    GemmArgs g{};
    g.A = B + (int64_t)q0 * nn; g.B = gam; g.C = T; g.M = n; g.N = n; g.K = n;
    g.sAb = nn; g.sAi = n; g.sAk = 1; g.sBb = 0; g.sBk = n; g.sBj = 1;
    g.sCb = n; g.sCi = (int64_t)qc * n; g.sCj = 1; g.alpha = 1; g.beta = 0;
    ESMP2_HIP(gemm_native(s, qc, g));      // the hand-written kernel: no library workspace
    g = GemmArgs{};
    g.A = T; g.B = B + (int64_t)q0 * nn; g.C = K; g.M = n; g.N = n; g.K = qc * n;
    g.sAi = (int64_t)qc * n; g.sAk = 1; g.sBk = n; g.sBj = 1; g.sCi = n; g.sCj = 1; g.alpha = 1;
    g.beta = q0 == 0 ? 0.0 : 1.0;
    ESMP2_HIP(gemm_native(s, 1, g));
  }
  hipLaunchKernelGGL(k_fock_combine, dim3(nblk(nn)), dim3(256), 0, s, hcore, B, (const double*)d, (const double*)K, n,
                     n_aux, F_out);
  ESMP2_HIP(hipGetLastError());
  return ESMP2_OK;
}

esmp2_status esmp2_fock_from_core(esmp2_handle h, int n_occ, int n_vir, int n_aux, const double* hcore,
                                  const double* B, const double* C, double* F_out) {
  if (!h) return ESMP2_INVALID_ARG;
  if (!hcore || !B || !C || !F_out) return fail(h, ESMP2_INVALID_ARG, "null pointer");
  if (n_occ < 1 || n_vir < n_occ || n_aux < 1 || n_occ + n_vir > 256)
    return fail(h, ESMP2_INVALID_ARG, "need 1 <= n_occ <= n_vir, n_aux >= 1, n_occ + n_vir <= 256");
  ESMP2_HIP(hipSetDevice(h->device));
  const int n = n_occ + n_vir;
  const int64_t nn = (int64_t)n * n;
  hipStream_t s = h->stream;
  double *gam = nullptr, *d = nullptr, *T = nullptr, *K = nullptr;
  auto cleanup = [&]() {
    if (gam) (void)hipFree(gam);
    if (d) (void)hipFree(d);
    if (T) (void)hipFree(T);
    if (K) (void)hipFree(K);
  };
  if (hipMalloc(&gam, sizeof(double) * nn) != hipSuccess || hipMalloc(&d, sizeof(double) * n_aux) != hipSuccess ||
      hipMalloc(&T, sizeof(double) * nn * n_aux) != hipSuccess || hipMalloc(&K, sizeof(double) * nn) != hipSuccess) {
    cleanup();
    return fail(h, ESMP2_OOM, "device allocation failed");
  }
  hipLaunchKernelGGL(k_ref_density, dim3(nblk(nn)), dim3(256), 0, s, C, n_occ, n_vir, gam);
  hipLaunchKernelGGL(k_coulomb_weights, dim3(n_aux), dim3(256), 0, s, B, (const double*)gam, n, d);
  // T[p][Q][r] = (B[Q] gamma)[p][r]
  GemmArgs g{};
  g.A = B; g.B = gam; g.C = T; g.M = n; g.N = n; g.K = n;
  g.sAb = nn; g.sAi = n; g.sAk = 1; g.sBb = 0; g.sBk = n; g.sBj = 1;
  g.sCb = n; g.sCi = (int64_t)n_aux * n; g.sCj = 1; g.alpha = 1; g.beta = 0;
  hipError_t e1 = gemm(s, n_aux, g);
  // K[p][q] = sum_{Q, r} T[p][Q][r] B[Q][r][q]
  g = GemmArgs{};
  g.A = T; g.B = B; g.C = K; g.M = n; g.N = n; g.K = n_aux * n;
  g.sAi = (int64_t)n_aux * n; g.sAk = 1; g.sBk = n; g.sBj = 1; g.sCi = n; g.sCj = 1; g.alpha = 1; g.beta = 0;
  hipError_t e2 = gemm(s, 1, g);
  hipLaunchKernelGGL(k_fock_combine, dim3(nblk(nn)), dim3(256), 0, s, hcore, B, (const double*)d, (const double*)K, n,
                     n_aux, F_out);
  hipError_t e3 = hipStreamSynchronize(s);
  hipError_t e4 = hipGetLastError();
  cleanup();
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess)
    return fail(h, ESMP2_HIP_ERROR, "HIP error in esmp2_fock_from_core");
  return ESMP2_OK;
}

}  // extern "C"
