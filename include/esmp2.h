/*
 * esmp2.h -- C ABI of the MI355X (gfx950) hot path of N^5 excited-state-specific
 * second-order perturbation theory (ESMP2-TOP(1), singlet).
 *
 * The calls follow the paper's statement of the problem:
 *   1. rotate the ESMF reference to the transition-orbital-pair (TOP) basis
 *      (Sec. II.A: SVD of the singles coefficients, C = U Lambda V^T, and the
 *      occupied-occupied / virtual-virtual rotations that make the reference a
 *      sum of n_occ pair excitations);
 *   2. build the right-hand side b = Q V |Psi0> = Q H |Psi0> on the first-order
 *      space of doubles and L-triples (Sec. II.B, Eq. for Psi1 and the triples
 *      matrix element) and the directly inverted S-triple energy (Sec. II.D);
 *   3. apply sigma = (H0 - E0) x, the modified zeroth-order Hamiltonian
 *      (Sec. II.C, the Q F Q replacement: full Fock operator on doubles +
 *      L-triples);
 *   4. solve Q (H0 - E0) Q Psi1 = -Q V Psi0 by preconditioned conjugate
 *      gradient (Sec. III.A) and return E2 = <Psi0|V|Psi1>.
 *
 * Conventions
 *   - Orbitals: n_occ occupied then n_vir virtual spatial orbitals, N = n_occ+n_vir.
 *   - Hamiltonian input: the Fock matrix F (of the reference's one-body density)
 *     and a factor B with (pq|rs) = sum_Q B[Q][p][q] B[Q][r][s]; the one-electron
 *     operator is h = F - G[gamma(Psi0)].
 *   - Reference: Psi0 = sum_ia C[i][a] (E^up_ai + E^dn_ai)/sqrt(2) |Phi>, singlet,
 *     ||C||_F = 1.
 *   - Large TOPs (paper Sec. II.C): the n_top TOPs of the largest singular values
 *     are "large"; the L-triples are the triples containing a large TOP (spatial
 *     occupied l among the holes and spatial virtual l' among the particles).
 *     n_top = 1 is ESMP2-TOP(1), the default and fast path; n_top = n_occ is
 *     TOP(all).
 *   - TOP basis: singular values in descending order; the TOP virtual of occupied
 *     l is virtual l; the remaining virtuals (AVOs) diagonalise the Fock matrix in
 *     their span (ascending).  Every occupied TOP orbital and AVO is signed so that
 *     its largest-magnitude coefficient in the input basis is positive; a TOP
 *     virtual takes the sign that makes its singular value positive.
 *   - Amplitude layout ("seven boxes", t = occupied 0, t' = virtual 0), each box
 *     contiguous in this order, occupied pair outer, virtual pair inner, pairs
 *     written "(p<q)" packed row-major over the strict upper triangle:
 *       0 T2   (i<j),(a<b)                 a+_{a u} a+_{b u} a_{j u} a_{i u}|Phi>
 *       1 S2   i,j,a,b (dense)             a+_{a u} a+_{b d} a_{j d} a_{i u}|Phi>
 *       2 T3L  (j<k) in 1..,(b<c) in 1..   a+_{t'u}a+_{b u}a+_{c u}a_{k u}a_{j u}a_{t u}|Phi>
 *       3 H1P1 (j<k),(b<c)                 a+_{t'u}a+_{b d}a+_{c d}a_{k d}a_{j d}a_{t u}|Phi>
 *       4 H1P2 (j<k), a in 1.., c in 1..   a+_{a u}a+_{t'd}a+_{c d}a_{k d}a_{j d}a_{t u}|Phi>
 *       5 H2P1 i in 1..,k in 1..,(b<c)     a+_{t'u}a+_{b d}a+_{c d}a_{k d}a_{t d}a_{i u}|Phi>
 *       6 H2P2 i,k in 1.., a,c in 1..      a+_{a u}a+_{t'd}a+_{c d}a_{k d}a_{t d}a_{i u}|Phi>
 *     (u/d = spin up/down).  Boxes other than S2 stand for a spin-flip pair of
 *     determinants (inner-product weight 2); S2 entries are single determinants
 *     (weight 1) and enter the operator flip-symmetrised.
 *   - With n_top = k > 1 the vector holds the boxes above (set 0, TOP t = 0) and
 *     then, for each further large TOP s = 1 .. k-1, the five L-boxes 2..6 again
 *     with TOP s in place of TOP 0 (occupied orbitals 0 and s swapped, virtuals
 *     0' and s' swapped in the operator strings): set s starts at
 *     box_offsets[2] + s (box_offsets[7] - box_offsets[2]).  A triple that
 *     contains a larger TOP r < s is stored in set r only; its slot in set s is
 *     masked (always zero).
 *
 * Memory and streams
 *   - A handle is bound to one device and one stream at creation.  All work is
 *     ordered on that stream; calls return after queueing unless they return
 *     host scalars (documented per call), in which case they synchronise it.
 *   - Pointers marked "device" must be device memory of the handle's device.
 *     The caller keeps ownership of every pointer it passes; the handle owns
 *     its internal copies and work buffers (released by esmp2_destroy).
 *   - A handle is not thread safe.
 *
 * Errors: every call returns esmp2_status; no exception crosses the ABI and
 * nothing aborts.  esmp2_last_error() returns a message for the last failure.
 */
#ifndef ESMP2_H
#define ESMP2_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct esmp2_handle_* esmp2_handle;

typedef enum {
  ESMP2_OK = 0,
  ESMP2_INVALID_ARG = 1,    /* bad size, null pointer, NaN/Inf input, n_vir < n_occ */
  ESMP2_BAD_ORDER = 2,      /* call sequence violated (e.g. sigma before rotate)   */
  ESMP2_NOT_SPD = 3,        /* a diagonal denominator <= 0 or p.Ap <= 0 in CG       */
  ESMP2_NOT_CONVERGED = 4,  /* max_iter reached; result holds the partial state     */
  ESMP2_OOM = 5,            /* device allocation failed                              */
  ESMP2_HIP_ERROR = 6,      /* a HIP runtime call failed                             */
  ESMP2_UNSUPPORTED = 7     /* option not implemented for these sizes / this mode    */
} esmp2_status;

typedef enum {
  ESMP2_FP64 = 0,           /* FP64 everywhere                                       */
  ESMP2_FP32 = 1,           /* the operator in FP32 (FP32 inputs, Fock blocks rounded
                               to FP32, FP32 matrix-core accumulation)               */
  ESMP2_BF16 = 2            /* the FP32 operator except that the virtual-pair Fock
                               products (the Sylvester part) take BF16 operands: F'
                               and the amplitudes are rounded to BF16 (nearest even)
                               on the way into the matrix cores, which accumulate in
                               FP32.  FP32 vectors.  TOP basis only, padded virtual
                               dimension 80, 112 or 160 (else ESMP2_UNSUPPORTED).  In
                               a solve: FP64 iterative refinement around inner solves
                               with this operator (inner_tol 0 selects 1e-2)       */
} esmp2_precision;

typedef enum {
  ESMP2_BASIS_TOP = 0,            /* solve in the TOP basis                           */
  ESMP2_BASIS_SEMICANONICAL = 1   /* solve after rotating the occupied orbitals other
                                     than t and the virtuals other than t' so that their
                                     Fock blocks are diagonal ("pinned semicanonical")   */
} esmp2_basis;

typedef struct {
  double tol;               /* stop when ||b + A x||_W / ||b||_W <= tol (e.g. 1e-8)   */
  int max_iter;             /* conjugate-gradient iteration cap                      */
  int precision;            /* esmp2_precision of the solve: FP64, or FP32 / BF16
                               inner solves inside FP64 iterative refinement         */
  const double* x0;         /* device, n_amp, initial guess (warm start) or NULL      */
  double* x_out;            /* device, n_amp, receives the solution, or NULL          */
  double* resid_hist;       /* host, max_iter entries of ||r||/||b|| per iteration, or NULL
                               (FP32: the inner residual estimate times the outer one) */
  double inner_tol;         /* FP32 / BF16: smallest relative residual reduction asked of
                               one inner FP32 solve, in [0, 1); 0 selects 1e-5         */
  int basis;                /* esmp2_basis of the Krylov solve (results are the same) */
} esmp2_solve_opts;

typedef struct {
  double e2;                /* E2 = e2_dl + e2_s                                      */
  double e2_dl;             /* doubles + L-triples part, Hylleraas form b.x - x.r     */
  double e2_s;              /* directly inverted S-triples part                       */
  double e0;                /* E0 = <Psi0|F|Psi0>                                     */
  double rel_resid;         /* final ||b + A x||_W / ||b||_W                          */
  int iterations;           /* conjugate-gradient iterations (all inner ones in FP32) */
  int outer;                /* refinement steps (FP32 / BF16 precision), 0 otherwise  */
  int status;               /* esmp2_status of the solve                              */
} esmp2_solve_result;

/* Create a handle on `device`, ordering all work on `stream` (a hipStream_t,
 * NULL = the default stream).  *out receives the handle. */
esmp2_status esmp2_create(esmp2_handle* out, int device, void* stream);

/* Release the handle and all device memory it owns.  NULL is accepted. */
esmp2_status esmp2_destroy(esmp2_handle h);

/* Bind a problem (copies the inputs; the caller keeps ownership).
 *   F: device, N x N row-major, symmetric (the Fock matrix, input orbital basis)
 *   B: device, n_aux x N x N row-major, B[Q][p][q] == B[Q][q][p]
 *   C: device, n_occ x n_vir row-major, ||C||_F = 1
 *   spin: 0 = singlet reference, 1 = the M_s = 0 component of the triplet
 *         (paper Sec. II.A: the beta singles enter Psi0 with the opposite
 *         sign; the first-order amplitudes are then antisymmetric under the
 *         flip of every spin)
 *   n_top: number of large TOPs, 1 <= n_top <= n_occ (else ESMP2_INVALID_ARG).
 *         n_top > 1 (ESMP2-TOP(k), up to TOP(all)) applies the operator by a
 *         generic determinant-level kernel, O(N_o + N_v) per amplitude, and
 *         supports the solve in the TOP basis (FP64, or FP64 refinement around
 *         the same operator on FP32 vectors), esmp2_sigma (FP64 or FP32),
 *         esmp2_build_rhs and esmp2_export_determinants; BF16, the
 *         pinned-semicanonical basis and the gradient return
 *         ESMP2_UNSUPPORTED.
 * Requires 2 <= n_occ <= n_vir, n_aux >= 1.  Checks F, B, C for NaN/Inf
 * (synchronises the stream).  Resets any previous problem. */
esmp2_status esmp2_set_problem(esmp2_handle h, int n_occ, int n_vir, int n_aux,
                               const double* F, const double* B, const double* C,
                               int spin, int n_top);

/* Bind a problem stated in the TOP basis already (paper Sec. II.A: the basis in
 * which the singles coefficients are diagonal), for a caller that holds the
 * rotated quantities, e.g. to differentiate E2 with respect to them:
 *   Ft: device, N x N row-major, symmetric: the TOP-basis Fock matrix, occupied
 *       orbitals first (t = occupied 0), then the virtuals (t' = virtual 0, the
 *       partner of occupied l is virtual l for l < n_occ)
 *   Bt: device, n_aux x N x N row-major, symmetric in its orbital pair
 *   lam: device or host, n_occ singular values, lam[0] the largest, all >= 0,
 *        sum lam^2 = 1 (within 1e-10)
 *   spin: 0 singlet, 1 triplet (as in esmp2_set_problem)
 * Copies the inputs (the caller keeps ownership), checks them for NaN/Inf and
 * synchronises.  esmp2_rotate_top then keeps the basis as given (identity
 * rotation, lambda_out reports lam); everything else is as after
 * esmp2_set_problem.  Resets any previous problem. */
esmp2_status esmp2_set_problem_top(esmp2_handle h, int n_occ, int n_vir, int n_aux,
                                   const double* Ft, const double* Bt, const double* lam, int spin);

/* Rotate to the TOP basis (paper Sec. II.A).  lambda_out: host, n_occ doubles
 * (descending singular values) or NULL; when non-NULL the call synchronises. */
esmp2_status esmp2_rotate_top(esmp2_handle h, double* lambda_out);

/* Size of the amplitude vector and the start offsets of the seven boxes;
 * box_offsets has 8 entries (box_offsets[7] == *n_amp for n_top = 1; for n_top
 * = k > 1, *n_amp = box_offsets[2] + k (box_offsets[7] - box_offsets[2]) and
 * the offsets are those of set 0).  Either may be NULL. */
esmp2_status esmp2_space(esmp2_handle h, int64_t* n_amp, int64_t* box_offsets);

/* Right-hand side b_mu = <mu|H|Psi0> on the seven boxes, E0 and the
 * S-triple energy E2_S = -sum_S b^2/D (paper Sec. II.B-II.D).
 *   b_out: device, n_amp doubles, or NULL.  For n_top = 1 the TOP-basis b and
 *   Jacobi diagonal are formed when b_out, a TOP-basis solve or the gradient
 *   first needs them (a semicanonical solve builds its own b from the same
 *   integral factors).
 *   e0, e2_s: host scalars or NULL.  The call synchronises the stream (the
 *   denominator check: the smallest denominator, from the orbital energies).  E2_S is summed on the handle's side stream, beside
 *   the solve that follows; a non-NULL e2_s waits for it, with NULL it is
 *   waited for only by esmp2_solve, whose result reports it.
 * Returns ESMP2_NOT_SPD if a denominator of the first-order space is <= 0. */
esmp2_status esmp2_build_rhs(esmp2_handle h, double* b_out, double* e0, double* e2_s);

/* y = (H0 - E0) x on doubles + L-triples (paper Sec. II.C).
 *   x, y: device, n_amp elements each (double for ESMP2_FP64, float for
 *   ESMP2_FP32 and ESMP2_BF16); x and y must not overlap.  Requires
 *   esmp2_rotate_top.  ESMP2_BF16 returns ESMP2_UNSUPPORTED unless the padded
 *   virtual dimension is 80, 112 or 160. */
esmp2_status esmp2_sigma(esmp2_handle h, const void* x, void* y, int precision);

/* y = (H0 - E0) x in a chosen basis of the first-order space (paper Sec. II.C;
 * doubles + L-triples are mapped onto themselves by every rotation of the
 * occupied orbitals other than t and of the virtuals other than t', Sec. II.B).
 *   basis = ESMP2_BASIS_TOP: esmp2_sigma.
 *   basis = ESMP2_BASIS_SEMICANONICAL: x and y are amplitudes of the pinned-
 *     semicanonical basis: occupied orbitals 1.. rotated by the eigenvectors of
 *     F~_oo[1:,1:] and virtuals 1.. by those of F~_vv[1:,1:] (t and t' fixed;
 *     eigenvalues ascending, each eigenvector signed so that its largest-
 *     magnitude component is positive; new orbital P' = sum_P T[P][P'] P).  In
 *     that basis the two Fock blocks are diagonal and the operator is applied
 *     by the O(n_occ^2 n_vir^2) arrow kernels; its diagonal constants omega and
 *     kappa stay those of the TOP basis.  The first such call after
 *     esmp2_rotate_top builds the rotation and the operator blocks.
 *   x, y: device, n_amp elements (double for ESMP2_FP64, float for ESMP2_FP32;
 *   ESMP2_BF16 is ESMP2_UNSUPPORTED in the semicanonical basis), not
 *   overlapping.  Requires esmp2_rotate_top.  Queued on the handle's stream. */
esmp2_status esmp2_sigma_basis(esmp2_handle h, const void* x, void* y, int precision, int basis);

/* Determinant coefficients of an amplitude vector (paper Sec. II.B: Psi1 over
 * the M_s = 0 doubles and triples of the closed shell; reading: canonical
 * phase with the alpha string first, then the beta string, each ascending).
 *   x: device, n_amp doubles, amplitudes of the TOP basis (e.g. esmp2_solve's
 *      x_out)
 *   coeff: device, n doubles; det_key: device, n int64; n >= 2 n_amp - n_S2
 *      (n_S2 = box_offsets[2] - box_offsets[1]).  Entries 0 .. n_amp-1 hold the
 *      determinant of every stored amplitude in layout order, entries n_amp ..
 *      2 n_amp - n_S2 - 1 the spin-flip partner of every amplitude outside S2
 *      in layout order (S2 stores both members of each flip pair, so each S2
 *      determinant appears once, with the flip-symmetrised amplitude
 *      (x + sg x_partner)/2, sg = +1 singlet, -1 triplet; a flip partner
 *      outside S2 carries sg x).  Coefficient = phase of the amplitude's
 *      operator string (the layout table above) in the canonical order, times
 *      the amplitude.  With n_top > 1, n_amp is the TOP(k) size and a masked
 *      slot writes key -1 and coefficient 0 in both of its entries.
 *   det_key: the determinant as its excitation from the closed shell: holes in
 *      bits 0-29 and particles in bits 30-59, 10 bits per spin-orbital, each
 *      group ascending, 1023 in the unused third slots of a double.
 *      Spin-orbital numbering: alpha orbital p -> p, beta p -> N + p; spatial
 *      orbitals: occupied 0 .. n_occ-1, then the virtuals (virtual a -> n_occ + a).
 * Requires esmp2_set_problem (any later state).  Queued on the handle's stream;
 * does not synchronise. */
esmp2_status esmp2_export_determinants(esmp2_handle h, const double* x, double* coeff, int64_t* det_key,
                                       int64_t n);

/* Jacobi-preconditioned conjugate gradient for A x = -b (A = H0 - E0 on D + L,
 * weighted inner product), then E2 (paper Sec. III.A and Sec. II.C).  Builds the
 * right-hand side first if esmp2_build_rhs has not been called.  Synchronises.
 * With precision = ESMP2_FP32 (or ESMP2_BF16: the same with the BF16 operator,
 * TOP basis only), iterative refinement: the FP64 residual
 * r = -b - A x is recomputed with the FP64 operator after each inner solve
 * A d = r / ||r|| run by FP32 conjugate gradient (FP32 operator and vectors, FP64
 * reductions) to a relative reduction max(inner_tol, tol / (2 ||r||/||b||)); the
 * FP64 x accumulates ||r|| d.  The stopping test, x and E2 are FP64 in both modes;
 * result.iterations counts the inner iterations and result.outer the FP64 steps.
 * basis = ESMP2_BASIS_SEMICANONICAL: doubles + L-triples are mapped onto
 * themselves by any rotation of the occupied orbitals other than t and of the
 * virtuals other than t' (Sec. II.B: an L-triple keeps t and t'), so the
 * operator is covariant and E2 unchanged; the solve runs after the rotation
 * that diagonalises those two Fock blocks, where the Jacobi preconditioner is
 * close to the operator.  The rotation's eigenproblems are solved by
 * esmp2_rotate_top on the side stream; the first such solve after build_rhs
 * forms the operator blocks and builds b in the new basis from the rotated
 * integral factors and singles amplitudes.  In FP64 the conjugate gradient
 * decides convergence on the device and the host reads each iteration's
 * outcome one iteration behind (one extra, empty iteration is queued after
 * the last); from x0 = NULL with tol < 1 the kernel that builds b also forms
 * the start (r = -b, its preconditioned copy and their two dots) and the host
 * reads nothing before the first iteration.  From x0 = NULL without x_out no x
 * is formed: E2_DL is the Hylleraas value of the iterates accumulated from the
 * solve's scalars, -sum_i alpha_i rho_i (for conjugate gradient from zero
 * <b, p_i>_W = -rho_i and <x_k, r_k>_W = 0; equal to the value from x to
 * rounding).  In both bases x0 and x_out are amplitudes of the TOP basis
 * (rotated on the way in and out). */
esmp2_status esmp2_solve(esmp2_handle h, const esmp2_solve_opts* opts,
                         esmp2_solve_result* result);

/* Derivatives of E2 (paper Sec. II.C-II.D) with respect to the TOP-basis Fock
 * matrix F~ and factor B~, with the rotation and lam held fixed.  E2_DL is the
 * stationary value of 2 <b, x>_W + <x, A x>_W at the solution x of A x = -b; A is
 * symmetric, so the adjoint solution is x itself and
 *   dE2 = 2 <x, db>_W + <x, dA x>_W + dE2_S       (x held fixed),
 * evaluated without a second solve.
 *   x: device, n_amp doubles: the TOP-basis solution (esmp2_solve's x_out) of the
 *      problem whose right-hand side was built last; its accuracy bounds the
 *      gradient's (the error is first order in the residual)
 *   dF: device, N x N, or NULL; dB: device, n_aux x N x N, or NULL (not both).
 * Both outputs are symmetric and hold G with dE2 = sum_pq G[p][q] dF[p][q] for
 * every symmetric perturbation (per auxiliary index for B~); entries that E2
 * does not depend on are zero.  Requires esmp2_build_rhs.  Allocates a
 * workspace on first use (about 8 n_occ^2 n_vir^2 + 2 (n_occ n_vir)^2 doubles,
 * kept by the handle) and queues the work on the handle's stream without
 * synchronising.  The scatter steps use FP64 atomic adds, so the last bits
 * may differ between runs. */
esmp2_status esmp2_gradient(esmp2_handle h, const double* x, double* dF, double* dB);

/* The Fock operator of the reference's one-body density (paper Sec. II.C: the
 * zeroth-order Hamiltonian uses the Fock operator of Psi0's density), for a
 * caller that holds the one-electron operator instead of F:
 *   F = h + G[gamma],  G[g]_pq = sum_rs g_rs ((pq|rs) - (ps|rq)/2),
 *   gamma = spin-summed density of Psi0: 2 - C C^T (occupied block), C^T C
 *   (virtual block), zero between them; (pq|rs) = sum_Q B[Q][p][q] B[Q][r][s].
 * hcore (N x N), B (n_aux x N x N), C (n_occ x n_vir), F_out (N x N): device,
 * row-major, input orbital basis.  Allocates and frees temporary device memory
 * (about n_aux N^2 doubles) and synchronises.  Needs a handle (for its device
 * and stream) but no problem bound to it; F_out can then go to
 * esmp2_set_problem. */
esmp2_status esmp2_fock_from_core(esmp2_handle h, int n_occ, int n_vir, int n_aux, const double* hcore,
                                  const double* B, const double* C, double* F_out);

/* Allocation-free form of esmp2_fock_from_core, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, result and layout; the
 * intermediates (the density, the exchange matrix, the Coulomb weights and a
 * 16-auxiliary-index chunk of the exchange GEMM) live in a static workspace
 * of 9.57 MB per GPU that the library holds until the process ends, so it
 * calls no allocator.  Limits: n_occ + n_vir <= 256 and n_aux <= 16384, else
 * ESMP2_INVALID_ARG.  Queued on the handle's stream; does not synchronise.
 * Every call on one GPU shares that GPU's workspace: calls that overlap on
 * one GPU (two streams, or two host threads) race and must be ordered by the
 * caller.  Nothing in the workspace needs to start at zero. */
esmp2_status esmp2_fock_from_core_noalloc(esmp2_handle h, int n_occ, int n_vir, int n_aux, const double* hcore,
                                          const double* B, const double* C, double* F_out);

/* Batched workload: n independent states, one handle each (esmp2_set_problem
 * done, every handle on its own stream for the states to overlap on the
 * device).  For every handle: rotation, right-hand side, solve with `opts`,
 * E2 into results[i] (host array of n).  A pool of n_threads host threads
 * (<= 0: 8) takes the states in order for their set-up, issued on each
 * state's stream.  With opts->precision ESMP2_FP64, opts->basis
 * ESMP2_BASIS_SEMICANONICAL, one large TOP per state and every handle on one
 * device, the conjugate gradients of all states then run together on the
 * first handle's stream: one launch per step covers every state, each state's
 * scalars, convergence test and stop (tol, max_iter) are decided on the
 * device, and the host reads only the number of states still iterating; the
 * results equal each state's own esmp2_solve to rounding (the reductions are
 * split over fewer blocks).  Any other options: each thread runs
 * esmp2_solve for its states.  opts->x0, x_out and resid_hist must be NULL.
 * Synchronises.  Every state is attempted; returns ESMP2_OK or the status of
 * the first failing state (results[i].status holds each one).  Temporary
 * device memory: one record of about 1 KB per state. */
esmp2_status esmp2_solve_batch(esmp2_handle* handles, int n, const esmp2_solve_opts* opts,
                               esmp2_solve_result* results, int n_threads);

/* C = A B for row-major FP64 matrices (A: m x k, B: k x n, C: m x n, all device),
 * on the matrix cores, queued on the handle's stream.  This is the dense GEMM the
 * library uses for the TOP-basis rotation and the integral blocks; it is exported
 * so that its operand layout can be validated directly. */
esmp2_status esmp2_gemm_f64(esmp2_handle h, int m, int n, int k, const double* A, const double* B, double* C);

/* Timing of the virtual-pair Sylvester kernel (the dominant sigma kernel) with
 * HIP events recorded on the handle's stream around each of its launches.
 * vv_ms[3], vv_launches[3] (host, indexed by esmp2_precision) receive the
 * accumulated milliseconds and launch counts since the last call, which are then
 * reset; recording is switched on (enable != 0) or off.  Waits for the recorded
 * events.  Either output may be NULL. */
esmp2_status esmp2_profile(esmp2_handle h, int enable, double* vv_ms, int64_t* vv_launches);

/* Variants of the virtual-pair Sylvester products (the dominant sigma kernel):
 *   0  the specialised kernel: one batch matrix per workgroup of 8 wavefronts
 *      with balanced tile lists (padded virtual dimension 80, 112 or 160; the
 *      only variant with BF16 operands)
 *   1..5  the generic kernel with output blocks of 32 v x 32 v per workgroup
 * Without a choice, a handle uses the variant esmp2_autotune recorded for its
 * (n_occ, n_vir, precision) in this process, else 0 where available, else
 * min((mv / 16 + 1) / 2, 5) (mv = n_vir rounded up to 16). */
#define ESMP2_SYLVESTER_VARIANTS 6

/* Autotuner: times every available variant on this handle's problem (`reps`
 * launches each after one warm-up, HIP events on the handle's stream, on a
 * zero input in the handle's own work vectors), records the fastest for
 * (n_occ, n_vir, precision) for every handle of the process, and clears this
 * handle's own choice so that the recorded one applies.  Synchronises.
 *   variant_out: host, the fastest variant, or NULL
 *   ms_out: host, ESMP2_SYLVESTER_VARIANTS average milliseconds per launch
 *           (-1 for a variant not available at this size), or NULL
 * Requires esmp2_rotate_top; reps in [1, 1000]; ESMP2_UNSUPPORTED for BF16 at
 * a size without the specialised kernel. */
esmp2_status esmp2_autotune(esmp2_handle h, int precision, int reps, int* variant_out, double* ms_out);

/* Fix the variant of one precision for this handle (-1: automatic, as above).
 * ESMP2_INVALID_ARG for a variant not available at this size and precision. */
esmp2_status esmp2_set_sylvester_variant(esmp2_handle h, int precision, int variant);

/* Message of the last failing call on this handle (never NULL). */
const char* esmp2_last_error(esmp2_handle h);

#ifdef __cplusplus
}
#endif
#endif /* ESMP2_H */
