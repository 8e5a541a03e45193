/*
 * libmm -- modal and Cholesky theta-methods for eddy-current transients on
 * one MI355X (gfx950), FP64 throughout.
 *
 * The problem follows the Galerkin circuit system of Ventre, Chiariello,
 * Isernia, Mottola, Tamburrino, "Modal Decomposition in Numerical
 * Computation of Eddy Current Transients" (arXiv 2407.11993), Sec. 3.1,
 * eqs. discrete_version_1a/b:
 *
 *     R I + L dI/dt + E^T phi = V0 + VD,        E I = iD,
 *
 * with L the dense SPD inductance matrix, R the sparse SPD resistance matrix,
 * E the reduced electrode incidence ((Ne-1) x N, Sec. 3.1 eq. definition_E),
 * and V0 = -M0 di0/dt for solenoidal sources with mutual inductances M0
 * (Sec. 3.1, eq. induced_voltages_0).  Currents injected at electrodes are
 * handled by the paper's split I = K Ii + E^T (E E^T)^{-1} iD
 * (eq. current_electrodes), K an orthonormal basis of ker E.
 *
 * Conventions
 *   - Every array argument is a DEVICE pointer unless stated otherwise.
 *     Dense matrices are column-major.  The caller owns its inputs and
 *     outputs; the library copies what it keeps.
 *   - Calls are ordered on the context's HIP stream and may return before
 *     the work completes, like any stream-ordered call.  Calls that must
 *     inspect a device-side result (the factorisation pivots, the
 *     eigensolver's convergence) synchronise that stream.
 *   - Status codes are returned synchronously; mm_last_error() gives the text.
 *   - One context per host thread.
 *   - Waveforms are sampled at t_k = k dt, k = 0..n_steps, row-major by step:
 *     i_src[k * n_src + c], i_D[k * (Ne-1) + a].  Each step call continues
 *     from the state left by the previous one (I(0) = 0 after setup or reset).
 */
#ifndef MM_H
#define MM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MM_OK = 0,
  MM_E_INVALID = 1,     /* bad argument or unsupported size */
  MM_E_NOMEM = 2,       /* device allocation failed */
  MM_E_NOT_SPD = 3,     /* a Cholesky pivot was not positive (index in message) */
  MM_E_NO_CONVERGE = 4, /* a secular equation did not converge */
  MM_E_STATE = 5,       /* call out of order (e.g. step_modal before decompose) */
  MM_E_DEVICE = 6       /* a HIP runtime call failed */
} mm_status;

typedef struct mm_ctx mm_ctx;

/* The problem statement (Sec. 3.1).  All pointers are device pointers.
 * Every floating-point input must be finite (MM_E_INVALID otherwise). */
typedef struct {
  int64_t n;                /* unknowns N */
  const double* xyz;        /* when L is NULL: n x 3, row i = centre of cell i
                               (row-major); L_ij = h / sqrt(|x_i - x_j|^2 + h^2)
                               is then generated on the device (an SPD stand-in
                               of the inductance matrix, Sec. 3.1 L_jk), and no
                               dense copy of L is ever stored */
  double h;                 /* kernel width, > 0 (used with xyz only) */
  int64_t r_nnz;            /* R: symmetric positive definite, CSR, n x n */
  const int64_t* r_rowptr;  /* n + 1 */
  const int32_t* r_col;     /* r_nnz, sorted per row */
  const double* r_val;      /* r_nnz */
  int32_t n_e;              /* electrodes Ne: 0, or >= 2 */
  int64_t e_nnz;            /* E: (Ne-1) x n CSR, full row rank */
  const int64_t* e_rowptr;
  const int32_t* e_col;
  const double* e_val;
  int32_t n_src;            /* solenoidal sources (columns of M0), 0..4096 */
  const double* M0;         /* n x n_src, column-major */
  int32_t n_probe;          /* probe rows, 1..4096 */
  const double* P;          /* n x n_probe, column-major: column p is probe
                               row p; signal_p = P(:,p)^T dI/dt */
  const double* L;          /* NULL, or the inductance matrix itself (Sec. 3.1,
                               the Galerkin L_jk of eq. discrete_version_1a):
                               n x n, column-major with leading dimension ldl,
                               symmetric positive definite.  Only its lower
                               triangle is read.  BORROWED: the library reads it
                               at setup (electrode reduction), at every
                               decomposition and at every Cholesky
                               factorisation, and never writes it, so it must
                               stay valid and unchanged until mm_destroy.  xyz
                               and h are then ignored.  It costs 8 n^2 bytes of
                               device memory beside the library's own buffers
                               (the projected decomposition holds one n0^2
                               buffer). */
  int64_t ldl;              /* leading dimension of L, >= n */
} mm_problem;

/* Copy the problem to the device and prepare the context.  `stream` is a
 * hipStream_t (NULL = the default stream).  On success *out owns all device
 * memory the library allocates for this problem.  With electrodes (Ne >= 2)
 * this also builds the reduced problem of Sec. 3.1 (eqs. discrete_version_2,
 * circuit_equations_v2): K is the Householder complement of im E^T, and
 * K^T L K, K^T R K, R_D, L_D, K^T M0 and the probe weights are formed on the
 * device.  MM_E_INVALID if E is not of full row rank, or if
 * 2 (Ne - 1) + n_src > 8. */
mm_status mm_setup(const mm_problem* problem, void* stream, mm_ctx** out);

/* The one-off modal decomposition (Sec. 3.2, eq. generalized_eigenvalues_
 * discrete: Li v = tau Ri v, lam = 1 / tau), taken from the resistance side:
 * Ri = F F^T with F = H A^{1/2}, H the banded (block-bidiagonal) Cholesky
 * factor of R's block of the kept unknowns and A = I + Z S Z^T the electrodes'
 * low-rank correction; C' = F^{-1} Li F^{-T} = Q' T Q'^T (two-stage
 * tridiagonalisation + divide and conquer); the pencil's Li-normalised
 * eigenvectors V = F^{-T} Q' T^{-1/2} (V^T Li V = I, V^T Ri V = Lam, the V_n of
 * eq. modal_decomposition_discrete), columns by ascending lam, and the
 * projections V^T [F, P] of the sources and probes onto the modes.  No dense
 * factorisation of L.  Independent of theta and dt.  Device memory: at most
 * two and a half n0^2 buffers at any time (C', then Q' beside it while the
 * merges use C's storage); only V (n0^2) is kept afterwards.  Synchronises the
 * stream.  Errors: MM_E_INVALID when R's bandwidth in the given numbering
 * exceeds 8192; MM_E_NOT_SPD when R's block or Ri is not positive definite,
 * or Li is not (a time constant <= 0); MM_E_NO_CONVERGE; MM_E_NOMEM. */
mm_status mm_decompose(mm_ctx* ctx);

/* The decomposition as the modal signals need it (Sec. 3.2 feeding Sec. 3.3.2):
 * the eigenvalues and the projected source and probe weights
 * T^{-1/2} Q'^T F^{-1} [F, P], without forming the eigenvector matrix Q'.
 * Q' = Q1 Q2 Z is applied to the few columns only: Q1^T panel by panel after
 * the band reduction, Q2^T by every bulge-chase task as it generates its
 * reflector, Z^T by one product after divide and conquer.  Afterwards
 * mm_step_modal, mm_eigenvalues and mm_batch_* work as after mm_decompose;
 * mm_probe(MM_MODAL) and mm_adjoint_modal return MM_E_STATE (they need V).
 * Up to 32 forcing columns (2 (Ne-1) + n_src) and probes in all ride along
 * the bulge chase; with more (Sec. 4.4 observes 301 points) the chase keeps
 * its reflectors (half an n0^2 buffer beside C') and Q2^T is applied to the
 * columns afterwards.  Synchronises the stream.  Errors: those of
 * mm_decompose. */
mm_status mm_decompose_projected(mm_ctx* ctx);

/* The modal theta-method (Sec. 3.3.2) for n_steps steps:
 *   (1 + theta dt lam_n) dy_n = -dt lam_n y_n + (modal forcing)_n.
 * The forcing is the Cholesky method's right-hand side (Sec. 3.3.1,
 * eq. time_integration) written in the modal basis.  signal (n_steps x
 * n_probe, row-major by step) receives P^T (I^{k+1} - I^k) / dt for
 * k = 0..n_steps-1.  i_src: (n_steps+1) x n_src; i_D: (n_steps+1) x (Ne-1)
 * or NULL when Ne = 0.  Requires mm_decompose.  theta in [0, 1], dt > 0.
 * Up to 8 probes the probe sums are reduced inside the stepping kernel; with
 * more (Sec. 4.4 observes 301 points) the steps run in chunks whose
 * amplitude increments dY (n0 x L, at most 2 GiB) are written out and
 * projected as one matrix product P~^T dY; the signal is the same up to the
 * order of the sums.  This holds for mm_step_modal_exact,
 * mm_step_modal_selective (without MM_STEP_SCAN) and mm_step_cholesky
 * (current increments, P^T dI) too. */
mm_status mm_step_modal(mm_ctx* ctx, double theta, double dt, int64_t n_steps,
                        const double* i_src, const double* i_D, double* signal);

/* mm_step_modal without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, state, signal and errors as
 * mm_step_modal, and the same kernels; the probe partial sums live in a
 * file-scope device array of 2^23 doubles (64 MiB) that every GPU the
 * library runs on holds until the process ends.  Limits: at most 8 probes,
 * and n_steps * ceil(n0 / 256) * n_probe <= 2^23 per call (MM_E_INVALID
 * otherwise; longer runs are several calls, the state continues).  All calls
 * on one GPU share its array: calls that overlap in time on one GPU (two
 * streams, two host threads) race. */
mm_status mm_step_modal_noalloc(mm_ctx* ctx, double theta, double dt, int64_t n_steps,
                                const double* i_src, const double* i_D, double* signal);

/* Exact integration of the decoupled modal equations (Sec. 3.2, eq.
 * modal_decomposition_discrete), the analytical route Sec. 3.3 leaves to
 * later work: every source waveform is taken linear between its samples
 * (first-order hold), so on step k each mode obeys y' + lam y = e1 + e2 s/dt
 * and is advanced in closed form,
 *   y^{k+1} = exp(-lam dt) y^k + beta e1 + gamma e2,
 *   beta = (1 - exp(-x)) / x, gamma = (1 - beta) / x, x = lam dt.
 * No time-step error for such waveforms; the cost per step is that of
 * mm_step_modal.  Arguments, state, signal and errors as mm_step_modal
 * (dt > 0); the two may be mixed on one state. */
mm_status mm_step_modal_exact(mm_ctx* ctx, double dt, int64_t n_steps,
                              const double* i_src, const double* i_D, double* signal);

/* The modal stepping of mm_step_modal (exact = 0, theta in [0, 1]) or of
 * mm_step_modal_exact (exact != 0, theta ignored), parallel in time, for
 * few modes and many steps: every mode's step is the affine map
 * y -> A y + b_k, so the steps are cut into chunks that run from a zero state
 * in parallel, are chained by A^L per mode, and run again from their start
 * states (twice the mode-steps, (N/256) x (T/L) workgroups instead of N/256).
 * Same arguments, state, signal (to rounding) and errors as those calls; at
 * most 65535 x 2^16 steps and 8 probes.  Allocates 2 T/L N doubles of
 * workspace. */
mm_status mm_step_modal_scan(mm_ctx* ctx, double theta, int32_t exact, double dt,
                             int64_t n_steps, const double* i_src, const double* i_D,
                             double* signal);

/* Selective solution of the decoupled modal equations (Sec. 3.2: each
 * scalar equation can be solved on its own, so only a chosen subset need
 * be).  Mode n is kept when its coupling score
 *   score_n = max_j |W(n, j)| * max_p |P~(n, p)|
 * (W the modal forcing weights of the columns [R_D | L_D | K^T M0], P~ the
 * modal probe weights; every source counts with unit amplitude) exceeds
 * tol times the largest score.  tol = 0 drops only modes with no forcing or
 * no probe weight, which cannot change a probe signal; a larger tol drops
 * weakly coupled modes, an approximation.  The score weights the columns
 * neither by the run's waveforms (R_D is driven by dt i_D, the others by
 * increments) nor by 1/lambda_n, so for tol > 0 it is a heuristic whose
 * reach depends on the units of the sources and electrodes and on dt.  With degenerate eigenvalues the
 * eigensolver's basis of each eigenspace decides which of its modes carry
 * the coupling, so the kept count can differ between eigensolvers while the
 * signals agree.
 * *n_kept (host) receives the count; kept (device, n0 entries, or NULL)
 * receives the kept mode indices in ascending eigenvalue order.  The kept set
 * gets its own state, taken from the modal state at this call (zero after
 * mm_reset_state); the full modal state, the reconstruction and the adjoint
 * are not affected.  Synchronises the stream.  Requires mm_decompose or
 * mm_decompose_projected (a new decomposition discards the selection);
 * MM_E_INVALID for tol < 0, not finite, or n_kept NULL. */
mm_status mm_select_modes(mm_ctx* ctx, double tol, int64_t* n_kept, int64_t* kept);

/* mm_step_modal (theta in [0, 1]), or mm_step_modal_exact with
 * MM_STEP_EXACT in flags (theta ignored), on the modes kept by
 * mm_select_modes only, from the kept set's own state; with MM_STEP_SCAN
 * the steps run parallel in time as in mm_step_modal_scan (same signal to
 * rounding), which pays off when few modes are kept for many steps.
 * Arguments, signal and errors as those calls, MM_E_INVALID for unknown
 * flags, and MM_E_STATE before mm_select_modes.  mm_reset_state zeroes this
 * state too. */
#define MM_STEP_EXACT 1u
#define MM_STEP_SCAN 2u
mm_status mm_step_modal_selective(mm_ctx* ctx, double theta, uint32_t flags, double dt,
                                  int64_t n_steps, const double* i_src, const double* i_D,
                                  double* signal);

/* Steady-state phasors of the probe signals under sinusoidal sources, from
 * the decomposition (Sec. 3.2, eq. modal_decomposition_discrete; the
 * frequency-domain comparison of Sec. 4.6): with i0_c(t) = Re{A_c e^{jwt}}
 * and iD_a(t) = Re{D_a e^{jwt}} every mode has the phasor
 *   y_n = (W u(w))_n / (lam_n + j w),
 * u: -D on the R_D columns, -j w D on the L_D columns, -j w A on the source
 * columns, and the probe signal P dI/dt has the phasor
 *   S_p(w) = j w (Pt^T y + P A_D D)_p.
 * O(N) per frequency instead of a complex factorisation of R + j w L.
 * All pointers are device memory; complex numbers are (re, im) pairs:
 * omega (n_w, rad per unit time), amp_src (n_w x n_src pairs, row-major by
 * frequency; NULL when n_src = 0), amp_D (n_w x (Ne-1) pairs; NULL when
 * Ne = 0), out (n_w x n_probe pairs).  Requires mm_decompose or
 * mm_decompose_projected; ordered on the context's stream.  Errors:
 * MM_E_STATE before the decomposition, MM_E_INVALID for missing arrays, more
 * than 8 forcing columns or probes, or n_w > 65535. */
mm_status mm_modal_phasors(mm_ctx* ctx, int64_t n_w, const double* omega,
                           const double* amp_src, const double* amp_D, double* out);

/* The classical theta-method (Sec. 3.3.1, eq. time_integration): the
 * factor Z = Li + theta dt Ri = C C^T is computed on the first call and
 * whenever theta or dt change; each step does one forward and one backward
 * substitution.  Same arguments and outputs as mm_step_modal.  Synchronises
 * the stream when it (re)factors.  Errors: MM_E_NOT_SPD. */
mm_status mm_step_cholesky(mm_ctx* ctx, double theta, double dt, int64_t n_steps,
                           const double* i_src, const double* i_D,
                           double* signal);

#define MM_MODAL 0
#define MM_CHOLESKY 1

/* Reconstruction of the current (Sec. 3.1, eq. current_electrodes):
 * I = K Ii + E^T (E E^T)^{-1} iD, with Ii = V y for the modal state.
 * rows == NULL: out (n) receives I.  Otherwise rows is n x n_rows
 * (column-major) and out (n_rows) receives rows^T I. */
mm_status mm_probe(mm_ctx* ctx, int32_t which, int32_t n_rows,
                   const double* rows, double* out);

/* Set both states back to I = 0. */
mm_status mm_reset_state(mm_ctx* ctx);

/* Checkpoint and restart of one method's time stepping (Sec. 3.3: every step
 * continues from the state the previous one left).  The state is n doubles
 * (device): the method's reduced unknowns, n0 of them (which = MM_MODAL: the
 * modal amplitudes y; MM_CHOLESKY: the reduced currents Ii), followed by the
 * Ne - 1 injected currents of its last step.  The reduced unknowns depend on
 * the basis of ker E and, for MM_MODAL, on the decomposition, so a state is
 * meaningful only for a context of the same problem (and, for MM_MODAL, the
 * same decomposition).  The selective stepper's own state is not included.
 * mm_get_state: MM_E_STATE for MM_MODAL before a decomposition and for
 * MM_CHOLESKY before its first step; mm_set_state: MM_E_STATE for MM_MODAL
 * before a decomposition.  Stream-ordered copies. */
mm_status mm_get_state(mm_ctx* ctx, int32_t which, double* out);
mm_status mm_set_state(mm_ctx* ctx, int32_t which, const double* in);

/* Eigenvalues lam_n = 1/tau_n of the reduced pencil, ascending (n0 doubles,
 * device).  Requires mm_decompose. */
mm_status mm_eigenvalues(mm_ctx* ctx, double* out);

/* ---- Batched modal runs ----------------------------------------------------
 * Many independent runs of the modal theta-method (Sec. 3.3.2) in one launch:
 * run r drives source src[r] (a column of M0) with its own waveform and
 * observes probe probe[r] (a column of P), from a zero state, for lens[r]
 * steps; injected currents are zero.  One mode group of one run per
 * workgroup; every thread keeps its modes in registers for the whole run.
 *   lens, src, probe: HOST arrays of n_runs entries.
 *   waves:   device, packed waveforms: run r's samples at t_k = k dt,
 *            k = 0..lens[r], start at sum_{q<r} (lens[q] + 1).
 *   signals: device, packed outputs: run r's lens[r] samples start at
 *            sum_{q<r} lens[q]; s^{k+1} = P(:, probe)^T dI^k / dt as for
 *            mm_step_modal.
 *   tile:    -1 = autotune (each workgroup shape is timed on the batch cut
 *            to 256 steps per run, the fastest kept), or an index 0..5 into
 *            the library's tile list (threads x modes per thread:
 *            256x1, 256x2, 256x4, 128x4, 256x8, 128x8).
 * The plan keeps the waves and signals pointers: mm_batch_run replays one
 * captured HIP graph (stepping launch + signal pass) on the context's
 * stream; refill `waves` in place between runs.  Requires mm_decompose;
 * the plan must be destroyed before its context. */
typedef struct mm_batch mm_batch;
mm_status mm_batch_create(mm_ctx* ctx, double theta, double dt, int32_t n_runs,
                          const int64_t* lens, const int32_t* src, const int32_t* probe,
                          const double* waves, double* signals, int32_t tile,
                          mm_batch** out);
mm_status mm_batch_run(mm_batch* batch);
/* out[0] = threads per workgroup, out[1] = modes per thread, out[2] = mode
 * groups per run, out[3] = total steps (sum of lens). */
mm_status mm_batch_info(const mm_batch* batch, int64_t* out);
void mm_batch_destroy(mm_batch* batch);

/* ---- Adjoint -----------------------------------------------------------------
 * Gradient of the probe-signal misfit
 *     J = sum_r sum_{k=0}^{n_steps-1} (s_r^{k+1} - s_obs[r * n_steps + k])^2
 * over n_runs modal runs (Sec. 3.3.2) that share one source waveform i_src
 * (device, n_steps + 1 samples): run r drives source src[r] and observes
 * probe probe[r] (HOST arrays), from a zero state.  The modal recursion is
 * run backward (the exact adjoint of the theta-method of Sec. 3.3.1 in the
 * modal basis); amplitudes are checkpointed every ckpt_every steps and
 * recomputed per segment, so memory grows with n_steps / ckpt_every, not
 * n_steps.  Outputs (device): *J; dJ_dR (r_nnz): dJ/dR at every stored entry
 * of R, each entry treated as independent (for a symmetric model R(rho) the
 * chain rule adds both triangles); dJ_di (n_steps + 1): dJ/d i_src(t_k).
 * Requires mm_decompose and Ne = 0.  Synchronises the stream. */
mm_status mm_adjoint_modal(mm_ctx* ctx, double theta, double dt, int64_t n_steps,
                           int32_t n_runs, const int32_t* src, const int32_t* probe,
                           const double* i_src, const double* s_obs, int64_t ckpt_every,
                           double* J, double* dJ_dR, double* dJ_di);

/* Sizes: out[0] = n, out[1] = n0 = n - (Ne-1), out[2] = decomposed (0/1). */
mm_status mm_info(const mm_ctx* ctx, int64_t* out /* host, 3 */);

void mm_destroy(mm_ctx* ctx);

/* Text of the last error on this context (or of the last mmk_ call on this
 * thread when ctx is NULL). */
const char* mm_last_error(const mm_ctx* ctx);

/* ------------------------------------------------------------------------
 * Dense building blocks, exposed for the stage-by-stage tests.  Device
 * pointers, column-major, ordered on `stream`; workspaces are allocated and
 * freed inside each call (which therefore synchronises the stream).
 * ------------------------------------------------------------------------ */

/* C = alpha op(A) op(B) + beta C on the FP64 matrix cores. */
mm_status mmk_dgemm(int32_t trans_a, int32_t trans_b, int64_t m, int64_t n,
                    int64_t k, double alpha, const double* A, int64_t lda,
                    const double* B, int64_t ldb, double beta, double* C,
                    int64_t ldc, void* stream);

/* mmk_dgemm with structure the product skips work for:
 *   MMK_LOWER    only C's lower triangle (i >= j) is computed and written;
 *   MMK_A_LOWER  op(A) is lower triangular, MMK_A_UPPER upper triangular;
 *   MMK_B_LOWER  op(B) is lower triangular;
 *   b_band >= 0  op(B)(l, j) = 0 for l > j + b_band (-1: no band).
 * The zero parts of op(A) and op(B) must be stored as zeros: whole 16-wide
 * k-slices are skipped where a tile's rows or columns have only zeros, the
 * rest is read as stored. */
#define MMK_LOWER 1
#define MMK_A_LOWER 2
#define MMK_A_UPPER 4
#define MMK_B_LOWER 8
mm_status mmk_dgemm_tri(int32_t trans_a, int32_t trans_b, int64_t m, int64_t n,
                        int64_t k, double alpha, const double* A, int64_t lda,
                        const double* B, int64_t ldb, double beta, double* C,
                        int64_t ldc, int32_t flags, int64_t b_band, void* stream);

/* C = alpha A B + beta C with A (m x m) symmetric, only its lower triangle
 * read; B and C are m x n. */
mm_status mmk_dsymm_lower(int64_t m, int64_t n, double alpha, const double* A,
                          int64_t lda, const double* B, int64_t ldb, double beta,
                          double* C, int64_t ldc, void* stream);

/* A = G G^T (lower, in place, strict upper triangle zeroed); *info (host)
 * = -1 or the first non-positive pivot.  (The factorisation of Sec. 3.3.1
 * and of Li in Sec. 3.2.) */
mm_status mmk_dpotrf(int64_t n, double* A, int64_t lda, int64_t* info,
                     void* stream);

/* A <- A^{-1} for lower-triangular A. */
mm_status mmk_dtrtri(int64_t n, double* A, int64_t lda, void* stream);

/* Band reduction C = Q1 B Q1^T (1 <= nb <= 64): A is symmetric and only its
 * lower triangle is read; that triangle is overwritten (the upper one is left
 * as it was); AB (ldab x n, ldab >= 2 nb + 1) receives the lower band,
 * AB(d, j) = B(j+d, j). */
mm_status mmk_dsy2sb(int64_t n, double* A, int64_t lda, int32_t nb, double* AB,
                     int64_t ldab, void* stream);

/* Band to tridiagonal by bulge chasing (1 <= nb <= 64): d (n), e (n-1). */
mm_status mmk_dsb2st(int64_t n, int32_t nb, double* AB, int64_t ldab, double* d,
                     double* e, void* stream);

/* Tridiagonal divide and conquer: w (n, ascending), Z (n x n, ld n). */
mm_status mmk_dstedc(int64_t n, const double* d, const double* e, double* w,
                     double* Z, void* stream);

/* Full symmetric eigensolver: A (full symmetric, destroyed) = Z diag(w) Z^T,
 * w ascending, Z (n x n, ld n). */
mm_status mmk_dsyevd(int64_t n, double* A, int64_t lda, int32_t nb, double* w,
                     double* Z, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MM_H */
