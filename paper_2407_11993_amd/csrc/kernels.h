// Launchers of the libmm kernels (internal; the public interface is mm.h).
#pragma once
#include "common.h"

namespace mm {

// ---- dense factorisations (potrf.hip) ------------------------------------
int64_t potrf_ws_elems(int64_t n);
// A = G G^T in place (lower; the strict upper triangle is zeroed).  The first
// failing pivot (global index) is atomically min-ed into *d_status, which the
// caller initialises to INT64_MAX.
void potrf_lower(double* A, int64_t lda, int64_t n, double* ws, int64_t ws_elems,
                 int64_t* d_status, hipStream_t s);
int64_t trtri_ws_elems(int64_t n);
// A <- A^{-1} for lower-triangular A (strict upper triangle zero on entry).
void trtri_lower(double* A, int64_t lda, int64_t n, double* ws, int64_t ws_elems,
                 hipStream_t s);
// Inverses of the nb x nb diagonal blocks of lower-triangular A (strict
// upper triangle zero), packed as ceil(n/nb) blocks of nb*nb (column-major,
// zero padded).  ws: trtri_ws_elems(nb) doubles.
void diag_block_inverses(const double* A, int64_t lda, int64_t n, int nb,
                         double* Dinv, double* ws, int64_t ws_elems, hipStream_t s);
void copy_matrix(const double* S, int64_t lds, double* D, int64_t ldd,
                 int64_t m, int64_t n, hipStream_t s);

// ---- setup (setup.hip) -----------------------------------------------------
// Sparse matrix in CSR form.  The logical matrix is the stored one with its
// first `off` rows and columns dropped: logical entry (i, j) is stored entry
// (i + off, j + off); `rows` counts logical rows.
struct Csr {
  int64_t rows = 0, cols = 0, nnz = 0;
  int64_t off = 0;
  const int64_t* rowptr = nullptr;
  const int32_t* col = nullptr;
  const double* val = nullptr;
};
// Symmetric low-rank term  U Yc^T + Yc U^T  with Yc = Y1 + w2 Y2 (Y2 may be
// null); U, Y1, Y2 are n x m column-major with leading dimension ld.
struct LowRank {
  const double* U = nullptr;
  const double* Y1 = nullptr;
  const double* Y2 = nullptr;
  double w2 = 0.0;
  int64_t ld = 0;
  int m = 0;
};
// Where the inductance matrix comes from: a borrowed dense matrix (its lower
// triangle, column-major with leading dimension ld) or, when L is null, the
// smooth kernel h / sqrt(|x_i - x_j|^2 + h^2) of the cell centres xyz (n x 3,
// row-major).  Logical entry (i, j) is entry (i + off, j + off): off = m
// selects the trailing block the electrode reduction keeps.
struct LSrc {
  const double* xyz = nullptr;
  double h = 0.0;
  const double* L = nullptr;
  int64_t ld = 0;
  int64_t off = 0;
};
// out(i, j) = L(i, j) - (U Yc^T + Yc U^T)_ij for i >= j (lower triangle +
// diagonal), or the full matrix if `full`.
void assemble_L(const LSrc& src, int64_t n, double* out, int64_t ld, bool full,
                hipStream_t s, const LowRank& lr = LowRank{});
// *d_flag = 1 if one of count doubles at p (or, for the _lower form, an entry
// of the lower triangle of the n x n matrix A) is NaN or infinite; the flag
// is left unchanged otherwise.
void flag_nonfinite(const double* p, int64_t count, int64_t* d_flag, hipStream_t s);
void flag_nonfinite_lower(const double* A, int64_t lda, int64_t n, int64_t* d_flag,
                          hipStream_t s);
// Z(i,j) += alpha R(i,j) for the lower-triangle entries of R.
void add_csr_lower(double* Z, int64_t ld, double alpha, const Csr& R, hipStream_t s);
// max_j (j - min{c : R(c,j) != 0}) over the stored rows of symmetric R (an
// upper bound for the logical matrix of any offset), written to *d_out.
void csr_lower_band(const Csr& R, int64_t* d_out, hipStream_t s);
// W = A R for dense A (n x n, column-major) and symmetric sparse R.
void dense_times_csr(const double* A, int64_t lda, const Csr& R, double* W,
                     int64_t ldw, hipStream_t s);
// A(i,j) = A(j,i) for i < j (copy the lower triangle to the upper).
void symmetrize_from_lower(double* A, int64_t lda, int64_t n, hipStream_t s);
void fill(double* p, int64_t count, double v, hipStream_t s);
void fill_i64(int64_t* p, int64_t count, int64_t v, hipStream_t s);

// ---- the resistance side of the pencil (band.hip) -------------------------
// Block size (a multiple of 64, >= 64) for R's bandwidth `band`.
int64_t band_block(int64_t band);
// R (logical, n x n, lower band <= Bb) = H H^T with H block lower bidiagonal
// in blocks of Bb: Hinv receives the inverses of the diagonal blocks, Hs the
// sub-diagonal blocks (nblk = ceil(n / Bb) blocks of Bb x Bb each).  The
// first failing pivot (local to its block) is min-ed into *d_status (left
// INT64_MAX if none); MM_E_INVALID if an entry lies outside the band.
int64_t band_factor_ws_elems(int Bb);
void band_factor(const Csr& R, int64_t n, int Bb, double* Hinv, double* Hs, double* ws,
                 int64_t ws_elems, int64_t* d_status, hipStream_t s);
// X <- H^{-1} X and X <- H^{-T} X (X n x ncols; tmp Bb x ncols doubles),
// X <- X H^{-T} (X nrows x n; tmp nrows x Bb doubles).
void band_solve_left(const double* Hinv, const double* Hs, int64_t n, int Bb, double* X,
                     int64_t ldx, int64_t ncols, double* tmp, hipStream_t s);
void band_solve_left_t(const double* Hinv, const double* Hs, int64_t n, int Bb, double* X,
                       int64_t ldx, int64_t ncols, double* tmp, hipStream_t s);
void band_solve_right_t(const double* Hinv, const double* Hs, int64_t n, int Bb, double* X,
                        int64_t ldx, int64_t nrows, double* tmp, hipStream_t s);
// Gamma (2m x 2m) with (I + Z S Z^T)^{-1/2} = I + Z Gamma Z^T from Gz = Z^T Z,
// S = -[[0, I_m], [I_m, 0]]; *d_bad = 1 if I + Z S Z^T is not definite.
void lowrank_gamma(const double* Gz, int m, double* Gamma, int64_t* d_bad, hipStream_t s);
// K = Gamma Qm Gamma / 2 (k x k, k <= 8)
void lowrank_gqg(const double* Gamma, const double* Qm, int k, double* K, hipStream_t s);
// From the time constants tau (ascending) and ZY (n0 x (nf + np)):
// lam_n = 1 / tau_r, W(n, :) = tau_r^{-1/2} ZY(r, :nf), P(n, :) likewise, r = n0-1-n.
void modes_from_tau(const double* tau, const double* ZY, int64_t n0, int nf, int np,
                    double* lam, double* W, double* P, hipStream_t s);
// In place: X(:, n) <- tau_r^{-1/2} X(:, r), r = n0-1-n; lam_n = 1 / tau_r.
void reverse_scale_cols(double* X, int64_t ld, int64_t n0, const double* tau, double* lam,
                        hipStream_t s);

// ---- electrode reduction (electrode.hip) ----------------------------------
// Householder QR of E^T for the m x n electrode matrix E (CSR, m <= 8):
// E^T = H [Re; 0] with H = H_0 ... H_{m-1} = I - V T V^T.  Writes V (n x m,
// unit diagonal, zero above it), small = [T | Re^{-T}] (two m x m blocks,
// column-major) and *d_status = 1 if E is rank deficient.  work: n m doubles.
void electrode_qr(const Csr& E, int64_t n, int m, double* V, double* small, double* work,
                  int64_t* d_status, hipStream_t s);
// X <- H X (trans false) or H^T X for X (n x k, ld ldx).  ws: apply_h_ws_elems.
int64_t apply_h_ws_elems(int m, int64_t k);
void apply_h(const double* V, const double* T, int64_t n, int m, double* X, int64_t ldx,
             int64_t k, bool trans, double* ws, int64_t ws_elems, hipStream_t s);
// Y = X T - 1/2 V (T^T V^T X T) for X = A V: then H^T A H = A - V Y^T - Y V^T.
void two_sided_y(const double* V, const double* T, int64_t n, int m, const double* X,
                 double* Y, double* ws, int64_t ws_elems, hipStream_t s);
// out (n x k) = L U for the inductance matrix of src, U non-zero only on rows idx.
void l_times_rows(const LSrc& src, int64_t n, const int32_t* idx, int ns,
                  const double* U, int64_t ldu, int k, double* out, int64_t ldo,
                  hipStream_t s);
// out (R.rows x k) = R U (logical R, offset honoured), k <= 8.
void csr_times_dense(const Csr& R, const double* U, int64_t ldu, int k, double* out,
                     int64_t ldo, hipStream_t s);
// z = [Rinv^T iD ; Ii]  (m + n0 entries)
void electrode_lift(const double* RinvT, const double* iD, int m, const double* Ii,
                    int64_t n0, double* z, hipStream_t s);
// mark[i] = 1 if row i of A (rows x k) or of B has a non-zero entry.
void mark_rows(const double* A, const double* B, int64_t ld, int64_t rows, int k,
               unsigned char* mark, hipStream_t s);
// D (ns x k) = rows idx of S (ld lds)
void gather_rows(const double* S, int64_t lds, const int32_t* idx, int ns, int k, double* D,
                 hipStream_t s);

// Sparse low-rank part of the reduced resistance, R_i = R'' - V Y^T - Y V^T
// with V, Y non-zero only on the rows idx (ns of them): Vs, Ys are ns x m.
struct RLowRank {
  int ns = 0, m = 0;
  const int32_t* idx = nullptr;
  const double* Vs = nullptr;
  const double* Ys = nullptr;
};

// ---- Cholesky theta-method (step_chol.hip) --------------------------------
// Block size of the triangular solves for order n (256 .. 2048), and
// the number of probe partial sums they produce per step.
int trsv_block(int64_t n);
int64_t trsv_parts(int64_t n);


struct Forcing {
  // f^k = F u^k with F (n0 x nf, column-major) and u^k from the waveforms:
  //   u_a         = -dt (iD_a^k + theta (iD_a^{k+1} - iD_a^k))   a < m
  //   u_{m+a}     = -(iD_a^{k+1} - iD_a^k)                       a < m
  //   u_{2m+c}    = -(i0_c^{k+1} - i0_c^k)                       c < n_src
  const double* F = nullptr;
  int nf = 0, m = 0, n_src = 0;
  const double* i_src = nullptr;  // (T+1) x n_src, row-major by step
  const double* i_D = nullptr;    // (T+1) x m
};

struct CholStep {
  int64_t n0 = 0;
  const double* pf = nullptr;  // forward panels (trsv_prescale)
  const double* pb = nullptr;  // backward panels (trsv_prescale)
  int B = 128;                 // block size (trsv_block(n0))
  const double* Dinv = nullptr;  // inverses of the B x B diagonal blocks of the factor
  const double* DinvT = nullptr; // the same blocks transposed
  int64_t* kstep = nullptr;    // device step counter and its per-step copy (two int64)
  bool use_graph = true;       // replay one captured step per time step
  Csr Ri;                      // reduced resistance, sparse part
  RLowRank Rlr;                // reduced resistance, low-rank part (electrodes)
  Forcing f;
  double theta = 0.5, dt = 1.0;
  double* I = nullptr;         // state Ii (n0)
  double* b = nullptr;         // work vector (n0)
  double* y = nullptr;         // work vector (n0)
  const double* Pt = nullptr;  // probe weights (n0 x n_probe, column-major)
  int n_probe = 0;
  double* probe_partial = nullptr;  // n_steps x trsv_parts(n0) x n_probe
  // many probes: with n_probe = 0 and dI_out set, step k writes its
  // increment dI to column k of dI_out (n0 x n_steps)
  double* dI_out = nullptr;
};
void chol_steps(const CholStep& c, int64_t k0, int64_t n_steps, hipStream_t s);
// Once per factorisation: with C the factor (lower, leading dimension n) and
// D_J^{-1} = Dinv (block J), form the forward panels W_IK = D_I^{-1} C_IK and
// the backward panels V_KJ = C_KJ D_J^{-1} in row-contiguous layout (pf, pb;
// trsv_panel_elems doubles in all).
int64_t trsv_panel_elems(int64_t n, int B);
void trsv_prescale(const double* Cf, int64_t n, int B, const double* Dinv, double* pf,
                   double* pb, hipStream_t s);
// DinvT(block b) = Dinv(block b)^T for nblocks blocks of B x B.
void transpose_blocks(const double* Dinv, int64_t nblocks, int B, double* DinvT,
                      hipStream_t s);
// signal(k, p) = (sum_j probe_partial(k, j, p) + sum_a Pd(p, a) diD_a^k) / dt
void probe_finish(const double* probe_partial, int64_t n_steps, int64_t nparts,
                  int n_probe, const double* Pd, int m, const double* i_D,
                  int64_t k0, double dt, double* signal, hipStream_t s);

// ---- modal theta-method (step_modal.hip) ----------------------------------
struct ModalStep {
  int64_t n0 = 0;
  const double* lam = nullptr;   // n0
  const double* W = nullptr;     // modal forcing weights (n0 x nf)
  Forcing f;                     // F unused; nf, m, n_src and waveforms used
  const double* Pt = nullptr;    // modal probe weights (n0 x n_probe)
  int n_probe = 0;
  double theta = 0.5, dt = 1.0;
  bool exact = false;            // exact per-mode integration instead of theta
  double* y = nullptr;           // modal amplitudes (state)
  double* probe_partial = nullptr;  // n_steps x n_groups x n_probe
  // many probes: with n_probe = 0 and dy_out set, the steps write the
  // amplitude increments instead (n0 x n_steps, column k = step k), whose
  // projection P~^T dY is then one matrix product
  double* dy_out = nullptr;
};
int modal_groups(int64_t n0);

// Steady-state probe phasors for sinusoidal sources (phasor.hip).  Complex
// numbers are (re, im) pairs; amp_src n_w x n_src, amp_D n_w x m, out
// n_w x n_probe, all row-major by frequency; partial holds
// n_w x phasor_groups(n0) x n_probe pairs.
struct ModalPhasor {
  int64_t n0 = 0;
  const double* lam = nullptr;   // n0
  const double* W = nullptr;     // n0 x (2m + n_src): R_D, L_D, source columns
  const double* Pt = nullptr;    // n0 x n_probe
  const double* PD = nullptr;    // n_probe x m (direct electrode term), or nullptr
  int m = 0, n_src = 0, n_probe = 0;
  int64_t n_w = 0;
  const double* omega = nullptr;    // n_w
  const double* amp_src = nullptr;  // n_w x n_src pairs
  const double* amp_D = nullptr;    // n_w x m pairs
  double* partial = nullptr;
  double* out = nullptr;            // n_w x n_probe pairs
};
// Selective modal stepping (select.hip): score[n] = max_j |W(n, j)| *
// max_p |Pt(n, p)| (W n0 x nf, Pt n0 x np, ld n0); idx (n0 entries) receives
// the modes with score > tol * max score in ascending order, count[0] their
// number.  gather_modes copies the kept modes' lam, W and Pt rows and state
// into compact arrays of leading dimension nk.
void select_modes(const double* W, int nf, const double* Pt, int np, int64_t n0, double tol,
                  double* score, int64_t* idx, int64_t* count, hipStream_t s);
void gather_modes(const int64_t* idx, int64_t nk, int64_t n0, const double* lam, const double* W,
                  int nf, const double* Pt, int np, const double* y, double* lam_s, double* W_s,
                  double* Pt_s, double* y_s, hipStream_t s);

int64_t phasor_groups(int64_t n0);
void modal_phasors(const ModalPhasor& mp, hipStream_t s);
void modal_steps(const ModalStep& m, int64_t k0, int64_t n_steps, hipStream_t s);
// The same steps cut into chunks of L steps run in parallel (few modes, many
// steps); ws holds 2 ceil(n_steps / L) n0 doubles.  scan_chunk picks L.
int64_t scan_chunk(int64_t n0, int64_t n_steps);
void modal_steps_scan(const ModalStep& m, int64_t n_steps, int64_t L, double* ws,
                      hipStream_t s);

// Batched runs of the modal theta-method: run r drives one forcing column
// wcol[r] of W with its own waveform (samples waves[woff[r] + k], k = 0..lens[r])
// and observes one probe column pcol[r] of Pm, from a zero state.  Run
// order[j] is placed on grid row j (longest first balances the tail).
struct BatchStep {
  int64_t n0 = 0;
  const double* lam = nullptr;
  const double* W = nullptr;   // n0 x (columns), leading dimension ldw
  int64_t ldw = 0;
  const double* Pm = nullptr;  // n0 x (columns), leading dimension n0
  double theta = 0.5, dt = 1.0;
  int n_runs = 0;
  const int32_t* order = nullptr;
  const int64_t* lens = nullptr;
  const int64_t* woff = nullptr;
  const int64_t* soff = nullptr;  // first signal index of each run
  const int32_t* wcol = nullptr;
  const int32_t* pcol = nullptr;
  const double* waves = nullptr;
  double* partial = nullptr;      // (sum of lens) x G
  int G = 0;                      // mode groups per run (batch_groups)
};
struct BatchTile {
  int threads, modes;  // threads per workgroup, modes per thread
};
extern const BatchTile kBatchTiles[];
extern const int kNumBatchTiles;
int batch_groups(int64_t n0, int tile);
// The stepping launch, then (if signal) signal[e] = sum_g partial[e G + g] / dt.
void batch_steps(const BatchStep& b, int tile, int64_t total_steps, double* signal,
                 hipStream_t s);

// ---- adjoint of the probe-signal misfit (adjoint.hip) ----------------------
// Runs r = 0..n_runs-1 share one waveform (T+1 samples) and drive forcing
// column wcol[r] of W, observed through probe column pcol[r] of Pm.
struct AdjointStep {
  int64_t n0 = 0, T = 0, K = 1, n_ckpt = 0;
  int G = 0, n_runs = 0;
  const double* lam = nullptr;
  const double* W = nullptr;
  int64_t ldw = 0;
  const double* Pm = nullptr;
  const int32_t* wcol = nullptr;
  const int32_t* pcol = nullptr;
  double theta = 0.5, dt = 1.0;
  const double* wave = nullptr;  // T + 1
  const double* obs = nullptr;   // n_runs x T
  double* ckpt = nullptr;        // n_runs x n_ckpt x n0
  double* part_sig = nullptr;    // n_runs x T x G
  double* resid = nullptr;       // n_runs x T
  double* nu = nullptr;          // n_runs x n0, zero before the backward pass
  double* part_u = nullptr;      // n_runs x T x G
};
int adjoint_groups(int64_t n0);
// Forward pass with checkpoints, residuals and J (sq: n_runs x T scratch).
void adjoint_forward(const AdjointStep& s, double* J, double* sq, hipStream_t st);
// Segment [k0, k1) (k0 a checkpoint): zeta into Zb and the backward
// recursion into Lb, both n0 x (n_runs * K), column r * K + (k - k0).
void adjoint_segment(const AdjointStep& s, int64_t k0, int64_t k1, double* Zb, double* Lb,
                     hipStream_t st);
// du (T) = dJ/du_k, di (T + 1) = dJ/di_j.
void adjoint_waveform_grad(const AdjointStep& s, double* du, double* di, hipStream_t st);
// out[p] = -Phi(i_p, j_p) at the stored entries of R (offset 0).
void adjoint_gather(const Csr& R, const double* Phi, int64_t ld, double* out, hipStream_t st);

}  // namespace mm
