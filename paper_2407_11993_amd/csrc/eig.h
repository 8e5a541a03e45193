// Internal launchers of the symmetric eigensolver C = Q Lam Q^T:
// band reduction (sy2sb.hip), bulge chase and back-transforms (sb2st.hip),
// tridiagonal divide and conquer (stedc.hip), driver (eig.hip).
#pragma once
#include "kernels.h"

#include <functional>
#include <vector>

namespace mm {

// ---- stage 1: C = Q1 B Q1^T (full symmetric storage, band nb) -------------
int64_t sy2sb_ws_elems(int64_t n, int nb);
int64_t sy2sb_npanels(int64_t n, int nb);
// tau_all: npanels x nb, T_all: npanels x nb x nb.
void sy2sb(double* A, int64_t lda, int64_t n, int nb, double* tau_all, double* T_all,
           double* ws, int64_t ws_elems, hipStream_t s);
// AB(d, j) = B(j + d, j) for d <= nb; rows nb+1..ldab-1 zeroed.
void extract_band(const double* A, int64_t lda, int64_t n, int nb, double* AB,
                  int64_t ldab, hipStream_t s);
// Z <- Q1 Z for the panel reflectors left in A's lower part by sy2sb.
void apply_q1(const double* A, int64_t lda, int64_t n, int nb, const double* T_all,
              double* Z, int64_t ldz, int64_t ncols, double* ws, int64_t ws_elems,
              hipStream_t s);
int64_t apply_q1_ws_elems(int64_t n, int nb, int64_t ncols);
// Y <- Q1^T Y (the panels' block reflectors transposed, first panel first);
// ws holds apply_q1t_ws_elems(n, nb, ncols) doubles.
int64_t apply_q1t_ws_elems(int64_t n, int nb, int64_t ncols);
void apply_q1t(const double* A, int64_t lda, int64_t n, int nb, const double* T_all,
               double* Y, int64_t ldy, int64_t ncols, double* ws, int64_t ws_elems,
               hipStream_t s);

// ---- stage 2: B = Q2 T Q2^T by bulge chasing -------------------------------
struct Sb2stPlan {
  int64_t n = 0;
  int nb = 0;
  std::vector<int64_t> offset;  // first task of sweep s (n entries + total)
  int64_t tasks = 0;
};
Sb2stPlan sb2st_plan(int64_t n, int nb);
// AB has ldab = 2 nb + 1 rows.  Writes d (n), e (n-1), and the reflectors
// V2 (tasks x nb) and tau2 (tasks); d_offset is plan.offset on the device.
// With ny > 0 (at most sb2st_max_cols()), Y (n x ny, ld ldy) becomes Q2^T Y.
int sb2st_max_cols();
void sb2st(double* AB, int64_t ldab, const Sb2stPlan& plan, const int64_t* d_offset,
           double* V2, double* tau2, double* d, double* e, hipStream_t s,
           double* Y = nullptr, int64_t ldy = 0, int ny = 0);
// Z <- Q2 Z (rows 0..n-1, ncols columns); ws: at least the block list plus
// one block's V and VT (2^15 doubles); apply_q2_ws_elems(n, nb) holds every
// block at once (a smaller ws processes the compact-WY blocks in batches).
int64_t apply_q2_ws_elems(int64_t n, int nb);
void apply_q2(const Sb2stPlan& plan, const int64_t* d_offset, const double* V2,
              const double* tau2, double* Z, int64_t ldz, int64_t ncols, double* ws,
              int64_t ws_elems, hipStream_t s);
// Y <- Q2^T Y for a few columns (the reflectors kept by sb2st), in a
// wavefront of launches over the same blocks; ws holds the block list,
// apply_q2t_ws_elems(n, nb) doubles.
int64_t apply_q2t_ws_elems(int64_t n, int nb);
void apply_q2t(const Sb2stPlan& plan, const int64_t* d_offset, const double* V2,
               const double* tau2, double* Y, int64_t ldy, int64_t ncols, double* ws,
               int64_t ws_elems, hipStream_t s);

// ---- tridiagonal divide and conquer ---------------------------------------
int64_t stedc_ws_elems(int64_t n);
// Eigenvalues (ascending) and eigenvectors of the symmetric tridiagonal
// (d, e): X (n x n, ldx = n) receives Z, or (pre P) P(Z_leaves) Z_merges when
// `pre` transforms the leaves' block-diagonal eigenvectors in place before
// the merges are applied (the eigensolver's back-transform: X = Q1 Q2 Z).
// U is n^2 doubles of scratch (it may not overlap X or ws; `pre` may still
// read it, the merges write it only afterwards).  d and e are not modified.
// *d_status receives a non-zero code if a secular equation did not converge.
void stedc(const double* d, const double* e, int64_t n, double* lam, double* X,
           int64_t ldx, double* U, double* ws, int64_t ws_elems, int64_t* d_status,
           hipStream_t s, const std::function<void(double*)>& pre = {});
// Eigenvalues and ZY = Z^T Y (n x ny) without forming Z: every node of the
// tree keeps its eigenvectors' projections and boundary entries only.  U is
// n^2 doubles of scratch for the merges' eigenvector blocks (it may not
// overlap Y, ZY or ws); ws holds stedc_project_ws_elems(n, ny) doubles.
int64_t stedc_project_ws_elems(int64_t n, int ny);
void stedc_project(const double* d, const double* e, int64_t n, double* lam, const double* Y,
                   int64_t ldy, int ny, double* ZY, int64_t ldzy, double* U, double* ws,
                   int64_t ws_elems, int64_t* d_status, hipStream_t s);

// ---- driver -----------------------------------------------------------------
struct EigWork {
  int nb = 64;
  double* tau1 = nullptr;
  double* T1 = nullptr;
  double* AB = nullptr;
  double* V2 = nullptr;
  double* tau2 = nullptr;
  int64_t* d_offset = nullptr;
  double* d = nullptr;
  double* e = nullptr;
  double* ws = nullptr;
  int64_t ws_elems = 0;
  // optional phase marks (the caller's progress trace): called with the name
  // of each finished phase
  std::function<void(const char*)> mark;
};
// C (symmetric, only its lower triangle read; destroyed: it keeps the stage-1
// reflectors, then serves as the divide and conquer's scratch) -> lam, Q.
// w.ws must hold syevd_ws_elems(n, nb) doubles.
int64_t syevd_ws_elems(int64_t n, int nb);
void syevd(double* C, int64_t ldc, int64_t n, double* lam, double* Q, int64_t ldq,
           const EigWork& w, const Sb2stPlan& plan, int64_t* d_status, hipStream_t s);
// Eigenvalues and Q^T Y for a few columns Y (n x ny), without forming Q:
// Y <- Q2^T Q1^T Y on the way through the band reduction and the bulge chase
// (up to sb2st_max_cols() columns the chase takes Y along; with more, w.V2
// and w.tau2 keep its reflectors and apply_q2t follows it), then ZY = Z^T Y
// from the projected divide and conquer.  w.ws must hold
// syevd_project_ws_elems(n, nb, ny) doubles.  C is destroyed: once its band
// is extracted, its storage (ldc n >= n^2 doubles) is the divide and
// conquer's eigenvector scratch.
int64_t syevd_project_ws_elems(int64_t n, int nb, int ny);
void syevd_project(double* C, int64_t ldc, int64_t n, double* lam, double* Y, int64_t ldy,
                   int ny, double* ZY, int64_t ldzy, const EigWork& w, const Sb2stPlan& plan,
                   int64_t* d_status, hipStream_t s);

}  // namespace mm
