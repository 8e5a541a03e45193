// Symmetric eigensolver driver C = Q Lam Q^T (the modal decomposition's
// standard form, Sec. 3.2):
//   sy2sb (band nb)  ->  sb2st (tridiagonal)  ->  stedc  ->  Q = Q1 (Q2 Z).
// Q1 is applied panel by panel, last panel first, as the compact WY product
//   Z(r0:, :) -= V (T (V^T Z(r0:, :)))   on the matrix cores.
#include "eig.h"

namespace mm {
namespace {

// the back-transform's block reflectors are built in batches of at most this
// many doubles (2 GiB)
constexpr int64_t kQ2WsCap = (int64_t)1 << 28;

// V(:, c) (m rows, leading dimension ldv) = column c of the panel's
// reflectors: unit diagonal, zero above it.
__global__ void extract_v_k(const double* P, int64_t ldp, int64_t m, int nb, double* V,
                            int64_t ldv) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * nb) return;
  const int64_t i = e % m;
  const int c = (int)(e / m);
  double v = 0.0;
  if (i == c) v = 1.0;
  else if (i > c) v = P[i + (int64_t)c * ldp];
  V[i + c * ldv] = v;
}

}  // namespace

// Q1 is applied in groups of up to Q1G panels: H_p H_{p+1} ... H_{p+g-1} =
// I - Vg Tg Vg^T with Vg = [V_p ... V_{p+g-1}] on the group's common rows
// (V_{p+j} zero above its own first row) and Tg upper triangular, built one
// panel at a time (Schreiber & Van Loan's compact WY aggregation):
//   Tg <- [[Tg, -Tg (Vg^T V_j) T_j], [0, T_j]],
// so the products with Z have depth g nb instead of nb.
constexpr int Q1G = 4;

int64_t apply_q1_ws_elems(int64_t n, int nb, int64_t ncols) {
  const int64_t kg = (int64_t)Q1G * nb;
  return n * kg + 2 * kg * ncols + 8 * kg * ncols + 3 * kg * kg;
}

void apply_q1(const double* A, int64_t lda, int64_t n, int nb, const double* T_all, double* Z,
              int64_t ldz, int64_t ncols, double* ws, int64_t ws_elems, hipStream_t s) {
  MM_REQUIRE(ws_elems >= apply_q1_ws_elems(n, nb, ncols), kInvalid,
             "apply_q1: workspace too small");
  const int64_t np = sy2sb_npanels(n, nb);
  const int64_t kg = (int64_t)Q1G * nb;
  double* V = ws;                       // m x kg (the group's reflectors)
  double* W = V + n * kg;               // kg x ncols
  double* W2 = W + kg * ncols;          // kg x ncols
  double* split = W2 + kg * ncols;
  const int64_t split_elems = 8 * kg * ncols;
  double* S = split + split_elems;      // kg x kg:  Vg^T Vg
  double* Tg = S + kg * kg;             // kg x kg
  double* Tw = Tg + kg * kg;            // kg x nb scratch
  // groups from the last panel down: group [p0, p0 + g)
  for (int64_t p1 = np; p1 > 0;) {
    const int64_t g = std::min<int64_t>(Q1G, p1);
    const int64_t p0 = p1 - g;
    p1 = p0;
    const int64_t r0 = (p0 + 1) * nb, m = n - r0;  // the group's common rows
    const int64_t kk = g * nb;
    fill(V, m * kk, 0.0, s);
    for (int64_t q = 0; q < g; ++q) {
      const int64_t p = p0 + q, j = p * nb, rq = (p + 1) * nb, mq = n - rq;
      const double* P = A + rq + j * lda;
      hipLaunchKernelGGL(extract_v_k, dim3((unsigned)ceil_div(mq * nb, 256)), dim3(256), 0, s, P,
                         lda, mq, nb, V + (rq - r0) + q * nb * m, m);
    }
    MM_HIP_TRY(hipGetLastError());
    // Tg: the diagonal blocks are the panels' T, the others from S = Vg^T Vg
    fill(Tg, kk * kk, 0.0, s);
    for (int64_t q = 0; q < g; ++q)
      copy_matrix(T_all + (p0 + q) * (int64_t)nb * nb, nb, Tg + q * nb * (kk + 1), kk, nb, nb, s);
    if (g > 1) {
      Gemm gs;  // S = Vg^T Vg (only its strictly upper blocks are read)
      gs.m = kk; gs.n = kk; gs.k = m;
      gs.A = V; gs.lda = m; gs.ta = true;
      gs.B = V; gs.ldb = m;
      gs.C = S; gs.ldc = kk;
      gemm(gs, s, split, split_elems);
      for (int64_t q = 1; q < g; ++q) {
        const int64_t c0 = q * nb;
        Gemm ga;  // Tw = Tg[0:c0, 0:c0] S[0:c0, c0:c0+nb]   (Tg upper)
        ga.m = c0; ga.n = nb; ga.k = c0;
        ga.A = Tg; ga.lda = kk; ga.a_upper = true;
        ga.B = S + c0 * kk; ga.ldb = kk;
        ga.C = Tw; ga.ldc = kk;
        gemm(ga, s);
        Gemm gb;  // Tg[0:c0, c0:c0+nb] = -Tw T_q   (T_q upper: op(B)(k, j) = 0 for k > j)
        gb.m = c0; gb.n = nb; gb.k = nb;
        gb.alpha = -1.0;
        gb.A = Tw; gb.lda = kk;
        gb.B = Tg + c0 * (kk + 1); gb.ldb = kk; gb.b_band = 0;
        gb.C = Tg + c0 * kk; gb.ldc = kk;
        gemm(gb, s);
      }
    }
    // W = Vg^T Z(r0:, :)
    Gemm g1;
    g1.m = kk; g1.n = ncols; g1.k = m;
    g1.A = V; g1.lda = m; g1.ta = true;
    g1.B = Z + r0; g1.ldb = ldz;
    g1.C = W; g1.ldc = kk;
    gemm(g1, s, split, split_elems);
    // W2 = Tg W   (Tg upper: op(A)(i,k) = 0 for k < i)
    Gemm g2;
    g2.m = kk; g2.n = ncols; g2.k = kk;
    g2.A = Tg; g2.lda = kk; g2.a_upper = true;
    g2.B = W; g2.ldb = kk;
    g2.C = W2; g2.ldc = kk;
    gemm(g2, s);
    // Z(r0:, :) -= Vg W2
    Gemm g3;
    g3.m = m; g3.n = ncols; g3.k = kk;
    g3.alpha = -1.0; g3.beta = 1.0;
    g3.A = V; g3.lda = m;
    g3.B = W2; g3.ldb = kk;
    g3.C = Z + r0; g3.ldc = ldz;
    gemm(g3, s);
  }
}

// Split-K shares of the few-column products V^T Y: one per 128 rows (a
// product of nb x ncols outputs over m rows runs on m / 128 workgroups).
static int64_t q1t_splits(int64_t n) { return std::max<int64_t>(8, std::min<int64_t>(1024, n / 128)); }

int64_t apply_q1t_ws_elems(int64_t n, int nb, int64_t ncols) {
  return n * nb + 2 * (int64_t)nb * ncols + q1t_splits(n) * nb * ncols;
}

void apply_q1t(const double* A, int64_t lda, int64_t n, int nb, const double* T_all, double* Y,
               int64_t ldy, int64_t ncols, double* ws, int64_t ws_elems, hipStream_t s) {
  MM_REQUIRE(ws_elems >= apply_q1t_ws_elems(n, nb, ncols), kInvalid,
             "apply_q1t: workspace too small");
  const int64_t np = sy2sb_npanels(n, nb);
  double* V = ws;                       // m x nb
  double* W = V + n * nb;               // nb x ncols
  double* W2 = W + nb * ncols;          // nb x ncols
  double* split = W2 + nb * ncols;
  const int64_t split_elems = q1t_splits(n) * nb * ncols;
  for (int64_t p = 0; p < np; ++p) {
    const int64_t j = p * nb, r0 = j + nb, m = n - r0;
    const double* P = A + r0 + j * lda;
    hipLaunchKernelGGL(extract_v_k, dim3((unsigned)ceil_div(m * nb, 256)), dim3(256), 0, s, P,
                       lda, m, nb, V, m);
    MM_HIP_TRY(hipGetLastError());
    const double* T = T_all + p * (int64_t)nb * nb;
    // W = V^T Y(r0:, :)
    Gemm g1;
    g1.m = nb; g1.n = ncols; g1.k = m;
    g1.A = V; g1.lda = m; g1.ta = true;
    g1.B = Y + r0; g1.ldb = ldy;
    g1.C = W; g1.ldc = nb;
    gemm(g1, s, split, split_elems);
    // W2 = T^T W   (T^T lower: op(A)(i,k) = 0 for k > i)
    Gemm g2;
    g2.m = nb; g2.n = ncols; g2.k = nb;
    g2.A = T; g2.lda = nb; g2.ta = true; g2.a_lower = true;
    g2.B = W; g2.ldb = nb;
    g2.C = W2; g2.ldc = nb;
    gemm(g2, s);
    // Y(r0:, :) -= V W2
    Gemm g3;
    g3.m = m; g3.n = ncols; g3.k = nb;
    g3.alpha = -1.0; g3.beta = 1.0;
    g3.A = V; g3.lda = m;
    g3.B = W2; g3.ldb = nb;
    g3.C = Y + r0; g3.ldc = ldy;
    gemm(g3, s);
  }
}

void syevd_project(double* C, int64_t ldc, int64_t n, double* lam, double* Y, int64_t ldy,
                   int ny, double* ZY, int64_t ldzy, const EigWork& w, const Sb2stPlan& plan,
                   int64_t* d_status, hipStream_t s) {
  MM_REQUIRE(ny >= 1, kInvalid, "syevd_project: at least one projected column");
  const int nb = w.nb;
  MM_REQUIRE(w.ws_elems >= syevd_project_ws_elems(n, nb, ny), kInvalid,
             "syevd_project: workspace too small");
  const bool along = ny <= sb2st_max_cols();  // Y rides along the bulge chase
  MM_REQUIRE(along || (w.V2 && w.tau2), kInvalid,
             "syevd_project: more columns than the bulge chase carries need V2 and tau2");
  auto mark = [&](const char* what) { if (w.mark) w.mark(what); };
  sy2sb(C, ldc, n, nb, w.tau1, w.T1, w.ws, w.ws_elems, s);
  apply_q1t(C, ldc, n, nb, w.T1, Y, ldy, ny, w.ws, w.ws_elems, s);
  mark("band reduction");
  const int64_t ldab = 2 * nb + 1;
  extract_band(C, ldc, n, nb, w.AB, ldab, s);
  if (along) {
    sb2st(w.AB, ldab, plan, w.d_offset, nullptr, nullptr, w.d, w.e, s, Y, ldy, ny);
  } else {
    sb2st(w.AB, ldab, plan, w.d_offset, w.V2, w.tau2, w.d, w.e, s);
    apply_q2t(plan, w.d_offset, w.V2, w.tau2, Y, ldy, ny, w.ws, w.ws_elems, s);
  }
  mark("bulge chase");
  // C is dead from here on (its reflectors were applied to Y, its band copied)
  stedc_project(w.d, w.e, n, lam, Y, ldy, ny, ZY, ldzy, C, w.ws, w.ws_elems, d_status, s);
  mark("divide and conquer");
}

int64_t syevd_project_ws_elems(int64_t n, int nb, int ny) {
  int64_t w = std::max(sy2sb_ws_elems(n, nb), stedc_project_ws_elems(n, ny));
  w = std::max(w, apply_q1t_ws_elems(n, nb, ny));
  if (ny > sb2st_max_cols()) w = std::max(w, apply_q2t_ws_elems(n, nb));
  return w;
}

int64_t syevd_ws_elems(int64_t n, int nb) {
  const int64_t bt = std::max(apply_q1_ws_elems(n, nb, n),
                              std::min(apply_q2_ws_elems(n, nb), kQ2WsCap));
  return std::max(sy2sb_ws_elems(n, nb), stedc_ws_elems(n) + bt);
}

void syevd(double* C, int64_t ldc, int64_t n, double* lam, double* Q, int64_t ldq,
           const EigWork& w, const Sb2stPlan& plan, int64_t* d_status, hipStream_t s) {
  MM_REQUIRE(ldq == n, kInvalid, "syevd: ldq must equal n");
  MM_REQUIRE(w.ws_elems >= syevd_ws_elems(n, w.nb), kInvalid, "syevd: workspace too small");
  const int nb = w.nb;
  auto mark = [&](const char* what) { if (w.mark) w.mark(what); };
  sy2sb(C, ldc, n, nb, w.tau1, w.T1, w.ws, w.ws_elems, s);
  mark("band reduction");
  const int64_t ldab = 2 * nb + 1;
  extract_band(C, ldc, n, nb, w.AB, ldab, s);
  sb2st(w.AB, ldab, plan, w.d_offset, w.V2, w.tau2, w.d, w.e, s);
  mark("bulge chase");
  // the divide and conquer keeps its arrays at the start of ws; the
  // back-transform of its leaves (Q1 Q2 Z_leaves, before any merge) works
  // behind them.  C's reflectors are read there; afterwards its storage
  // (ldc n >= n^2 doubles) is the merges' scratch U.
  const int64_t n_dc = stedc_ws_elems(n);
  double* ws_bt = w.ws + n_dc;
  const int64_t n_bt = w.ws_elems - n_dc;
  stedc(w.d, w.e, n, lam, Q, ldq, C, w.ws, n_dc, d_status, s, [&](double* X) {
    apply_q2(plan, w.d_offset, w.V2, w.tau2, X, ldq, n, ws_bt, n_bt, s);
    mark("back-transform Q2");
    apply_q1(C, ldc, n, nb, w.T1, X, ldq, n, ws_bt, n_bt, s);
    mark("back-transform Q1");
  });
  mark("divide and conquer merges");
}

}  // namespace mm
