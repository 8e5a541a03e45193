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

__global__ void extract_v_k(const double* P, int64_t ldp, int64_t m, int nb, double* V) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * nb) return;
  const int64_t i = e % m;
  const int c = (int)(e / m);
  double v = 0.0;
  if (i == c) v = 1.0;
  else if (i > c) v = P[i + (int64_t)c * ldp];
  V[e] = v;
}

}  // namespace

int64_t apply_q1_ws_elems(int64_t n, int nb, int64_t ncols) {
  return n * nb + 2 * nb * ncols + 8 * nb * ncols;
}

void apply_q1(const double* A, int64_t lda, int64_t n, int nb, const double* T_all, double* Z,
              int64_t ldz, int64_t ncols, double* ws, int64_t ws_elems, hipStream_t s) {
  MM_REQUIRE(ws_elems >= apply_q1_ws_elems(n, nb, ncols), kInvalid,
             "apply_q1: workspace too small");
  const int64_t np = sy2sb_npanels(n, nb);
  double* V = ws;                       // m x nb
  double* W = V + n * nb;               // nb x ncols
  double* W2 = W + nb * ncols;          // nb x ncols
  double* split = W2 + nb * ncols;
  const int64_t split_elems = 8 * nb * ncols;
  for (int64_t p = np - 1; p >= 0; --p) {
    const int64_t j = p * nb, r0 = j + nb, m = n - r0;
    const double* P = A + r0 + j * lda;
    hipLaunchKernelGGL(extract_v_k, dim3((unsigned)ceil_div(m * nb, 256)), dim3(256), 0, s, P,
                       lda, m, nb, V);
    MM_HIP_TRY(hipGetLastError());
    const double* T = T_all + p * (int64_t)nb * nb;
    // W = V^T Z(r0:, :)
    Gemm g1;
    g1.m = nb; g1.n = ncols; g1.k = m;
    g1.A = V; g1.lda = m; g1.ta = true;
    g1.B = Z + r0; g1.ldb = ldz;
    g1.C = W; g1.ldc = nb;
    gemm(g1, s, split, split_elems);
    // W2 = T W   (T upper: op(A)(i,k) = 0 for k < i)
    Gemm g2;
    g2.m = nb; g2.n = ncols; g2.k = nb;
    g2.A = T; g2.lda = nb; g2.a_upper = true;
    g2.B = W; g2.ldb = nb;
    g2.C = W2; g2.ldc = nb;
    gemm(g2, s);
    // Z(r0:, :) -= V W2
    Gemm g3;
    g3.m = m; g3.n = ncols; g3.k = nb;
    g3.alpha = -1.0; g3.beta = 1.0;
    g3.A = V; g3.lda = m;
    g3.B = W2; g3.ldb = nb;
    g3.C = Z + r0; g3.ldc = ldz;
    gemm(g3, s);
  }
}

void apply_q1t(const double* A, int64_t lda, int64_t n, int nb, const double* T_all, double* Y,
               int64_t ldy, int64_t ncols, double* ws, int64_t ws_elems, hipStream_t s) {
  MM_REQUIRE(ws_elems >= apply_q1_ws_elems(n, nb, ncols), kInvalid,
             "apply_q1t: workspace too small");
  const int64_t np = sy2sb_npanels(n, nb);
  double* V = ws;                       // m x nb
  double* W = V + n * nb;               // nb x ncols
  double* W2 = W + nb * ncols;          // nb x ncols
  double* split = W2 + nb * ncols;
  const int64_t split_elems = 8 * nb * ncols;
  for (int64_t p = 0; p < np; ++p) {
    const int64_t j = p * nb, r0 = j + nb, m = n - r0;
    const double* P = A + r0 + j * lda;
    hipLaunchKernelGGL(extract_v_k, dim3((unsigned)ceil_div(m * nb, 256)), dim3(256), 0, s, P,
                       lda, m, nb, V);
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
  MM_REQUIRE(ny >= 1 && ny <= sb2st_max_cols(), kInvalid,
             "syevd_project: 1..32 projected columns");
  const int nb = w.nb;
  auto mark = [&](const char* what) { if (w.mark) w.mark(what); };
  sy2sb(C, ldc, n, nb, w.tau1, w.T1, w.ws, w.ws_elems, s);
  apply_q1t(C, ldc, n, nb, w.T1, Y, ldy, ny, w.ws, w.ws_elems, s);
  mark("band reduction");
  const int64_t ldab = 2 * nb + 1;
  extract_band(C, ldc, n, nb, w.AB, ldab, s);
  sb2st(w.AB, ldab, plan, w.d_offset, w.V2, w.tau2, w.d, w.e, s, Y, ldy, ny);
  mark("bulge chase");
  // C is dead from here on (its reflectors were applied to Y, its band copied)
  stedc_project(w.d, w.e, n, lam, Y, ldy, ny, ZY, ldzy, C, w.ws, w.ws_elems, d_status, s);
  mark("divide and conquer");
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
