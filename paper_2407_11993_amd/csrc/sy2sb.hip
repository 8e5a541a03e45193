// Stage 1 of the two-stage tridiagonalisation: C = Q1 B Q1^T with B banded
// (lower bandwidth nb).  The symmetric matrix is kept in full column-major
// storage.  For panel p (columns j..j+nb-1, rows r0 = j+nb .. n-1):
//
//   1. Householder QR of the m x nb panel, one launch per column.  Each
//      workgroup owns a slice of rows; a launch finishes the previous column
//      (every workgroup sums the previous launch's per-slice partials in slice
//      order, so all agree bit for bit) and emits the partials of the next
//      column: the squared norm below the diagonal and the dot products with
//      the columns to its right.  No grid-wide barrier is needed.
//   2. The reflectors are copied to an explicit m x nb matrix V (unit
//      diagonal) and the triangular factor T of H = I - V T V^T is formed.
//   3. Two-sided update of the trailing matrix A22 <- H^T A22 H on the
//      matrix cores:  X = A22 V T,  Y = X - 1/2 V (T^T V^T X),
//      A22 -= V Y^T + Y V^T.
//
// Only the lower triangle of A is read or written: A22 V reads A22 as a
// symmetric matrix stored in its lower triangle, and the rank-2nb update
// writes the lower triangle only (half the work and traffic of a full one).
//
// R overwrites the panel's top nb x nb block; V stays below it (the implicit
// unit diagonal at row r0 + c of column j + c) for the back-transform.
#include "kernels.h"
#include "eig.h"

namespace mm {
namespace {

constexpr int QT = 256;     // threads per workgroup of the panel QR
constexpr int QROWS = 256;  // panel rows per workgroup

// Per-launch scratch, double buffered by column parity (launch c reads what
// launch c-1 wrote while writing its own):
//   part[buf][g][0]      : squared norm of column c over slice g, rows > c
//   part[buf][g][1 + jj] : dot(column c, column c+1+jj) over slice g, rows > c
//   rowv[buf][jj]        : A(c, c+jj) after the launch's update (a snapshot,
//                          because slice 0 updates row c while the other
//                          slices still need the value of the previous one)
// Each thread owns exactly one panel row (QROWS == QT) and holds the columns
// of that row it works on in registers: every global load of a launch is
// issued at its start, so a launch costs about one memory latency.
constexpr int MAXNB = 64;

__global__ void __launch_bounds__(QT) panel_qr_step(double* P, int64_t ldp, int64_t m,
                                                    int nb, int c, double* scratch,
                                                    int G, double* tau) {
  const int t = threadIdx.x;
  const int g = blockIdx.x;
  const int64_t i = (int64_t)g * QROWS + t;  // this thread's panel row
  const int stride = nb + 1;
  const int64_t per_buf = (int64_t)G * stride + nb;
  __shared__ double red2[MAXNB][QT + 1];  // products, column-major by row
  __shared__ double red[4][MAXNB + 1];
  __shared__ double tot[MAXNB + 1];
  __shared__ double wv[MAXNB + 1];
  __shared__ double sh[3];
  const int b0 = c >= 1 ? c - 1 : 0;  // first column held in registers
  const int nx = nb - b0;             // columns held
  // ---- issue every load: the row, the previous column's partials, its row
  double x[MAXNB];
  const bool row_ok = i < m;
  const double* prow = P + (row_ok ? i : 0) + (int64_t)b0 * ldp;
#pragma unroll
  for (int u = 0; u < MAXNB; ++u) x[u] = (row_ok && u < nx) ? prow[(int64_t)u * ldp] : 0.0;
  const int cp = c - 1;
  const bool finish = c >= 1 && cp < m;
  if (finish) {
    const double* part = scratch + (cp & 1) * per_buf;
    const double* rowv = part + (int64_t)G * stride;
    const int ncol = nb - cp;
    // four threads per column, each summing a contiguous quarter of slices
    const int j = t & 63, h = t >> 6, G4 = (G + 3) / 4;
    double ps = 0.0;
    for (int u0 = 0; u0 < G4; u0 += 16) {
      double xs[16];  // clamped addresses: all sixteen loads in flight at once
#pragma unroll
      for (int u = 0; u < 16; ++u)
        xs[u] = part[(int64_t)min(h * G4 + u0 + u, G - 1) * stride + min(j, ncol - 1)];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int q = h * G4 + u0 + u;
        ps += (u0 + u < G4 && q < G && j < ncol) ? xs[u] : 0.0;
      }
    }
    red[h][j] = ps;
    const double rv = (t < ncol) ? rowv[t] : 0.0;
    __syncthreads();
    if (t < ncol) tot[t] = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
    __syncthreads();
    if (t == 0) {
      const double a0 = rv;
      const double sig2 = tot[0];
      double tv = 0.0, beta = a0, scale = 0.0;
      if (sig2 > 0.0) {
        beta = -copysign(sqrt(a0 * a0 + sig2), a0);
        tv = (beta - a0) / beta;
        scale = 1.0 / (a0 - beta);
      }
      sh[0] = tv; sh[1] = beta; sh[2] = scale;
      if (g == 0) tau[cp] = tv;
    }
    __syncthreads();
    const double tv = sh[0], scale = sh[2];
    // w_j = tau v^T A(:, j) = tau (A(cp, j) + scale * dot_j),  j > cp
    if (t >= 1 && t < ncol) wv[t] = tv * (rv + scale * tot[t]);
    __syncthreads();
    if (tv != 0.0 && row_ok && i >= cp) {
      const double vi = (i > cp) ? x[0] * scale : 1.0;
      x[0] = (i > cp) ? vi : sh[1];  // v below the diagonal, R(cp, cp) = beta
#pragma unroll
      for (int u = 1; u < MAXNB; ++u)
        if (u < nx) x[u] -= vi * wv[u];
      double* wrow = P + i + (int64_t)b0 * ldp;
#pragma unroll
      for (int u = 0; u < MAXNB; ++u)
        if (u < nx) wrow[(int64_t)u * ldp] = x[u];
    }
  } else if (c >= 1 && g == 0 && t == 0) {
    tau[cp] = 0.0;
  }
  if (c >= nb || c >= m) return;
  // ---- partials of column c over rows > c, from the registers -----------------
  double* part = scratch + (c & 1) * per_buf;
  double* po = part + (int64_t)g * stride;
  const int uc = c - b0;  // register index of column c (0 or 1)
  const int ncol = nb - c;
  const bool mine = row_ok && i > c;
  const double a = mine ? (uc ? x[1] : x[0]) : 0.0;
#pragma unroll
  for (int u = 0; u < MAXNB; ++u) {
    const int jj = u - uc;
    if (jj >= 0 && jj < ncol) red2[jj][t] = a * x[u];
  }
  // snapshot of row c (owned by slice 0, thread c)
  if (g == 0 && t == c) {
    double* rowv = part + (int64_t)G * stride;
#pragma unroll
    for (int u = 0; u < MAXNB; ++u) {
      const int jj = u - uc;
      if (jj >= 0 && jj < ncol) rowv[jj] = x[u];
    }
  }
  __syncthreads();
  {
    const int j = t & 63, h = t >> 6;
    double s2 = 0.0;
    if (j < ncol) {
#pragma unroll 16
      for (int r = 0; r < 64; ++r) s2 += red2[j][64 * h + r];
    }
    red[h][j] = s2;
  }
  __syncthreads();
  if (t < ncol) po[t] = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
}

// Explicit V (m x nb, column-major, ld m) from the stored reflectors.
__global__ void extract_v(const double* P, int64_t ldp, int64_t m, int nb, double* V) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * nb) return;
  const int64_t i = e % m;
  const int c = (int)(e / m);
  double v = 0.0;
  if (i == c) v = 1.0;
  else if (i > c) v = P[i + (int64_t)c * ldp];
  V[e] = v;
}

// T (nb x nb, upper) from tau and the Gram matrix S = V^T V:
//   T(c,c) = tau_c,  T(0:c, c) = -tau_c T(0:c, 0:c) S(0:c, c).
// Columns with tau_c = 0 give zero columns.
__global__ void form_t(const double* S, const double* tau, int nb, double* T) {
  __shared__ double col[128];
  const int t = threadIdx.x;
  for (int e = t; e < nb * nb; e += blockDim.x) T[e] = 0.0;
  __syncthreads();
  for (int c = 0; c < nb; ++c) {
    const double tc = tau[c];
    if (t < c) {
      double s = 0.0;
      for (int q = t; q < c; ++q) s += T[t + q * nb] * S[q + c * nb];
      col[t] = -tc * s;
    }
    __syncthreads();
    if (t < c) T[t + c * nb] = col[t];
    if (t == 0) T[c + c * nb] = tc;
    __syncthreads();
  }
}

}  // namespace

int64_t sy2sb_ws_elems(int64_t n, int nb) {
  const int64_t G = ceil_div(n, QROWS);
  const int64_t stride = nb + 1;
  // scratch (2 (G stride + nb)) + V|Y|V (n x 3nb) + X (n x nb) + small (4 nb^2)
  // + split-K partials (8 n nb)
  return 2 * (G * stride + nb) + n * 3 * nb + n * nb + 4 * (int64_t)nb * nb + 8 * n * nb;
}

int64_t sy2sb_npanels(int64_t n, int nb) {
  int64_t p = 0;
  for (int64_t j = 0; j + nb < n - 1; j += nb) ++p;
  return p;
}

void sy2sb(double* A, int64_t lda, int64_t n, int nb, double* tau_all, double* T_all,
           double* ws, int64_t ws_elems, hipStream_t s) {
  MM_REQUIRE(nb >= 1 && nb <= MAXNB, kInvalid, "sy2sb: band must be 1..64");
  MM_REQUIRE(ws_elems >= sy2sb_ws_elems(n, nb), kInvalid, "sy2sb: workspace too small");
  const int64_t Gmax = ceil_div(n, QROWS);
  const int stride = nb + 1;
  double* part = ws;
  double* VYV = part + 2 * (Gmax * stride + nb);  // n x 3nb
  double* X = VYV + n * 3 * nb;                // n x nb
  double* Sm = X + n * nb;                     // nb x nb
  double* Pm = Sm + (int64_t)nb * nb;          // nb x nb
  double* Zm = Pm + (int64_t)nb * nb;          // nb x nb
  double* split = Zm + 2 * (int64_t)nb * nb;   // split-K workspace
  const int64_t split_elems = 8 * n * nb;
  int64_t p = 0;
  for (int64_t j = 0; j + nb < n - 1; j += nb, ++p) {
    const int64_t r0 = j + nb;
    const int64_t m = n - r0;
    double* P = A + r0 + j * lda;
    double* tau = tau_all + p * nb;
    double* T = T_all + p * (int64_t)nb * nb;
    const int G = (int)ceil_div(m, QROWS);
    for (int c = 0; c <= nb; ++c)
      hipLaunchKernelGGL(panel_qr_step, dim3(G), dim3(QT), 0, s, P, lda, m, nb, c, part,
                         G, tau);
    MM_HIP_TRY(hipGetLastError());
    // V, the Gram matrix and T
    double* V = VYV;                 // columns 0..nb-1
    double* Y = VYV + m * nb;        // columns nb..2nb-1
    double* V2 = VYV + 2 * m * nb;   // columns 2nb..3nb-1
    hipLaunchKernelGGL(extract_v, dim3((unsigned)ceil_div(m * nb, 256)), dim3(256), 0, s,
                       P, lda, m, nb, V);
    hipLaunchKernelGGL(extract_v, dim3((unsigned)ceil_div(m * nb, 256)), dim3(256), 0, s,
                       P, lda, m, nb, V2);
    MM_HIP_TRY(hipGetLastError());
    Gemm gs;  // S = V^T V
    gs.m = nb; gs.n = nb; gs.k = m;
    gs.A = V; gs.lda = m; gs.ta = true;
    gs.B = V; gs.ldb = m;
    gs.C = Sm; gs.ldc = nb;
    gemm(gs, s, split, split_elems);
    hipLaunchKernelGGL(form_t, dim3(1), dim3(128), 0, s, Sm, tau, nb, T);
    MM_HIP_TRY(hipGetLastError());
    double* A22 = A + r0 + r0 * lda;
    // X0 = A22 V  (m x nb; A22 symmetric, lower triangle stored)
    Gemm g1;
    g1.m = m; g1.n = nb; g1.k = m;
    g1.A = A22; g1.lda = lda; g1.a_sym = true;
    g1.B = V; g1.ldb = m;
    g1.C = X; g1.ldc = m;
    gemm(g1, s, split, split_elems);
    // Y = X0 T  (T upper: op(B)(k,j) = 0 for k > j)
    Gemm g2;
    g2.m = m; g2.n = nb; g2.k = nb;
    g2.A = X; g2.lda = m;
    g2.B = T; g2.ldb = nb; g2.b_band = 0;
    g2.C = Y; g2.ldc = m;
    gemm(g2, s);
    // Pm = V^T Y   (nb x nb)
    Gemm g3;
    g3.m = nb; g3.n = nb; g3.k = m;
    g3.A = V; g3.lda = m; g3.ta = true;
    g3.B = Y; g3.ldb = m;
    g3.C = Pm; g3.ldc = nb;
    gemm(g3, s, split, split_elems);
    // Zm = T^T Pm
    Gemm g4;
    g4.m = nb; g4.n = nb; g4.k = nb;
    g4.A = T; g4.lda = nb; g4.ta = true;
    g4.B = Pm; g4.ldb = nb;
    g4.C = Zm; g4.ldc = nb;
    gemm(g4, s);
    // Y -= 1/2 V Zm
    Gemm g5;
    g5.m = m; g5.n = nb; g5.k = nb;
    g5.alpha = -0.5; g5.beta = 1.0;
    g5.A = V; g5.lda = m;
    g5.B = Zm; g5.ldb = nb;
    g5.C = Y; g5.ldc = m;
    gemm(g5, s);
    // A22 -= [V Y] [Y V]^T  (lower triangle)
    Gemm g6;
    g6.m = m; g6.n = m; g6.k = 2 * nb;
    g6.alpha = -1.0; g6.beta = 1.0;
    g6.A = VYV; g6.lda = m;
    g6.B = VYV + m * nb; g6.ldb = m; g6.tb = true;
    g6.C = A22; g6.ldc = lda;
    g6.lower = true;
    gemm(g6, s);
  }
}

// Band of the reduced matrix, lower storage AB(d, j) = B(j + d, j), d <= 2nb
// (rows nb+1..2nb zeroed for the bulge chase).
__global__ void extract_band_k(const double* A, int64_t lda, int64_t n, int nb,
                               double* AB, int64_t ldab) {
  const int64_t j = blockIdx.x;
  for (int d = threadIdx.x; d < ldab; d += blockDim.x) {
    double v = 0.0;
    if (d <= nb && j + d < n) v = A[(j + d) + j * lda];
    AB[d + j * ldab] = v;
  }
}

void extract_band(const double* A, int64_t lda, int64_t n, int nb, double* AB,
                  int64_t ldab, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(extract_band_k, dim3((unsigned)n), dim3(128), 0, s, A, lda, n, nb, AB, ldab);
  MM_HIP_TRY(hipGetLastError());
}

}  // namespace mm
