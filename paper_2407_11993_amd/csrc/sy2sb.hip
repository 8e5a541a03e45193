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
// issued at its start, so a launch costs about one memory latency.  The row
// and the partial sums are stored written through (the next launch reads them
// on other XCDs).
constexpr int MAXNB = 64;
// partials read per thread at once when the previous column's sums are
// formed (each thread sums a quarter of the workgroups' partials)
#ifndef MM_SY2SB_PB
#define MM_SY2SB_PB 32
#endif
constexpr int PB = MM_SY2SB_PB;

// CW: columns summed per pass of the partial sums through LDS.  CW = 64
// (one pass, 132 KB of LDS: one workgroup per CU) for panels of up to 256 row
// blocks; CW = 32 (two passes, 66 KB: two workgroups per CU) for taller ones,
// which then run in one round instead of two.
template <int CW>
__global__ void __launch_bounds__(QT) __attribute__((amdgpu_waves_per_eu(CW == 32 ? 2 : 1)))
    panel_qr_step(double* P, int64_t ldp, int64_t m, int nb, int c, double* scratch, int G,
                  double* tau) {
  const int t = threadIdx.x;
  const int g = blockIdx.x;
  const int64_t i = (int64_t)g * QROWS + t;  // this thread's panel row
  const int stride = nb + 1;
  const int64_t per_buf = (int64_t)G * stride + nb;
  constexpr int TPC = QT / CW;  // threads per column in the sums
  __shared__ double red2[CW][QT + 1];  // products of CW columns, by row
  __shared__ double redc[TPC][CW + 1];
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
    for (int u0 = 0; u0 < G4; u0 += PB) {
      double xs[PB];  // clamped addresses: all PB loads in flight at once
#pragma unroll
      for (int u = 0; u < PB; ++u)
        xs[u] = part[(int64_t)min(h * G4 + u0 + u, G - 1) * stride + min(j, ncol - 1)];
#pragma unroll
      for (int u = 0; u < PB; ++u) {
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
        if (u < nx) store_dev(&wrow[(int64_t)u * ldp], x[u]);
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
  // snapshot of row c (owned by slice 0, thread c)
  if (g == 0 && t == c) {
    double* rowv = part + (int64_t)G * stride;
#pragma unroll
    for (int u = 0; u < MAXNB; ++u) {
      const int jj = u - uc;
      if (jj >= 0 && jj < ncol) store_dev(&rowv[jj], x[u]);
    }
  }
  // the products a x_u summed over the workgroup's rows, CW columns at a time
  // through an LDS transpose
  for (int j0 = 0; j0 < ncol; j0 += CW) {
#pragma unroll
    for (int u = 0; u < MAXNB; ++u) {
      const int jj = u - uc - j0;
      if (jj >= 0 && jj < CW && j0 + jj < ncol) red2[jj][t] = a * x[u];
    }
    __syncthreads();
    {
      const int j = t % CW, h = t / CW;  // TPC threads per column, CW rows each
      double s2 = 0.0;
      if (j0 + j < ncol) {
#pragma unroll 16
        for (int r = 0; r < CW; ++r) s2 += red2[j][CW * h + r];
      }
      redc[h][j] = s2;
    }
    __syncthreads();
    if (t < CW && j0 + t < ncol) {
      double s2 = 0.0;
#pragma unroll
      for (int h = 0; h < TPC; ++h) s2 += redc[h][t];
      store_dev(&po[j0 + t], s2);
    }
    __syncthreads();  // red2 and redc are reused by the next CW columns
  }
}

// Explicit V (m x nb, column-major, ld ldv) from the stored reflectors.
__global__ void extract_v(const double* P, int64_t ldp, int64_t m, int nb, double* V,
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

// T (nb x nb, upper) from tau and the Gram matrix S = V^T V:
//   T(c,c) = tau_c,  T(0:c, c) = -tau_c T(0:c, 0:c) S(0:c, c).
// Columns with tau_c = 0 give zero columns.  S and T live in LDS (the
// recurrence reads T's finished columns nb times).
__global__ void __launch_bounds__(64) form_t(const double* S, const double* tau, int nb,
                                             double* T) {
  __shared__ double Ss[64][65];
  __shared__ double Ts[64][65];
  __shared__ double tv[64];
  const int t = threadIdx.x;
  for (int e = t; e < 64 * 64; e += 64) {
    const int r = e % 64, c = e / 64;
    Ss[r][c] = (r < nb && c < nb) ? S[r + c * nb] : 0.0;
    Ts[r][c] = 0.0;
  }
  if (t < nb) tv[t] = tau[t];
  __syncthreads();
  for (int c = 0; c < nb; ++c) {
    // row t of T is zero outside columns [t, c) so far: a fixed-length,
    // unrolled sum (its LDS reads pipeline, unlike a loop of t-dependent length)
    double v = 0.0;
#pragma unroll 16
    for (int q = 0; q < 64; ++q) v += Ts[t][q] * Ss[q][c];
    v = (t < c) ? -tv[c] * v : (t == c ? tv[c] : 0.0);
    __syncthreads();  // every read of column c's inputs is done
    if (t <= c) Ts[t][c] = v;
    __syncthreads();
  }
  for (int e = t; e < nb * nb; e += 64) T[e] = Ts[e % nb][e / nb];
}

}  // namespace

// Leading dimension of the panel buffers: columns start on 128-byte
// boundaries (the products read them row-wise in 128-byte pieces).
static inline int64_t ld16(int64_t m) { return ceil_div(m, 16) * 16; }

#ifndef MM_SY2SB_GP
#define MM_SY2SB_GP 6
#endif
constexpr int GP = MM_SY2SB_GP;  // panels per group
// split-K partials of the n x nb products, in units of n nb doubles (the
// symmetric products split up to this many ways at full height)
#ifndef MM_SY2SB_SPLIT_WS
#define MM_SY2SB_SPLIT_WS 32
#endif
constexpr int64_t SPLIT_WS = MM_SY2SB_SPLIT_WS;

int64_t sy2sb_ws_elems(int64_t n, int nb) {
  const int64_t G = ceil_div(n, QROWS);
  const int64_t stride = nb + 1;
  const int64_t np = ld16(n);
  // scratch (2 (G stride + nb)) + X (np x nb) + small (3 nb^2 + 2 GP nb^2)
  // + U1, U2 (np x 2 GP nb each) + split-K partials (SPLIT_WS n nb)
  return 2 * (G * stride + nb) + np * nb + (3 + 2 * GP) * (int64_t)nb * nb +
         2 * np * 2 * GP * nb + SPLIT_WS * n * nb;
}

int64_t sy2sb_npanels(int64_t n, int nb) {
  int64_t p = 0;
  for (int64_t j = 0; j + nb < n - 1; j += nb) ++p;
  return p;
}

namespace {

struct Sy2sbWs {
  double* part;
  double* X;      // n x nb
  double* Sm;     // nb x nb
  double* Pm;     // nb x nb
  double* Zm;     // nb x nb
  double* S2;     // 2 (GP - 1) nb x nb
  double* split;  // split-K partials
  int64_t split_elems;
};

// Householder QR of the m x nb panel P (ld lda): R over its top block, the
// reflectors below; V (unit diagonal, ld ldv) written to V1 and V2, T formed.
void qr_panel(double* P, int64_t lda, int64_t m, int nb, double* tau, double* T, double* V1,
              double* V2, int64_t ldv, const Sy2sbWs& w, hipStream_t s) {
  const int G = (int)ceil_div(m, QROWS);
  for (int c = 0; c <= nb; ++c) {
    if (G > 256)
      hipLaunchKernelGGL(panel_qr_step<32>, dim3(G), dim3(QT), 0, s, P, lda, m, nb, c, w.part, G,
                         tau);
    else
      hipLaunchKernelGGL(panel_qr_step<64>, dim3(G), dim3(QT), 0, s, P, lda, m, nb, c, w.part, G,
                         tau);
  }
  MM_HIP_TRY(hipGetLastError());
  const dim3 gv((unsigned)ceil_div(m * nb, 256));
  hipLaunchKernelGGL(extract_v, gv, dim3(256), 0, s, P, lda, m, nb, V1, ldv);
  hipLaunchKernelGGL(extract_v, gv, dim3(256), 0, s, P, lda, m, nb, V2, ldv);
  MM_HIP_TRY(hipGetLastError());
  Gemm gs;  // S = V^T V
  gs.m = nb; gs.n = nb; gs.k = m;
  gs.A = V1; gs.lda = ldv; gs.ta = true;
  gs.B = V1; gs.ldb = ldv;
  gs.C = w.Sm; gs.ldc = nb;
  gemm(gs, s, w.split, w.split_elems);
  hipLaunchKernelGGL(form_t, dim3(1), dim3(64), 0, s, w.Sm, tau, nb, T);
  MM_HIP_TRY(hipGetLastError());
}

// X = A22 V (A22 m x m symmetric, lower triangle stored) into w.X (ld ldv)
void sym_times_v(const double* A22, int64_t lda, int64_t m, int nb, const double* V,
                 int64_t ldv, const Sy2sbWs& w, hipStream_t s) {
  Gemm g;
  g.m = m; g.n = nb; g.k = m;
  g.A = A22; g.lda = lda; g.a_sym = true;
  g.B = V; g.ldb = ldv;
  g.C = w.X; g.ldc = ldv;
  gemm(g, s, w.split, w.split_elems);
}

// Y = X T - 1/2 V (T^T V^T X T)  (the two-sided update is A22 - V Y^T - Y V^T)
void form_y(const double* V, const double* T, int64_t m, int nb, double* Y, int64_t ldv,
            const Sy2sbWs& w, hipStream_t s) {
  Gemm g2;  // Y = X T  (T upper: op(B)(k,j) = 0 for k > j)
  g2.m = m; g2.n = nb; g2.k = nb;
  g2.A = w.X; g2.lda = ldv;
  g2.B = T; g2.ldb = nb; g2.b_band = 0;
  g2.C = Y; g2.ldc = ldv;
  gemm(g2, s);
  Gemm g3;  // Pm = V^T Y
  g3.m = nb; g3.n = nb; g3.k = m;
  g3.A = V; g3.lda = ldv; g3.ta = true;
  g3.B = Y; g3.ldb = ldv;
  g3.C = w.Pm; g3.ldc = nb;
  gemm(g3, s, w.split, w.split_elems);
  Gemm g4;  // Zm = T^T Pm
  g4.m = nb; g4.n = nb; g4.k = nb;
  g4.A = T; g4.lda = nb; g4.ta = true;
  g4.B = w.Pm; g4.ldb = nb;
  g4.C = w.Zm; g4.ldc = nb;
  gemm(g4, s);
  Gemm g5;  // Y -= 1/2 V Zm
  g5.m = m; g5.n = nb; g5.k = nb;
  g5.alpha = -0.5; g5.beta = 1.0;
  g5.A = V; g5.lda = ldv;
  g5.B = w.Zm; g5.ldb = nb;
  g5.C = Y; g5.ldc = ldv;
  gemm(g5, s);
}

// A -= U1 U2^T on the lower triangle (m x m, U1 and U2 m x k, ld ldu)
void lower_update(double* A, int64_t lda, int64_t m, int64_t k, const double* U1,
                  const double* U2, int64_t ldu, hipStream_t s) {
  Gemm g;
  g.m = m; g.n = m; g.k = k;
  g.alpha = -1.0; g.beta = 1.0;
  g.A = U1; g.lda = ldu;
  g.B = U2; g.ldb = ldu; g.tb = true;
  g.C = A; g.ldc = lda;
  g.lower = true;
  gemm(g, s);
}

}  // namespace

// Panels are taken in groups of up to GP.  Panel t of a group (columns
// j_t = j + (t-1) nb, rows R_t = [j_t + nb, n)) is reduced against the
// trailing matrix A as it was at the start of the group, corrected for the
// group's earlier panels s < t (whose updates A -= V_s Y_s^T + Y_s V_s^T are
// not yet applied):
//   * its columns (rows from j_t) receive those updates first;
//   * its product with the updated trailing matrix is
//       A'[R_t, R_t] V_t = A[R_t, R_t] V_t - U1[R_t] (U2[R_t]^T V_t),
//     with U1 = [V_1 Y_1 V_2 Y_2 ...] and U2 = [Y_1 V_1 Y_2 V_2 ...];
// and after the group's last panel q the trailing matrix A[R_q, R_q] receives
// all the group's updates at once, A -= U1 U2^T with k = 2 q nb.  V_s and Y_s
// are stored on the group's common rows [j + nb, n) from their own first row
// (j + s nb) on: every product above reads them at or below that row.
void sy2sb(double* A, int64_t lda, int64_t n, int nb, double* tau_all, double* T_all,
           double* ws, int64_t ws_elems, hipStream_t s) {
  MM_REQUIRE(nb >= 1 && nb <= MAXNB, kInvalid, "sy2sb: band must be 1..64");
  MM_REQUIRE(ws_elems >= sy2sb_ws_elems(n, nb), kInvalid, "sy2sb: workspace too small");
  const int64_t Gmax = ceil_div(n, QROWS);
  const int stride = nb + 1;
  Sy2sbWs w;
  w.part = ws;
  const int64_t np = ld16(n);
  w.X = w.part + 2 * (Gmax * stride + nb);           // np x nb
  w.Sm = w.X + np * nb;
  w.Pm = w.Sm + (int64_t)nb * nb;
  w.Zm = w.Pm + (int64_t)nb * nb;
  w.S2 = w.Zm + (int64_t)nb * nb;                    // 2 (GP - 1) nb x nb
  double* U1 = w.S2 + 2 * GP * (int64_t)nb * nb;     // np x 2 GP nb
  double* U2 = U1 + np * 2 * GP * nb;                // np x 2 GP nb
  w.split = U2 + np * 2 * GP * nb;
  w.split_elems = SPLIT_WS * n * nb;
  int64_t p = 0;
  for (int64_t j = 0; j + nb < n - 1;) {
    const int64_t m = n - (j + nb);  // rows of the group's first panel
    const int64_t mp = ld16(m);      // ld of U1, U2 and X
    // panels in this group: the next one joins while it has more than nb + 1 rows
    int q = 1;
    while (q < GP && j + (q + 2) * nb < n - 1) ++q;
    for (int t = 1; t <= q; ++t) {
      const int64_t jt = j + (t - 1) * nb;  // first column of panel t
      const int64_t rt = jt + nb;           // first row of R_t
      const int64_t mt = n - rt;
      const int64_t off = (t - 1) * nb;     // R_t on the common rows
      double* Tp = T_all + (p + t - 1) * (int64_t)nb * nb;
      double* V1 = U1 + (2 * t - 2) * nb * mp + off;
      double* Y1 = U1 + (2 * t - 1) * nb * mp + off;
      double* Y2 = U2 + (2 * t - 2) * nb * mp + off;
      double* V2 = U2 + (2 * t - 1) * nb * mp + off;
      const int64_t kprev = 2 * (int64_t)(t - 1) * nb;
      if (t > 1) {
        // panel t's columns, rows [jt, n) (R_{t-1}), get the group's updates so far
        Gemm g;
        g.m = n - jt; g.n = nb; g.k = kprev;
        g.alpha = -1.0; g.beta = 1.0;
        g.A = U1 + off - nb; g.lda = mp;
        g.B = U2 + off - nb; g.ldb = mp; g.tb = true;  // its first nb rows
        g.C = A + jt + jt * lda; g.ldc = lda;
        gemm(g, s);
      }
      qr_panel(A + rt + jt * lda, lda, mt, nb, tau_all + (p + t - 1) * nb, Tp, V1, V2, mp, w, s);
      sym_times_v(A + rt + rt * lda, lda, mt, nb, V1, mp, w, s);
      if (t > 1) {
        Gemm g;  // S2 = U2[R_t]^T V_t   (kprev x nb)
        g.m = kprev; g.n = nb; g.k = mt;
        g.A = U2 + off; g.lda = mp; g.ta = true;
        g.B = V1; g.ldb = mp;
        g.C = w.S2; g.ldc = kprev;
        gemm(g, s, w.split, w.split_elems);
        Gemm h;  // X -= U1[R_t] S2
        h.m = mt; h.n = nb; h.k = kprev;
        h.alpha = -1.0; h.beta = 1.0;
        h.A = U1 + off; h.lda = mp;
        h.B = w.S2; h.ldb = kprev;
        h.C = w.X; h.ldc = mp;
        gemm(h, s);
      }
      form_y(V1, Tp, mt, nb, Y1, mp, w, s);
      copy_matrix(Y1, mp, Y2, mp, mt, nb, s);
    }
    // the group's updates on the trailing matrix A[R_q, R_q]
    const int64_t rq = j + q * nb;
    const int64_t offq = (q - 1) * nb;
    lower_update(A + rq + rq * lda, lda, n - rq, 2 * (int64_t)q * nb, U1 + offq, U2 + offq, mp,
                 s);
    j += q * nb;
    p += q;
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
