// The resistance side of the pencil (Sec. 3.2, eq. generalized_eigenvalues_
// discrete as the paper writes it: Li v = tau Ri v).  R is sparse with a
// narrow band (a 7-point stencil on a grid: the band is the grid's row
// stride), so its Cholesky factor H is block bidiagonal in blocks of Bb >=
// the band:  H = [H_00; H_10 H_11; H_21 H_22; ...].  The factor costs
// O(n Bb^2), and every product with H^{-1} or H^{-T} is a chain of nblk
// matrix products of Bb rows (or columns), on the matrix cores.
//
// Storage: Hinv (nblk blocks of Bb x Bb) holds the inverses H_ii^{-1}
// (lower triangular), Hs (nblk blocks) the sub-diagonal blocks H_{i,i-1}
// (block 0 unused); both column-major, zero-padded past n.
#include "kernels.h"

#include <algorithm>

namespace mm {
namespace {

// Scatter the lower triangle of the logical R (offset honoured) into the
// diagonal blocks D (into Hinv's storage) and the sub-diagonal blocks S.
// One thread per logical row.  bad = 1 if an entry lies outside the two
// block diagonals (the band exceeds Bb).
__global__ void band_scatter_k(Csr R, int Bb, double* D, double* S, int64_t* bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= R.rows) return;
  const int64_t bi = i / Bb, ri = i % Bb;
  const int64_t bs = (int64_t)Bb * Bb;
  for (int64_t p = R.rowptr[i + R.off]; p < R.rowptr[i + R.off + 1]; ++p) {
    const int64_t j = (int64_t)R.col[p] - R.off;
    if (j < 0 || j > i) continue;
    const int64_t bj = j / Bb, cj = j % Bb;
    if (bj == bi) D[bi * bs + ri + cj * Bb] += R.val[p];
    else if (bj == bi - 1) S[bi * bs + ri + cj * Bb] += R.val[p];
    else *bad = 1;
  }
}

// Padding of the last diagonal block: unit diagonal past n, so that it
// factors and inverts as the identity there.
__global__ void band_pad_k(double* D, int64_t n, int Bb, int64_t nblk) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t last = (nblk - 1) * (int64_t)Bb;
  const int64_t r = last + q;
  if (q >= Bb || r < n) return;
  D[(nblk - 1) * (int64_t)Bb * Bb + q + q * (int64_t)Bb] = 1.0;
}

}  // namespace

int64_t band_block(int64_t band) {
  return std::max<int64_t>(64, ceil_div(std::max<int64_t>(band, 1), 64) * 64);
}

void band_factor(const Csr& R, int64_t n, int Bb, double* Hinv, double* Hs, double* ws,
                 int64_t ws_elems, int64_t* d_status, hipStream_t s) {
  const int64_t nblk = ceil_div(n, (int64_t)Bb);
  const int64_t bs = (int64_t)Bb * Bb;
  MM_REQUIRE(ws_elems >= band_factor_ws_elems(Bb), kInvalid, "band_factor: workspace");
  double* D = ws;                 // the current diagonal block, factored in place
  double* pws = ws + bs;          // potrf / trtri workspace
  const int64_t pwe = ws_elems - bs;
  fill(Hinv, nblk * bs, 0.0, s);
  fill(Hs, nblk * bs, 0.0, s);
  fill_i64(d_status, 1, 0, s);
  hipLaunchKernelGGL(band_scatter_k, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, R, Bb,
                     Hinv, Hs, d_status);
  hipLaunchKernelGGL(band_pad_k, dim3((unsigned)ceil_div(Bb, 256)), dim3(256), 0, s, Hinv, n,
                     Bb, nblk);
  MM_HIP_TRY(hipGetLastError());
  int64_t bad = 0;
  MM_HIP_TRY(hipMemcpyAsync(&bad, d_status, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MM_HIP_TRY(hipStreamSynchronize(s));
  MM_REQUIRE(bad == 0, kInvalid, "R: an entry lies outside the band");
  fill_i64(d_status, 1, INT64_MAX, s);
  for (int64_t i = 0; i < nblk; ++i) {
    double* Di = Hinv + i * bs;  // R_ii on entry, H_ii^{-1} on exit
    if (i > 0) {
      // R_ii -= H_{i,i-1} H_{i,i-1}^T   (lower triangle)
      Gemm g;
      g.m = Bb; g.n = Bb; g.k = Bb;
      g.alpha = -1.0; g.beta = 1.0;
      g.A = Hs + i * bs; g.lda = Bb;
      g.B = Hs + i * bs; g.ldb = Bb; g.tb = true;
      g.C = Di; g.ldc = Bb;
      g.lower = true;
      gemm(g, s);
    }
    potrf_lower(Di, Bb, Bb, pws, pwe, d_status, s);  // Di = H_ii (strict upper zeroed)
    trtri_lower(Di, Bb, Bb, pws, pwe, s);            // Di = H_ii^{-1}
    if (i + 1 < nblk) {
      // H_{i+1,i} = R_{i+1,i} H_ii^{-T}:  S <- S Di^T, through D as scratch
      double* Si = Hs + (i + 1) * bs;
      copy_matrix(Si, Bb, D, Bb, Bb, Bb, s);
      Gemm g;
      g.m = Bb; g.n = Bb; g.k = Bb;
      g.A = D; g.lda = Bb;
      g.B = Di; g.ldb = Bb; g.tb = true;
      g.b_band = 0;  // Di^T is upper triangular: op(B)(k, j) = 0 for k > j
      g.C = Si; g.ldc = Bb;
      gemm(g, s);
    }
  }
}

int64_t band_factor_ws_elems(int Bb) {
  return (int64_t)Bb * Bb + std::max(potrf_ws_elems(Bb), trtri_ws_elems(Bb));
}

// X <- H^{-1} X (X: n x ncols, ld ldx), block rows top down:
//   X_i <- H_ii^{-1} (X_i - H_{i,i-1} X_{i-1});  tmp holds Bb x ncols.
void band_solve_left(const double* Hinv, const double* Hs, int64_t n, int Bb, double* X,
                     int64_t ldx, int64_t ncols, double* tmp, hipStream_t s) {
  const int64_t nblk = ceil_div(n, (int64_t)Bb);
  const int64_t bs = (int64_t)Bb * Bb;
  if (ncols <= 0) return;
  for (int64_t i = 0; i < nblk; ++i) {
    const int64_t r0 = i * Bb, rows = std::min<int64_t>(Bb, n - r0);
    if (i > 0) {
      Gemm g;
      g.m = rows; g.n = ncols; g.k = Bb;
      g.alpha = -1.0; g.beta = 1.0;
      g.A = Hs + i * bs; g.lda = Bb;
      g.B = X + r0 - Bb; g.ldb = ldx;
      g.C = X + r0; g.ldc = ldx;
      gemm(g, s);
    }
    Gemm g;
    g.m = rows; g.n = ncols; g.k = rows;
    g.A = Hinv + i * bs; g.lda = Bb; g.a_lower = true;
    g.B = X + r0; g.ldb = ldx;
    g.C = tmp; g.ldc = Bb;
    gemm(g, s);
    copy_matrix(tmp, Bb, X + r0, ldx, rows, ncols, s);
  }
}

// X <- H^{-T} X, block rows bottom up:
//   X_i <- H_ii^{-T} (X_i - H_{i+1,i}^T X_{i+1}).
void band_solve_left_t(const double* Hinv, const double* Hs, int64_t n, int Bb, double* X,
                       int64_t ldx, int64_t ncols, double* tmp, hipStream_t s) {
  const int64_t nblk = ceil_div(n, (int64_t)Bb);
  const int64_t bs = (int64_t)Bb * Bb;
  if (ncols <= 0) return;
  for (int64_t i = nblk - 1; i >= 0; --i) {
    const int64_t r0 = i * Bb, rows = std::min<int64_t>(Bb, n - r0);
    if (i + 1 < nblk) {
      const int64_t rows1 = std::min<int64_t>(Bb, n - r0 - Bb);
      Gemm g;
      g.m = rows; g.n = ncols; g.k = rows1;
      g.alpha = -1.0; g.beta = 1.0;
      g.A = Hs + (i + 1) * bs; g.lda = Bb; g.ta = true;
      g.B = X + r0 + Bb; g.ldb = ldx;
      g.C = X + r0; g.ldc = ldx;
      gemm(g, s);
    }
    Gemm g;
    g.m = rows; g.n = ncols; g.k = rows;
    g.A = Hinv + i * bs; g.lda = Bb; g.ta = true; g.a_upper = true;
    g.B = X + r0; g.ldb = ldx;
    g.C = tmp; g.ldc = Bb;
    gemm(g, s);
    copy_matrix(tmp, Bb, X + r0, ldx, rows, ncols, s);
  }
}

// X <- X H^{-T} (X: nrows x n, ld ldx), block columns left to right:
//   X_j <- (X_j - X_{j-1} H_{j,j-1}^T) H_jj^{-T};  tmp holds nrows x Bb.
void band_solve_right_t(const double* Hinv, const double* Hs, int64_t n, int Bb, double* X,
                        int64_t ldx, int64_t nrows, double* tmp, hipStream_t s) {
  const int64_t nblk = ceil_div(n, (int64_t)Bb);
  const int64_t bs = (int64_t)Bb * Bb;
  if (nrows <= 0) return;
  for (int64_t j = 0; j < nblk; ++j) {
    const int64_t c0 = j * Bb, cols = std::min<int64_t>(Bb, n - c0);
    if (j > 0) {
      Gemm g;
      g.m = nrows; g.n = cols; g.k = Bb;
      g.alpha = -1.0; g.beta = 1.0;
      g.A = X + (c0 - Bb) * ldx; g.lda = ldx;
      g.B = Hs + j * bs; g.ldb = Bb; g.tb = true;
      g.C = X + c0 * ldx; g.ldc = ldx;
      gemm(g, s);
    }
    Gemm g;
    g.m = nrows; g.n = cols; g.k = cols;
    g.A = X + c0 * ldx; g.lda = ldx;
    g.B = Hinv + j * bs; g.ldb = Bb; g.tb = true;
    g.b_band = 0;  // H_jj^{-T} is upper triangular
    g.C = tmp; g.ldc = nrows;
    gemm(g, s);
    copy_matrix(tmp, nrows, X + c0 * ldx, ldx, nrows, cols, s);
  }
}

namespace {

// Eigen-decomposition of a symmetric k x k matrix (k <= 8, column-major) by
// cyclic Jacobi, in one thread: A is overwritten by its eigenvalues on the
// diagonal, W receives the eigenvectors (columns).
__device__ void small_jacobi(double* A, double* W, int k) {
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) W[i + j * k] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) {
        tot += A[i + j * k] * A[i + j * k];
        if (i != j) off += A[i + j * k] * A[i + j * k];
      }
    if (off <= 1e-32 * tot) break;
    for (int p = 0; p < k - 1; ++p)
      for (int q = p + 1; q < k; ++q) {
        const double apq = A[p + q * k];
        if (apq == 0.0) continue;
        const double th = (A[q + q * k] - A[p + p * k]) / (2.0 * apq);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
        const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
        for (int r = 0; r < k; ++r) {  // columns p, q
          const double a = A[r + p * k], b = A[r + q * k];
          A[r + p * k] = c * a - s * b;
          A[r + q * k] = s * a + c * b;
        }
        for (int r = 0; r < k; ++r) {  // rows p, q
          const double a = A[p + r * k], b = A[q + r * k];
          A[p + r * k] = c * a - s * b;
          A[q + r * k] = s * a + c * b;
        }
        for (int r = 0; r < k; ++r) {
          const double a = W[r + p * k], b = W[r + q * k];
          W[r + p * k] = c * a - s * b;
          W[r + q * k] = s * a + c * b;
        }
      }
  }
}

// A = I + Z S Z^T with S = -[[0, I_m], [I_m, 0]] (the reduced resistance's
// low-rank term relative to R's trailing block, in H's coordinates).  Given
// Gz = Z^T Z (k x k, k = 2m), writes Gamma with A^{-1/2} = I + Z Gamma Z^T:
// with Gz = W D W^T and U = Z W D^{-1/2} (orthonormal on D > 0),
// A = I + U B U^T, B = D^{1/2} W^T S W D^{1/2}, and with I + B = Wb Db Wb^T,
// Gamma = W D^{-1/2} Wb (Db^{-1/2} - I) Wb^T D^{-1/2} W^T.  bad = 1 if
// I + B is not positive definite.
__global__ void lowrank_gamma_k(const double* Gz, int m, double* Gamma, int64_t* bad) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int k = 2 * m;
  double A[64], W[64], B[64], Wb[64], T[64];
  for (int e = 0; e < k * k; ++e) A[e] = Gz[e];
  small_jacobi(A, W, k);
  double dmax = 0.0;
  for (int i = 0; i < k; ++i) dmax = fmax(dmax, A[i + i * k]);
  double ds[8];  // D^{1/2} on the kept directions, 0 on the dropped ones
  for (int i = 0; i < k; ++i) {
    const double d = A[i + i * k];
    ds[i] = d > 1e-14 * dmax ? sqrt(d) : 0.0;
  }
  // B = D^{1/2} W^T S W D^{1/2};  (S W)(r, j) = -W(r +- m, j)
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      double acc = 0.0;
      for (int r = 0; r < k; ++r) {
        const double swrj = -(r < m ? W[(r + m) + j * k] : W[(r - m) + j * k]);
        acc += W[r + i * k] * swrj;
      }
      B[i + j * k] = ds[i] * acc * ds[j] + (i == j ? 1.0 : 0.0);
    }
  small_jacobi(B, Wb, k);
  // T = Wb (Db^{-1/2} - I) Wb^T, on the kept directions only
  for (int i = 0; i < k; ++i)
    if (ds[i] > 0.0 && B[i + i * k] <= 0.0) *bad = 1;
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      double acc = 0.0;
      for (int q = 0; q < k; ++q) {
        const double db = B[q + q * k];
        const double f = db > 0.0 ? 1.0 / sqrt(db) - 1.0 : 0.0;
        acc += Wb[i + q * k] * f * Wb[j + q * k];
      }
      T[i + j * k] = acc;
    }
  // Gamma = W D^{-1/2} T D^{-1/2} W^T
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      double acc = 0.0;
      for (int p = 0; p < k; ++p) {
        if (ds[p] == 0.0) continue;
        for (int q = 0; q < k; ++q) {
          if (ds[q] == 0.0) continue;
          acc += W[i + p * k] * (T[p + q * k] / (ds[p] * ds[q])) * W[j + q * k];
        }
      }
      Gamma[i + j * k] = acc;
    }
}

// K = Gamma Qm Gamma / 2 (k x k)
__global__ void lowrank_gqg_k(const double* Gamma, const double* Qm, int k, double* K) {
  const int i = threadIdx.x % 8, j = threadIdx.x / 8;
  if (i >= k || j >= k) return;
  double acc = 0.0;
  for (int p = 0; p < k; ++p)
    for (int q = 0; q < k; ++q) acc += Gamma[i + p * k] * Qm[p + q * k] * Gamma[q + j * k];
  K[i + j * k] = 0.5 * acc;
}

// Modes from the time constants (tau ascending, eigenvector j of C' in
// column j): mode n takes tau index r = n0 - 1 - n, lam_n = 1 / tau_r, and
// its projected weights are tau_r^{-1/2} ZY(r, :).
__global__ void modes_from_tau_k(const double* tau, const double* ZY, int64_t n0, int nf,
                                 int np, double* lam, double* W, double* P) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= n0) return;
  const int64_t r = n0 - 1 - n;
  const double t = tau[r];
  lam[n] = 1.0 / t;
  const double sc = 1.0 / sqrt(t);
  for (int j = 0; j < nf; ++j) W[n + (int64_t)j * n0] = sc * ZY[r + (int64_t)j * n0];
  for (int p = 0; p < np; ++p) P[n + (int64_t)p * n0] = sc * ZY[r + (int64_t)(nf + p) * n0];
}

// Columns in the modes' order, scaled: V(:, n) = tau_r^{-1/2} X(:, r),
// r = n0 - 1 - n, in place (pairs of columns swapped); lam_n = 1 / tau_r.
__global__ void reverse_scale_cols_k(double* X, int64_t ld, int64_t n0, const double* tau,
                                     double* lam) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t n = blockIdx.y; n <= (n0 - 1) / 2; n += gridDim.y) {
    const int64_t r = n0 - 1 - n;
    const double sn = 1.0 / sqrt(tau[n]), sr = 1.0 / sqrt(tau[r]);
    if (i < n0) {
      const double a = X[i + n * ld], b = X[i + r * ld];
      X[i + n * ld] = sr * b;
      X[i + r * ld] = sn * a;
    }
    if (i == 0) {
      lam[n] = 1.0 / tau[r];
      lam[r] = 1.0 / tau[n];
    }
  }
}

}  // namespace

void lowrank_gamma(const double* Gz, int m, double* Gamma, int64_t* d_bad, hipStream_t s) {
  MM_REQUIRE(m >= 1 && m <= 4, kInvalid, "lowrank_gamma: 1 <= m <= 4");
  hipLaunchKernelGGL(lowrank_gamma_k, dim3(1), dim3(64), 0, s, Gz, m, Gamma, d_bad);
  MM_HIP_TRY(hipGetLastError());
}

void lowrank_gqg(const double* Gamma, const double* Qm, int k, double* K, hipStream_t s) {
  MM_REQUIRE(k >= 1 && k <= 8, kInvalid, "lowrank_gqg: 1 <= k <= 8");
  hipLaunchKernelGGL(lowrank_gqg_k, dim3(1), dim3(64), 0, s, Gamma, Qm, k, K);
  MM_HIP_TRY(hipGetLastError());
}

void modes_from_tau(const double* tau, const double* ZY, int64_t n0, int nf, int np,
                    double* lam, double* W, double* P, hipStream_t s) {
  if (n0 <= 0) return;
  hipLaunchKernelGGL(modes_from_tau_k, dim3((unsigned)ceil_div(n0, 256)), dim3(256), 0, s, tau,
                     ZY, n0, nf, np, lam, W, P);
  MM_HIP_TRY(hipGetLastError());
}

void reverse_scale_cols(double* X, int64_t ld, int64_t n0, const double* tau, double* lam,
                        hipStream_t s) {
  if (n0 <= 0) return;
  const unsigned gy = (unsigned)std::min<int64_t>(65535, (n0 + 1) / 2);
  hipLaunchKernelGGL(reverse_scale_cols_k, dim3((unsigned)ceil_div(n0, 256), gy), dim3(256), 0,
                     s, X, ld, n0, tau, lam);
  MM_HIP_TRY(hipGetLastError());
}

}  // namespace mm
