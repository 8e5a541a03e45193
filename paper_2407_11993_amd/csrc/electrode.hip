// Electrode reduction (Sec. 3.1, the injected-current decomposition): the
// currents split as  I = K Ii + A_D iD,  with K an orthonormal basis of
// X_0 = ker E and A_D = E^T (E E^T)^{-1}.  K is the Householder complement of
// im E^T:  E^T = H [Re; 0],  H = H_0 ... H_{m-1} = I - V T V^T,  K = H[:, m:],
// and A_D = H [Re^{-T}; 0].  The reduced matrices are the trailing blocks of
// the two-sided products, K^T A K = (H^T A H)[m:, m:], and
// H^T A H = A - V Y^T - Y V^T  with  Y = X T - 1/2 V (T^T V^T X T),  X = A V.
// V is non-zero only on the electrode cells and the first m rows, so the
// correction of the sparse resistance stays sparse.
#include "kernels.h"

namespace mm {
namespace {

constexpr int QT = 1024;  // threads of the single-workgroup QR kernels
constexpr int MAXM = 8;

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the QT threads; every thread gets the result.
__device__ double block_sum(double v, double* sh) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  v = wsum(v);
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < QT / 64; ++w) s += sh[w];
  return s;
}

// E^T as a dense n x m column-major block (A zeroed beforehand).
__global__ void e_dense_k(Csr E, int64_t n, double* A) {
  const int a = blockIdx.x;
  for (int64_t p = E.rowptr[a] + threadIdx.x; p < E.rowptr[a + 1]; p += blockDim.x)
    A[E.col[p] + (int64_t)a * n] = E.val[p];
}

// Householder step j of the QR of A = E^T (n x m): H_j = I - tau v v^T with
// v(j) = 1 maps A(j:, j) onto beta e_j; it is applied to the columns c > j.
// A(j, c) for c >= j then holds row j of Re.
__global__ void __launch_bounds__(QT) hh_step_k(double* A, int64_t n, int m, int j, Csr E,
                                                double* V, double* tau, int64_t* status) {
  __shared__ double sh[QT / 64];
  const int t = threadIdx.x;
  double* a = A + (int64_t)j * n;
  double s2 = 0.0;
  for (int64_t i = j + 1 + t; i < n; i += QT) s2 += a[i] * a[i];
  s2 = block_sum(s2, sh);
  double e2 = 0.0;  // squared norm of row j of E as given (rank test scale)
  for (int64_t p = E.rowptr[j] + t; p < E.rowptr[j + 1]; p += QT) e2 += E.val[p] * E.val[p];
  e2 = block_sum(e2, sh);
  const double a0 = a[j];
  const double nrm = sqrt(a0 * a0 + s2);
  if (!(nrm > 1e-12 * sqrt(e2))) {  // what is left of row j: linearly dependent
    for (int64_t i = t; i < n; i += QT) V[i + (int64_t)j * n] = (i == j) ? 1.0 : 0.0;
    if (t == 0) {
      tau[j] = 0.0;
      *status = 1;
    }
    return;
  }
  double tv = 0.0, beta = a0, scale = 0.0;
  if (s2 > 0.0) {
    beta = -copysign(nrm, a0);
    tv = (beta - a0) / beta;
    scale = 1.0 / (a0 - beta);
  }
  for (int64_t i = t; i < n; i += QT)
    V[i + (int64_t)j * n] = (i < j) ? 0.0 : (i == j ? 1.0 : a[i] * scale);
  for (int c = j + 1; c < m; ++c) {
    double* ac = A + (int64_t)c * n;
    const double acj = ac[j];  // read before the barriers: row j is updated below
    double d = 0.0;
    for (int64_t i = j + 1 + t; i < n; i += QT) d += a[i] * scale * ac[i];
    d = block_sum(d, sh) + acj;
    const double f = tv * d;
    for (int64_t i = j + t; i < n; i += QT) ac[i] -= f * (i == j ? 1.0 : a[i] * scale);
    __syncthreads();
  }
  __syncthreads();
  if (t == 0) {
    a[j] = beta;
    tau[j] = tv;
  }
}

// T of H = I - V T V^T from tau and S = V^T V (forward recurrence
// T(c,c) = tau_c, T(0:c, c) = -tau_c T(0:c, 0:c) S(0:c, c)), and Re^{-T}.
__global__ void __launch_bounds__(QT) hh_finish_k(const double* V, int64_t n, int m,
                                                  const double* tau, const double* A,
                                                  double* small) {
  __shared__ double sh[QT / 64];
  __shared__ double S[MAXM][MAXM];
  const int t = threadIdx.x;
  for (int a = 0; a < m; ++a)
    for (int b = a; b < m; ++b) {
      double d = 0.0;
      for (int64_t i = t; i < n; i += QT) d += V[i + (int64_t)a * n] * V[i + (int64_t)b * n];
      d = block_sum(d, sh);
      if (t == 0) S[a][b] = S[b][a] = d;
    }
  __syncthreads();
  if (t != 0) return;
  double* T = small;
  double* RinvT = small + m * m;
  for (int e = 0; e < m * m; ++e) T[e] = 0.0;
  for (int c = 0; c < m; ++c) {
    double col[MAXM];
    for (int r = 0; r < c; ++r) {
      double s = 0.0;
      for (int q = r; q < c; ++q) s += T[r + q * m] * S[q][c];
      col[r] = -tau[c] * s;
    }
    for (int r = 0; r < c; ++r) T[r + c * m] = col[r];
    T[c + c * m] = tau[c];
  }
  // Re(r, c) = A(r, c) for c >= r.  X = Re^{-T} is lower triangular:
  // Re^T X = I, row i: sum_{k <= i} Re(k, i) X(k, e) = delta_ie.
  for (int e = 0; e < m; ++e)
    for (int i = 0; i < m; ++i) {
      if (i < e) {
        RinvT[i + e * m] = 0.0;
        continue;
      }
      double s = (i == e) ? 1.0 : 0.0;
      for (int k = e; k < i; ++k) s -= A[k + (int64_t)i * n] * RinvT[k + e * m];
      RinvT[i + e * m] = s / A[i + (int64_t)i * n];
    }
}

__global__ void l_times_rows_k(LSrc src, int64_t n, const int32_t* __restrict__ idx, int ns,
                               const double* __restrict__ U, int64_t ldu, int k,
                               double* __restrict__ out, int64_t ldo) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double xi = 0.0, yi = 0.0, zi = 0.0;
  if (!src.L) {
    xi = src.xyz[3 * i]; yi = src.xyz[3 * i + 1]; zi = src.xyz[3 * i + 2];
  }
  const double h2 = src.h * src.h;
  double acc[MAXM];
#pragma unroll
  for (int c = 0; c < MAXM; ++c) acc[c] = 0.0;
  for (int q = 0; q < ns; ++q) {
    const int64_t s = idx[q];
    double l;
    if (src.L) {  // lower triangle of the borrowed matrix (off = 0 here)
      l = i >= s ? src.L[i + s * src.ld] : src.L[s + i * src.ld];
    } else {
      const double dx = xi - src.xyz[3 * s], dy = yi - src.xyz[3 * s + 1],
                   dz = zi - src.xyz[3 * s + 2];
      l = src.h / sqrt(dx * dx + dy * dy + dz * dz + h2);
    }
#pragma unroll
    for (int c = 0; c < MAXM; ++c)
      if (c < k) acc[c] += l * U[s + c * ldu];
  }
#pragma unroll
  for (int c = 0; c < MAXM; ++c)
    if (c < k) out[i + c * ldo] = acc[c];
}

__global__ void csr_times_dense_k(Csr R, const double* __restrict__ U, int64_t ldu, int k,
                                  double* __restrict__ out, int64_t ldo) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= R.rows) return;
  double acc[MAXM];
#pragma unroll
  for (int c = 0; c < MAXM; ++c) acc[c] = 0.0;
  for (int64_t p = R.rowptr[i + R.off]; p < R.rowptr[i + R.off + 1]; ++p) {
    const int64_t j = (int64_t)R.col[p] - R.off;
    if (j < 0) continue;
    const double v = R.val[p];
#pragma unroll
    for (int c = 0; c < MAXM; ++c)
      if (c < k) acc[c] += v * U[j + c * ldu];
  }
#pragma unroll
  for (int c = 0; c < MAXM; ++c)
    if (c < k) out[i + c * ldo] = acc[c];
}

__global__ void lift_k(const double* RinvT, const double* iD, int m, const double* Ii,
                       int64_t n0, double* z) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m + n0) return;
  if (e < m) {
    double s = 0.0;
    for (int b = 0; b < m; ++b) s += RinvT[e + b * m] * iD[b];
    z[e] = s;
  } else {
    z[e] = Ii[e - m];
  }
}

__global__ void mark_rows_k(const double* A, const double* B, int64_t ld, int64_t rows, int k,
                            unsigned char* mark) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  unsigned char f = 0;
  for (int c = 0; c < k; ++c) f |= (A[i + c * ld] != 0.0) || (B[i + c * ld] != 0.0);
  mark[i] = f;
}

__global__ void gather_rows_k(const double* S, int64_t lds, const int32_t* idx, int ns, int k,
                              double* D) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)ns * k) return;
  const int j = (int)(e % ns), c = (int)(e / ns);
  D[e] = S[idx[j] + (int64_t)c * lds];
}

unsigned blocks(int64_t count) { return (unsigned)std::max<int64_t>(1, ceil_div(count, 256)); }

}  // namespace

void electrode_qr(const Csr& E, int64_t n, int m, double* V, double* small, double* work,
                  int64_t* d_status, hipStream_t s) {
  MM_REQUIRE(m >= 1 && m <= MAXM && m < n, kInvalid, "electrode_qr: 1 <= m <= 8, m < n");
  double* A = work;       // n x m: E^T, then the QR's working copy
  double* tau = small + 2 * m * m;  // m entries after [T | Re^{-T}]
  fill(A, n * m, 0.0, s);
  hipLaunchKernelGGL(e_dense_k, dim3(m), dim3(256), 0, s, E, n, A);
  for (int j = 0; j < m; ++j)
    hipLaunchKernelGGL(hh_step_k, dim3(1), dim3(QT), 0, s, A, n, m, j, E, V, tau, d_status);
  hipLaunchKernelGGL(hh_finish_k, dim3(1), dim3(QT), 0, s, V, n, m, tau, A, small);
  MM_HIP_TRY(hipGetLastError());
}

int64_t apply_h_ws_elems(int m, int64_t k) { return 2 * m * k + 256 * m * k; }

void apply_h(const double* V, const double* T, int64_t n, int m, double* X, int64_t ldx,
             int64_t k, bool trans, double* ws, int64_t ws_elems, hipStream_t s) {
  if (m == 0 || k == 0) return;
  MM_REQUIRE(ws_elems >= apply_h_ws_elems(m, k), kInvalid, "apply_h: workspace too small");
  double* W1 = ws;
  double* W2 = ws + m * k;
  double* split = ws + 2 * m * k;
  const int64_t split_elems = ws_elems - 2 * m * k;
  Gemm g1;  // W1 = V^T X
  g1.m = m; g1.n = k; g1.k = n;
  g1.A = V; g1.lda = n; g1.ta = true;
  g1.B = X; g1.ldb = ldx;
  g1.C = W1; g1.ldc = m;
  gemm(g1, s, split, split_elems);
  Gemm g2;  // W2 = op(T) W1   (H^T = I - V T^T V^T)
  g2.m = m; g2.n = k; g2.k = m;
  g2.A = T; g2.lda = m; g2.ta = trans;
  g2.B = W1; g2.ldb = m;
  g2.C = W2; g2.ldc = m;
  gemm(g2, s);
  Gemm g3;  // X -= V W2
  g3.m = n; g3.n = k; g3.k = m;
  g3.alpha = -1.0; g3.beta = 1.0;
  g3.A = V; g3.lda = n;
  g3.B = W2; g3.ldb = m;
  g3.C = X; g3.ldc = ldx;
  gemm(g3, s);
}

void two_sided_y(const double* V, const double* T, int64_t n, int m, const double* X,
                 double* Y, double* ws, int64_t ws_elems, hipStream_t s) {
  MM_REQUIRE(ws_elems >= 2 * m * m + 256 * m * m, kInvalid, "two_sided_y: workspace too small");
  double* P = ws;
  double* Zm = ws + m * m;
  double* split = ws + 2 * m * m;
  Gemm g1;  // Y = X T
  g1.m = n; g1.n = m; g1.k = m;
  g1.A = X; g1.lda = n;
  g1.B = T; g1.ldb = m;
  g1.C = Y; g1.ldc = n;
  gemm(g1, s);
  Gemm g2;  // P = V^T Y
  g2.m = m; g2.n = m; g2.k = n;
  g2.A = V; g2.lda = n; g2.ta = true;
  g2.B = Y; g2.ldb = n;
  g2.C = P; g2.ldc = m;
  gemm(g2, s, split, ws_elems - 2 * m * m);
  Gemm g3;  // Zm = T^T P
  g3.m = m; g3.n = m; g3.k = m;
  g3.A = T; g3.lda = m; g3.ta = true;
  g3.B = P; g3.ldb = m;
  g3.C = Zm; g3.ldc = m;
  gemm(g3, s);
  Gemm g4;  // Y -= 1/2 V Zm
  g4.m = n; g4.n = m; g4.k = m;
  g4.alpha = -0.5; g4.beta = 1.0;
  g4.A = V; g4.lda = n;
  g4.B = Zm; g4.ldb = m;
  g4.C = Y; g4.ldc = n;
  gemm(g4, s);
}

void l_times_rows(const LSrc& src, int64_t n, const int32_t* idx, int ns,
                  const double* U, int64_t ldu, int k, double* out, int64_t ldo,
                  hipStream_t s) {
  MM_REQUIRE(k >= 1 && k <= MAXM, kInvalid, "l_times_rows: 1 <= k <= 8");
  MM_REQUIRE(src.off == 0, kInvalid, "l_times_rows: the full matrix only");
  hipLaunchKernelGGL(l_times_rows_k, dim3(blocks(n)), dim3(256), 0, s, src, n, idx, ns, U,
                     ldu, k, out, ldo);
  MM_HIP_TRY(hipGetLastError());
}

void csr_times_dense(const Csr& R, const double* U, int64_t ldu, int k, double* out,
                     int64_t ldo, hipStream_t s) {
  MM_REQUIRE(k >= 1 && k <= MAXM, kInvalid, "csr_times_dense: 1 <= k <= 8");
  hipLaunchKernelGGL(csr_times_dense_k, dim3(blocks(R.rows)), dim3(256), 0, s, R, U, ldu, k,
                     out, ldo);
  MM_HIP_TRY(hipGetLastError());
}

void electrode_lift(const double* RinvT, const double* iD, int m, const double* Ii,
                    int64_t n0, double* z, hipStream_t s) {
  hipLaunchKernelGGL(lift_k, dim3(blocks(m + n0)), dim3(256), 0, s, RinvT, iD, m, Ii, n0, z);
  MM_HIP_TRY(hipGetLastError());
}

void mark_rows(const double* A, const double* B, int64_t ld, int64_t rows, int k,
               unsigned char* mark, hipStream_t s) {
  hipLaunchKernelGGL(mark_rows_k, dim3(blocks(rows)), dim3(256), 0, s, A, B, ld, rows, k, mark);
  MM_HIP_TRY(hipGetLastError());
}

void gather_rows(const double* S, int64_t lds, const int32_t* idx, int ns, int k, double* D,
                 hipStream_t s) {
  if (ns <= 0) return;
  hipLaunchKernelGGL(gather_rows_k, dim3(blocks((int64_t)ns * k)), dim3(256), 0, s, S, lds, idx,
                     ns, k, D);
  MM_HIP_TRY(hipGetLastError());
}

}  // namespace mm
