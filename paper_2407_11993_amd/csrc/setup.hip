// Setup kernels: assembly of the inductance stand-in (HBM-write bound),
// sparse R operations of the standard form, small fills.
#include "kernels.h"

namespace mm {
namespace {

// One thread per element of a column segment; consecutive threads walk
// consecutive rows, so the column-major stores (and, from a borrowed matrix,
// the loads) are contiguous.  The optional symmetric low-rank term (the
// electrode reduction's two-sided Householder update) is subtracted on the fly.
__device__ __forceinline__ double l_entry(const LSrc& src, int64_t i, int64_t j, double xj,
                                          double yj, double zj) {
  if (src.L) {  // lower triangle of the borrowed matrix
    const int64_t r = i >= j ? i : j, c = i >= j ? j : i;
    return src.L[(r + src.off) + (c + src.off) * src.ld];
  }
  const double* x = src.xyz + 3 * (i + src.off);
  const double dx = x[0] - xj, dy = x[1] - yj, dz = x[2] - zj;
  return src.h / sqrt(dx * dx + dy * dy + dz * dz + src.h * src.h);
}

__global__ void assemble_L_k(LSrc src, int64_t n, double* __restrict__ L, int64_t ld, int full,
                             LowRank lr) {
  const int64_t j = blockIdx.x;
  double xj = 0.0, yj = 0.0, zj = 0.0;
  if (!src.L) {
    const double* x = src.xyz + 3 * (j + src.off);
    xj = x[0]; yj = x[1]; zj = x[2];
  }
  double uj[8], yj_[8];
  for (int a = 0; a < lr.m; ++a) {
    uj[a] = lr.U[j + a * lr.ld];
    yj_[a] = lr.Y1[j + a * lr.ld] + (lr.Y2 ? lr.w2 * lr.Y2[j + a * lr.ld] : 0.0);
  }
  const int64_t i_begin = full ? 0 : j;
  for (int64_t i = i_begin + threadIdx.x; i < n; i += blockDim.x) {
    double v = l_entry(src, i, j, xj, yj, zj);
    for (int a = 0; a < lr.m; ++a) {
      const double ui = lr.U[i + a * lr.ld];
      const double yi = lr.Y1[i + a * lr.ld] + (lr.Y2 ? lr.w2 * lr.Y2[i + a * lr.ld] : 0.0);
      v -= ui * yj_[a] + yi * uj[a];
    }
    L[i + j * ld] = v;
  }
}

// Grid-stride scan; any non-finite value sets the flag (a plain store of 1:
// every writer writes the same value).
__global__ void flag_nonfinite_k(const double* __restrict__ p, int64_t count,
                                 int64_t* __restrict__ flag) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    bad |= !isfinite(p[i]);
  if (bad) *flag = 1;
}

// One workgroup per column j, rows j..n-1.
__global__ void flag_nonfinite_lower_k(const double* __restrict__ A, int64_t lda, int64_t n,
                                       int64_t* __restrict__ flag) {
  bool bad = false;
  for (int64_t j = blockIdx.x; j < n; j += gridDim.x)
    for (int64_t i = j + threadIdx.x; i < n; i += blockDim.x) bad |= !isfinite(A[i + j * lda]);
  if (bad) *flag = 1;
}

__global__ void add_csr_lower_k(double* Z, int64_t ld, double alpha, Csr R) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= R.rows) return;
  for (int64_t p = R.rowptr[i + R.off]; p < R.rowptr[i + R.off + 1]; ++p) {
    const int64_t j = (int64_t)R.col[p] - R.off;
    if (j >= 0 && j <= i) Z[i + j * ld] += alpha * R.val[p];
  }
}

__global__ void csr_band_k(int64_t rows, const int64_t* rowptr, const int32_t* col,
                           unsigned long long* out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= rows) return;
  int64_t mn = j;
  for (int64_t p = rowptr[j]; p < rowptr[j + 1]; ++p) mn = min(mn, (int64_t)col[p]);
  atomicMax(out, (unsigned long long)(j - mn));
}

// W(:, j) = sum_{p in row j of R} R(j, c_p) A(:, c_p)   (R symmetric, logical
// indices: stored row j + off, columns c >= off shifted by off)
__global__ void dense_times_csr_k(const double* __restrict__ A, int64_t lda, Csr R, int64_t n,
                                  double* __restrict__ W, int64_t ldw) {
  const int64_t j = blockIdx.x;
  const int64_t p0 = R.rowptr[j + R.off], p1 = R.rowptr[j + R.off + 1];
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    double s = 0.0;
    for (int64_t p = p0; p < p1; ++p) {
      const int64_t c = (int64_t)R.col[p] - R.off;
      if (c >= 0) s += R.val[p] * A[i + c * lda];
    }
    W[i + j * ldw] = s;
  }
}

// Tiled transpose-copy of the lower triangle into the upper one.
__global__ void symmetrize_k(double* A, int64_t lda, int64_t n) {
  __shared__ double tile[32][33];
  const int64_t bi = blockIdx.x, bj = blockIdx.y;  // tile (bi, bj), bi > bj or ==
  if (bi < bj) return;
  const int tx = threadIdx.x, ty = threadIdx.y;  // 32 x 8
  // read lower tile (rows bi*32.., cols bj*32..)
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = bi * 32 + tx, j = bj * 32 + r;
    if (i < n && j < n) tile[r][tx] = A[i + j * lda];
  }
  __syncthreads();
  // write to upper tile (rows bj*32.., cols bi*32..): A(j, i) = A(i, j)
  for (int r = ty; r < 32; r += 8) {
    const int64_t j = bj * 32 + tx, i = bi * 32 + r;  // element (row j, col i)
    if (i < n && j < n && j < i) A[j + i * lda] = tile[tx][r];
  }
}

__global__ void fill_k(double* p, int64_t count, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void fill_i64_k(int64_t* p, int64_t count, int64_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

unsigned grid1(int64_t count, int per = 256) {
  int64_t g = ceil_div(count, per);
  if (g > 65535 * 16) g = 65535 * 16;
  return (unsigned)std::max<int64_t>(g, 1);
}

}  // namespace

void assemble_L(const LSrc& src, int64_t n, double* L, int64_t ld, bool full, hipStream_t s,
                const LowRank& lr) {
  if (n <= 0) return;
  MM_REQUIRE(n < (int64_t)1 << 31, kInvalid, "assemble_L: n too large");
  MM_REQUIRE(src.L || (src.xyz && src.h > 0.0), kInvalid, "assemble_L: no inductance source");
  MM_REQUIRE(lr.m >= 0 && lr.m <= 8 && (lr.m == 0 || (lr.U && lr.Y1)), kInvalid,
             "assemble_L: bad low-rank term");
  hipLaunchKernelGGL(assemble_L_k, dim3((unsigned)n), dim3(256), 0, s, src, n, L, ld, (int)full,
                     lr);
  MM_HIP_TRY(hipGetLastError());
}

void flag_nonfinite(const double* p, int64_t count, int64_t* d_flag, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(flag_nonfinite_k, dim3(grid1(count)), dim3(256), 0, s, p, count, d_flag);
  MM_HIP_TRY(hipGetLastError());
}

void flag_nonfinite_lower(const double* A, int64_t lda, int64_t n, int64_t* d_flag,
                          hipStream_t s) {
  if (n <= 0) return;
  const unsigned g = (unsigned)std::min<int64_t>(n, 65536);
  hipLaunchKernelGGL(flag_nonfinite_lower_k, dim3(g), dim3(256), 0, s, A, lda, n, d_flag);
  MM_HIP_TRY(hipGetLastError());
}

void add_csr_lower(double* Z, int64_t ld, double alpha, const Csr& R, hipStream_t s) {
  if (R.rows <= 0) return;
  hipLaunchKernelGGL(add_csr_lower_k, dim3(grid1(R.rows)), dim3(256), 0, s, Z, ld, alpha, R);
  MM_HIP_TRY(hipGetLastError());
}

void csr_lower_band(const Csr& R, int64_t* d_out, hipStream_t s) {
  fill_i64(d_out, 1, 0, s);
  hipLaunchKernelGGL(csr_band_k, dim3(grid1(R.rows)), dim3(256), 0, s, R.rows, R.rowptr,
                     R.col, (unsigned long long*)d_out);
  MM_HIP_TRY(hipGetLastError());
}

void dense_times_csr(const double* A, int64_t lda, const Csr& R, double* W,
                     int64_t ldw, hipStream_t s) {
  const int64_t n = R.rows;
  if (n <= 0) return;
  hipLaunchKernelGGL(dense_times_csr_k, dim3((unsigned)n), dim3(256), 0, s, A, lda, R, n, W,
                     ldw);
  MM_HIP_TRY(hipGetLastError());
}

void symmetrize_from_lower(double* A, int64_t lda, int64_t n, hipStream_t s) {
  if (n <= 1) return;
  const int64_t nt = ceil_div(n, 32);
  hipLaunchKernelGGL(symmetrize_k, dim3((unsigned)nt, (unsigned)nt), dim3(32, 8), 0, s, A, lda, n);
  MM_HIP_TRY(hipGetLastError());
}

void fill(double* p, int64_t count, double v, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(fill_k, dim3(grid1(count)), dim3(256), 0, s, p, count, v);
  MM_HIP_TRY(hipGetLastError());
}

void fill_i64(int64_t* p, int64_t count, int64_t v, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(fill_i64_k, dim3(grid1(count)), dim3(256), 0, s, p, count, v);
  MM_HIP_TRY(hipGetLastError());
}

}  // namespace mm
