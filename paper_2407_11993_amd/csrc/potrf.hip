// Dense FP64 Cholesky (lower) and triangular inverse, column-major.
//
// potrf: blocked right-looking factorisation A = G G^T with NB = 128 column
// panels.  The 128 x 128 diagonal block is factored inside LDS by one
// workgroup (itself blocked by 16), which also writes the inverse of its
// factor; the panel below is
// then G21 = A21 G11^{-T} (a GEMM against that inverse) and the trailing
// matrix takes the symmetric rank-128 update A22 -= G21 G21^T on the matrix
// cores (lower triangle only).  Used for Li = G G^T (modal method) and for
// Z = Li + theta dt Ri = C C^T (Cholesky method).
//
// trtri: G^{-1} by recursive halving,
//   inv([A 0; B C]) = [A^{-1} 0; -C^{-1} B A^{-1}  C^{-1}],
// with the leaves (<= 128) inverted in LDS and the two products done by the
// GEMM with the triangular structure of the operands exploited per tile.
#include "common.h"
#include "kernels.h"

namespace mm {
namespace {

constexpr int DB = 128;        // diagonal block size
constexpr int LDL = DB + 1;    // LDS leading dimension

// Stage the jb x jb (jb <= 128) block Ab (leading dimension lda) into LDS,
// keeping the lower triangle when `lower` (zero above): thread t reads rows
// t % 128 of the columns t / 128 + 2m, 32 loads in flight per batch.
__device__ void stage_block(const double* Ab, int64_t lda, int jb, bool lower, double* L) {
  const int t = threadIdx.x, i = t & 127, jh = t >> 7;
  const int ic = min(i, jb - 1);
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    double r[32];
#pragma unroll
    for (int m = 0; m < 32; ++m) {
      const int j = min(jh + 2 * (32 * b + m), jb - 1);
      r[m] = Ab[ic + (int64_t)j * lda];
    }
#pragma unroll
    for (int m = 0; m < 32; ++m) {
      const int j = jh + 2 * (32 * b + m);
      if (i < jb && j < jb) L[i + j * LDL] = (!lower || i >= j) ? r[m] : 0.0;
    }
  }
}

// In-LDS factorisation of the jb x jb (jb <= 128) lower triangle L[i + j*LDL],
// blocked by 16 columns: the 16 x 16 diagonal piece is factored by the first
// wave (right-looking, lane = one row and four columns of the piece), the
// rows below it by one thread per row (forward substitution), and the
// trailing lower triangle takes the rank-16 update in parallel.  Needs
// blockDim.x == 256.  A non-positive pivot is recorded in *bad (local index)
// and replaced by 1 so the work finishes.
//
// The single-wave loops rely on one wave's LDS operations completing in
// program order: every lane's reads of a column are issued before any lane
// writes it, so no workgroup barrier is needed inside them.
__device__ void lds_potrf16(double* L, int jb, int* bad) {
  const int t = threadIdx.x;
  for (int k0 = 0; k0 < jb; k0 += 16) {
    const int ke = min(k0 + 16, jb);
    if (t < 64) {
      const int i = k0 + (t & 15), jq = k0 + (t >> 4);
      for (int k = k0; k < ke; ++k) {
        double d = L[k + k * LDL];
        if (!(d > 0.0)) {
          if (t == 0 && *bad < 0) *bad = k;
          d = 1.0;
        }
        d = sqrt(d);
        const double li = (i > k && i < ke) ? L[i + k * LDL] / d : 0.0;
        double lj[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int j = jq + 4 * q;
          lj[q] = (j > k && j < ke) ? L[j + k * LDL] / d : 0.0;
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int j = jq + 4 * q;
          if (j > k && i >= j && i < ke) L[i + j * LDL] -= li * lj[q];
        }
        if (t < 16 && i > k && i < ke) L[i + k * LDL] = li;
        if (t == 0) L[k + k * LDL] = d;
        __builtin_amdgcn_wave_barrier();
      }
    }
    __syncthreads();
    for (int i = ke + t; i < jb; i += 256) {
      for (int k = k0; k < ke; ++k) {
        double x = L[i + k * LDL];
        for (int c = k0; c < k; ++c) x -= L[i + c * LDL] * L[k + c * LDL];
        L[i + k * LDL] = x / L[k + k * LDL];
      }
    }
    __syncthreads();
    const int a = t & 15, bq = t >> 4;
    for (int j = ke + bq; j < jb; j += 16)
      for (int i = ke + a; i < jb; i += 16)
        if (i >= j) {
          double x = L[i + j * LDL];
#pragma unroll 4
          for (int c = k0; c < ke; ++c) x -= L[i + c * LDL] * L[j + c * LDL];
          L[i + j * LDL] = x;
        }
    __syncthreads();
  }
}

// In-LDS inverse of the jb x jb lower triangle, in place, by 16-wide block
// columns from the right:  X_jj = L_jj^{-1} (one thread, unblocked, rows
// processed bottom-up so every original entry is read before it is
// overwritten), then X(je:, j0:je) = -X(je:, je:) L(je:, j0:je) X_jj with the
// already inverted trailing part.  Needs blockDim.x == 256.
__device__ void lds_trtri16(double* L, int jb) {
  __shared__ double Yb[128 * 16];
  const int t = threadIdx.x;
  const int nblk = (jb + 15) / 16;
  for (int bj = nblk - 1; bj >= 0; --bj) {
    const int j0 = bj * 16, je = min(j0 + 16, jb), w = je - j0;
    // X_jj = L_jj^{-1} row by row (L X = I): lane c owns column c; row r
    // reads the original row r of L and the finished rows above it
    if (t < 64) {
      const int c = t;
      for (int r = 0; r < w; ++r) {
        const double xrr = 1.0 / L[(j0 + r) + (j0 + r) * LDL];
        double sacc = 0.0;
        if (c < r)
          for (int k = c; k < r; ++k) sacc += L[(j0 + r) + (j0 + k) * LDL] * L[(j0 + k) + (j0 + c) * LDL];
        __builtin_amdgcn_wave_barrier();
        if (c < r) L[(j0 + r) + (j0 + c) * LDL] = -sacc * xrr;
        if (c == r) L[(j0 + r) + (j0 + r) * LDL] = xrr;
        __builtin_amdgcn_wave_barrier();
      }
    }
    __syncthreads();
    const int R = jb - je;
    for (int e = t; e < R * w; e += 256) {
      const int i = e % R, c = e / R;
      double sacc = 0.0;
      for (int k = je; k <= je + i; ++k) sacc += L[(je + i) + k * LDL] * L[k + (j0 + c) * LDL];
      Yb[i + c * 128] = sacc;
    }
    __syncthreads();
    for (int e = t; e < R * w; e += 256) {
      const int i = e % R, c = e / R;
      double sacc = 0.0;
      for (int k = c; k < w; ++k) sacc += Yb[i + k * 128] * L[(j0 + k) + (j0 + c) * LDL];
      L[(je + i) + (j0 + c) * LDL] = -sacc;
    }
    __syncthreads();
  }
}

// Factor the diagonal block A[j0.., j0..] in place and write its inverse to
// Linv (jb x jb, ld jb).  status[0] keeps the first failing global pivot.
__global__ void __launch_bounds__(256) potrf_diag(double* A, int64_t lda,
                                                  int64_t j0, int jb,
                                                  double* Linv, int64_t* status) {
  __shared__ double L[DB * LDL];
  __shared__ int bad;
  const int t = threadIdx.x;
  if (t == 0) bad = -1;
  double* Ab = A + j0 + j0 * lda;
  stage_block(Ab, lda, jb, false, L);
  __syncthreads();
  lds_potrf16(L, jb, &bad);
  for (int e = t; e < jb * jb; e += blockDim.x) {
    const int i = e % jb, j = e / jb;
    Ab[i + (int64_t)j * lda] = (i >= j) ? L[i + j * LDL] : 0.0;
  }
  __syncthreads();
  lds_trtri16(L, jb);
  for (int e = t; e < jb * jb; e += blockDim.x) {
    const int i = e % jb, j = e / jb;
    Linv[i + (int64_t)j * jb] = (i >= j) ? L[i + j * LDL] : 0.0;
  }
  if (t == 0 && bad >= 0) {
    const unsigned long long g = (unsigned long long)(j0 + bad);
    atomicMin((unsigned long long*)status, g);
  }
}

// Invert the lower-triangular diagonal blocks of size <= DB in place.
// Block b covers [b*bs, min((b+1)*bs, n)).
__global__ void __launch_bounds__(256) trtri_diag(double* A, int64_t lda,
                                                  int64_t n, int bs) {
  __shared__ double L[DB * LDL];
  const int t = threadIdx.x;
  const int64_t j0 = (int64_t)blockIdx.x * bs;
  const int jb = (int)min((int64_t)bs, n - j0);
  double* Ab = A + j0 + j0 * lda;
  stage_block(Ab, lda, jb, true, L);
  __syncthreads();
  lds_trtri16(L, jb);
  for (int e = t; e < jb * jb; e += blockDim.x) {
    const int i = e % jb, j = e / jb;
    Ab[i + (int64_t)j * lda] = (i >= j) ? L[i + j * LDL] : 0.0;
  }
}

__global__ void zero_upper(double* A, int64_t lda, int64_t n) {
  const int64_t j = blockIdx.x;
  for (int64_t i = threadIdx.x; i < j; i += blockDim.x) A[i + j * lda] = 0.0;
}

__global__ void copy_block(const double* S, int64_t lds, double* D, int64_t ldd,
                           int64_t m, int64_t n) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * n) return;
  const int64_t i = idx % m, j = idx / m;
  D[i + j * ldd] = S[i + j * lds];
}

void trtri_rec(double* A, int64_t lda, int64_t n, double* ws, hipStream_t s) {
  // leaves are inverted beforehand by trtri_diag with block size DB; here only
  // the off-diagonal blocks of the recursion are formed.
  if (n <= DB) return;
  // split on a multiple of DB so that leaves line up with trtri_diag blocks
  int64_t n1 = ceil_div(ceil_div(n, 2), DB) * DB;
  if (n1 >= n) n1 = ((n - 1) / DB) * DB;
  const int64_t n2 = n - n1;
  trtri_rec(A, lda, n1, ws, s);
  trtri_rec(A + n1 + n1 * lda, lda, n2, ws, s);
  // T = B A11^{-1}   (n2 x n1); A11^{-1} lower: op(B)(k,j) = 0 for k < j
  Gemm g1;
  g1.m = n2; g1.n = n1; g1.k = n1;
  g1.A = A + n1; g1.lda = lda;
  g1.B = A; g1.ldb = lda;
  g1.C = ws; g1.ldc = n2;
  g1.b_lower = true;
  gemm(g1, s);
  // B <- -C^{-1} T  (C^{-1} = A22^{-1} lower: op(A)(i,k) = 0 for k > i)
  Gemm g2;
  g2.m = n2; g2.n = n1; g2.k = n2;
  g2.alpha = -1.0;
  g2.A = A + n1 + n1 * lda; g2.lda = lda;
  g2.a_lower = true;
  g2.B = ws; g2.ldb = n2;
  g2.C = A + n1; g2.ldc = lda;
  gemm(g2, s);
}

}  // namespace

namespace {

constexpr int GB = 4;  // diagonal blocks per group

// Diagonal block [j0, j0 + jb) factored (with its inverse in Linv), then the
// block column below it, A21 <- A21 G11^{-T}, of m rows (also left in T, ld ldt).
void factor_block(double* A, int64_t lda, int64_t j0, int jb, int64_t m, double* Linv,
                  double* T, int64_t ldt, int64_t* d_status, hipStream_t s) {
  hipLaunchKernelGGL(potrf_diag, dim3(1), dim3(256), 0, s, A, lda, j0, jb, Linv, d_status);
  MM_HIP_TRY(hipGetLastError());
  if (m <= 0) return;
  // T = A21 G11^{-T}: op(B) = Linv^T, op(B)(k,j) = Linv(j,k) = 0 for k > j
  Gemm g;
  g.m = m; g.n = jb; g.k = jb;
  g.A = A + (j0 + jb) + j0 * lda; g.lda = lda;
  g.B = Linv; g.ldb = jb; g.tb = true; g.b_band = 0;
  g.C = T; g.ldc = ldt;
  gemm(g, s);
  const int64_t tot = m * jb;
  hipLaunchKernelGGL(copy_block, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, s,
                     T, ldt, A + (j0 + jb) + j0 * lda, lda, m, (int64_t)jb);
  MM_HIP_TRY(hipGetLastError());
}

int64_t ld16(int64_t m) { return ceil_div(m, 16) * 16; }

}  // namespace

// Right-looking blocked Cholesky in groups of up to GB diagonal blocks: block
// t of a group first receives the updates of the group's earlier blocks on
// its own columns, is factored, and leaves its scaled block column T_t in U;
// the trailing matrix below the group then receives all of them as one
// update A -= U U^T (k = 128 t, instead of t passes with k = 128).  U's rows
// are those below the group's first block; T_t is stored from its own first
// row on, and every product reads it only there.
void potrf_lower(double* A, int64_t lda, int64_t n, double* ws,
                 int64_t ws_elems, int64_t* d_status, hipStream_t s) {
  MM_REQUIRE(ws_elems >= potrf_ws_elems(n), kInvalid, "potrf: workspace too small");
  double* Linv = ws;                  // DB x DB
  double* U = ws + (int64_t)DB * DB;  // ldu x GB DB
  for (int64_t j0 = 0; j0 < n;) {
    const int64_t r1 = j0 + DB;       // U's first row
    const int64_t ldu = ld16(std::max<int64_t>(1, n - r1));
    // full blocks join the group while rows remain below them
    int q = 1;
    while (q < GB && j0 + (q + 1) * (int64_t)DB < n) ++q;
    if (n - j0 <= DB) q = 1;
    int64_t jnext = j0;
    for (int t = 1; t <= q; ++t) {
      const int64_t jt = j0 + (t - 1) * (int64_t)DB;
      const int jb = (int)std::min<int64_t>(DB, n - jt);
      const int64_t mt = n - jt - jb;
      if (t > 1) {
        // block t's columns, rows [jt, n), get the group's earlier blocks
        Gemm u;
        u.m = n - jt; u.n = jb; u.k = (int64_t)(t - 1) * DB;
        u.alpha = -1.0; u.beta = 1.0;
        u.A = U + (jt - r1); u.lda = ldu;
        u.B = U + (jt - r1); u.ldb = ldu; u.tb = true;  // its first jb rows
        u.C = A + jt + jt * lda; u.ldc = lda;
        gemm(u, s);
      }
      factor_block(A, lda, jt, jb, mt, Linv, U + (t - 1) * (int64_t)DB * ldu + (jt + jb - r1),
                   ldu, d_status, s);
      jnext = jt + jb;
    }
    const int64_t mq = n - jnext;
    if (mq > 0) {
      // A[jnext:, jnext:] -= U U^T (lower), U's rows from jnext
      Gemm u;
      u.m = mq; u.n = mq; u.k = (int64_t)q * DB;
      u.alpha = -1.0; u.beta = 1.0;
      u.A = U + (jnext - r1); u.lda = ldu;
      u.B = U + (jnext - r1); u.ldb = ldu; u.tb = true;
      u.C = A + jnext + jnext * lda; u.ldc = lda;
      u.lower = true;
      gemm(u, s);
    }
    j0 = jnext;
  }
  hipLaunchKernelGGL(zero_upper, dim3((unsigned)n), dim3(256), 0, s, A, lda, n);
  MM_HIP_TRY(hipGetLastError());
}

int64_t potrf_ws_elems(int64_t n) { return (int64_t)DB * DB + ld16(n) * GB * DB; }

void trtri_lower(double* A, int64_t lda, int64_t n, double* ws, int64_t ws_elems,
                 hipStream_t s) {
  MM_REQUIRE(ws_elems >= trtri_ws_elems(n), kInvalid, "trtri: workspace too small");
  const int64_t nblk = ceil_div(n, DB);
  hipLaunchKernelGGL(trtri_diag, dim3((unsigned)nblk), dim3(256), 0, s, A, lda, n, DB);
  MM_HIP_TRY(hipGetLastError());
  trtri_rec(A, lda, n, ws, s);
}

int64_t trtri_ws_elems(int64_t n) {
  const int64_t h = ceil_div(n, 2) + DB;
  return h * h;
}

void diag_block_inverses(const double* A, int64_t lda, int64_t n, int nb, double* Dinv,
                         double* ws, int64_t ws_elems, hipStream_t s) {
  MM_REQUIRE(nb >= 1, kInvalid, "diag_block_inverses: block size");
  if (n <= 0) return;
  const int64_t NB = ceil_div(n, nb);
  fill(Dinv, NB * nb * nb, 0.0, s);
  for (int64_t J = 0; J < NB; ++J) {
    const int64_t j0 = J * nb, jb = std::min<int64_t>(nb, n - j0);
    double* D = Dinv + J * nb * nb;
    copy_matrix(A + j0 + j0 * lda, lda, D, nb, jb, jb, s);
    trtri_lower(D, nb, jb, ws, ws_elems, s);
  }
}

void copy_matrix(const double* S, int64_t lds, double* D, int64_t ldd,
                 int64_t m, int64_t n, hipStream_t s) {
  if (m <= 0 || n <= 0) return;
  const int64_t tot = m * n;
  hipLaunchKernelGGL(copy_block, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, s,
                     S, lds, D, ldd, m, n);
  MM_HIP_TRY(hipGetLastError());
}

}  // namespace mm
