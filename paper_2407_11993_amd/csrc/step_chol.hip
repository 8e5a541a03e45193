// The classical theta-method (Sec. 3.3.1, eq. time_integration): per step
//   b = -dt Ri Ii + f^k;  C y = b;  C^T dI = y;  Ii += dI;  s = P dI / dt,
// with C the Cholesky factor of Z = Li + theta dt Ri.
//
// The two triangular solves read the factor once each (4 N^2 bytes per
// solve) and are HBM-bound.  They are blocked by NBLK = 512 columns and
// synchronised only by kernel boundaries (no workgroup ever waits on
// another):
//   forward,  for J = 0..NB-1:   y_J = D_J^{-1} b_J          (diag kernel)
//                                b_I -= C(I, J) y_J, I > J     (update kernel)
//   backward, for J = NB-1..0:   x_J = D_J^{-T} y_J          (diag kernel)
//                                y_I -= C(J, I)^T x_J, I < J   (update kernel)
// where D_J^{-1} are the inverses of the diagonal blocks of C, formed once
// per factorisation.  Both products are written so that each wave reads
// contiguous column segments of the column-major factor, and every sum is
// taken in a fixed order, so reruns are bit-identical.  The state update
// Ii += dI and the probe partial sums are fused into the backward diagonal
// kernel.
#include "kernels.h"

namespace mm {
namespace {

constexpr int NT = 256;
constexpr int ROWS_DIAG = 64;   // rows (fwd) / columns (bwd) per workgroup, diag kernels
constexpr int ROWS_UPD = 64;    // rows per workgroup, forward update
constexpr int COLS_UPD = 16;    // columns per workgroup, backward update

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double forcing_u(const Forcing& f, int j, int64_t k,
                                            double theta, double dt) {
  if (j < f.m) {
    const double a = f.i_D[k * f.m + j], b = f.i_D[(k + 1) * f.m + j];
    return -dt * (a + theta * (b - a));
  }
  if (j < 2 * f.m) {
    const int a = j - f.m;
    return -(f.i_D[(k + 1) * f.m + a] - f.i_D[k * f.m + a]);
  }
  const int c = j - 2 * f.m;
  return -(f.i_src[(k + 1) * f.n_src + c] - f.i_src[k * f.n_src + c]);
}

// b = -dt Ri I + F u^k
__global__ void chol_rhs_k(int64_t n0, Csr Ri, Forcing f, double theta, double dt,
                           int64_t k, const double* __restrict__ I, double* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n0) return;
  double s = 0.0;
  for (int64_t p = Ri.rowptr[i]; p < Ri.rowptr[i + 1]; ++p) s += Ri.val[p] * I[Ri.col[p]];
  double r = -dt * s;
  for (int j = 0; j < f.nf; ++j) r += f.F[i + (int64_t)j * n0] * forcing_u(f, j, k, theta, dt);
  b[i] = r;
}

// Forward diagonal block: y_J = D_J^{-1} b_J.  Workgroup w owns rows
// [w*64, w*64+64) of the block; wave q sums columns [q*B/4, (q+1)*B/4).
// Output to yout (the block's solution, separate from b so that the update
// kernel reads a consistent y_J).
__global__ void __launch_bounds__(NT) fwd_diag_k(int64_t n, int B, int64_t J,
                                                 const double* __restrict__ Dinv,
                                                 const double* __restrict__ b,
                                                 double* __restrict__ y) {
  __shared__ double r[512];
  __shared__ double part[4][ROWS_DIAG];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t J0 = J * B;
  const int jb = (int)min((int64_t)B, n - J0);
  for (int c = t; c < B; c += NT) r[c] = (c < jb) ? b[J0 + c] : 0.0;
  __syncthreads();
  const int row = blockIdx.x * ROWS_DIAG + lane;
  const double* D = Dinv + J * (int64_t)B * B;
  const int cq = B / 4;
  double s = 0.0;
  if (row < jb) {
    const int c0 = wave * cq;
    const int c1 = min(c0 + cq, row + 1);  // D_J^{-1} is lower triangular
    for (int c = c0; c < c1; ++c) s += D[row + (int64_t)c * B] * r[c];
  }
  part[wave][lane] = s;
  __syncthreads();
  if (t < ROWS_DIAG && blockIdx.x * ROWS_DIAG + t < jb) {
    const int rr = blockIdx.x * ROWS_DIAG + t;
    y[J0 + rr] = (part[0][t] + part[1][t]) + (part[2][t] + part[3][t]);
  }
}

// Forward update: b_I -= C(I, J) y_J for rows i in [J0 + B, n).  Workgroup
// owns 64 rows; wave q sums columns [q*B/4, (q+1)*B/4) of the block.
__global__ void __launch_bounds__(NT) fwd_update_k(int64_t n, int B, int64_t J,
                                                   const double* __restrict__ C, int64_t ld,
                                                   const double* __restrict__ y,
                                                   double* __restrict__ b) {
  __shared__ double yj[512];
  __shared__ double part[4][ROWS_UPD];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t J0 = J * B;
  for (int c = t; c < B; c += NT) yj[c] = y[J0 + c];  // J is not the last block
  __syncthreads();
  const int64_t row = J0 + B + (int64_t)blockIdx.x * ROWS_UPD + lane;
  const int cq = B / 4;
  double s = 0.0;
  if (row < n) {
    const double* Cp = C + row + (J0 + (int64_t)wave * cq) * ld;
    const double* yp = yj + wave * cq;
#pragma unroll 8
    for (int c = 0; c < cq; ++c) s += Cp[(int64_t)c * ld] * yp[c];
  }
  part[wave][lane] = s;
  __syncthreads();
  if (t < ROWS_UPD) {
    const int64_t rr = J0 + B + (int64_t)blockIdx.x * ROWS_UPD + t;
    if (rr < n) b[rr] -= (part[0][t] + part[1][t]) + (part[2][t] + part[3][t]);
  }
}

// Backward diagonal block: x_J = D_J^{-T} y_J; fused state update and probe
// partials.  Workgroup w owns outputs [w*64, w*64+64); output c is the dot
// product of column c of D_J^{-1} (rows c..jb-1) with y_J: one wave per
// output, 16 outputs per wave.
__global__ void __launch_bounds__(NT) bwd_diag_k(int64_t n, int B, int64_t J,
                                                 const double* __restrict__ Dinv,
                                                 const double* __restrict__ y,
                                                 double* __restrict__ x, double* __restrict__ state,
                                                 const double* __restrict__ Pt, int n_probe,
                                                 double* __restrict__ pp) {
  __shared__ double r[512];
  __shared__ double out[ROWS_DIAG];
  __shared__ double red[4];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t J0 = J * B;
  const int jb = (int)min((int64_t)B, n - J0);
  for (int c = t; c < B; c += NT) r[c] = (c < jb) ? y[J0 + c] : 0.0;
  __syncthreads();
  const double* D = Dinv + J * (int64_t)B * B;
  for (int q = 0; q < ROWS_DIAG / 4; ++q) {
    const int oc = wave * (ROWS_DIAG / 4) + q;   // output within this workgroup
    const int c = blockIdx.x * ROWS_DIAG + oc;   // output within the block
    double s = 0.0;
    if (c < jb)
      for (int rr = c + lane; rr < jb; rr += 64) s += D[rr + (int64_t)c * B] * r[rr];
    s = wave_sum(s);
    if (lane == 0) out[oc] = s;
  }
  __syncthreads();
  const int c = blockIdx.x * ROWS_DIAG + (t & 63);
  const bool mine = t < ROWS_DIAG && c < jb;
  if (mine) {
    x[J0 + c] = out[t];
    state[J0 + c] += out[t];
  }
  for (int p = 0; p < n_probe; ++p) {
    double v = mine ? Pt[(J0 + c) + (int64_t)p * n] * out[t] : 0.0;
    v = wave_sum(v);
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (t == 0) pp[blockIdx.x * n_probe + p] = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
  }
}

// Backward update: y_c -= C(J0.., c)^T x_J for columns c < J0.  Each wave
// handles COLS_UPD / 4 columns; a column's block segment is contiguous.
__global__ void __launch_bounds__(NT) bwd_update_k(int64_t n, int B, int64_t J,
                                                   const double* __restrict__ C, int64_t ld,
                                                   const double* __restrict__ x,
                                                   double* __restrict__ y) {
  __shared__ double xj[512];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t J0 = J * B;
  const int jb = (int)min((int64_t)B, n - J0);
  for (int c = t; c < B; c += NT) xj[c] = (c < jb) ? x[J0 + c] : 0.0;
  __syncthreads();
  for (int q = 0; q < COLS_UPD / 4; ++q) {
    const int64_t col = (int64_t)blockIdx.x * COLS_UPD + wave * (COLS_UPD / 4) + q;
    if (col >= J0) break;
    const double* Cc = C + J0 + col * ld;
    double s = 0.0;
    for (int rr = lane; rr < jb; rr += 64) s += Cc[rr] * xj[rr];
    s = wave_sum(s);
    if (lane == 0) y[col] -= s;
  }
}

__global__ void probe_finish_k(const double* pp, int64_t n_steps, int64_t nparts,
                               int n_probe, const double* Pd, int m, const double* i_D,
                               double dt, double* signal) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_steps * n_probe) return;
  const int64_t k = e / n_probe;
  const int p = (int)(e % n_probe);
  const double* q = pp + k * nparts * n_probe + p;
  double s = 0.0;
  for (int64_t j = 0; j < nparts; ++j) s += q[j * n_probe];
  for (int a = 0; a < m; ++a)
    s += Pd[p + (int64_t)a * n_probe] * (i_D[(k + 1) * m + a] - i_D[k * m + a]);
  signal[e] = s / dt;
}

}  // namespace

int trsv_block(int64_t n) { return n >= 4096 ? 512 : (n >= 1024 ? 256 : 128); }

int64_t trsv_parts(int64_t n) {
  const int B = trsv_block(n);
  return ceil_div(n, B) * (B / ROWS_DIAG);
}

void chol_steps(const CholStep& c, int64_t k0, int64_t n_steps, hipStream_t s) {
  const int64_t n = c.n0;
  const int B = c.B;
  MM_REQUIRE(B == 128 || B == 256 || B == 512, kInvalid, "chol_steps: block size");
  const int64_t NB = ceil_div(n, B);
  const int per_blk = B / ROWS_DIAG;
  const unsigned rgrid = (unsigned)ceil_div(n, 256);
  for (int64_t k = k0; k < k0 + n_steps; ++k) {
    double* pp = c.probe_partial + (k - k0) * NB * per_blk * c.n_probe;
    hipLaunchKernelGGL(chol_rhs_k, dim3(rgrid), dim3(256), 0, s, n, c.Ri, c.f, c.theta, c.dt, k,
                       c.I, c.b);
    for (int64_t J = 0; J < NB; ++J) {
      hipLaunchKernelGGL(fwd_diag_k, dim3(per_blk), dim3(NT), 0, s, n, B, J, c.Dinv, c.b, c.y);
      const int64_t below = n - (J + 1) * B;
      if (below > 0)
        hipLaunchKernelGGL(fwd_update_k, dim3((unsigned)ceil_div(below, ROWS_UPD)), dim3(NT), 0,
                           s, n, B, J, c.Cf, c.ld, c.y, c.b);
    }
    // backward: y (in c.y) -> x (in c.b)
    for (int64_t J = NB - 1; J >= 0; --J) {
      hipLaunchKernelGGL(bwd_diag_k, dim3(per_blk), dim3(NT), 0, s, n, B, J, c.Dinv, c.y, c.b,
                         c.I, c.Pt, c.n_probe, pp + J * per_blk * c.n_probe);
      const int64_t J0 = J * B;
      if (J0 > 0)
        hipLaunchKernelGGL(bwd_update_k, dim3((unsigned)ceil_div(J0, COLS_UPD)), dim3(NT), 0, s,
                           n, B, J, c.Cf, c.ld, c.b, c.y);
    }
  }
  MM_HIP_TRY(hipGetLastError());
}

void probe_finish(const double* probe_partial, int64_t n_steps, int64_t nparts,
                  int n_probe, const double* Pd, int m, const double* i_D, int64_t k0,
                  double dt, double* signal, hipStream_t s) {
  (void)k0;
  const int64_t tot = n_steps * n_probe;
  if (tot <= 0) return;
  hipLaunchKernelGGL(probe_finish_k, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, s,
                     probe_partial, n_steps, nparts, n_probe, Pd, m, i_D, dt, signal);
  MM_HIP_TRY(hipGetLastError());
}

}  // namespace mm
