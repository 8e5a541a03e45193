// The classical theta-method (Sec. 3.3.1, eq. time_integration): per step
//   b = -dt Ri Ii + f^k;  C y = b;  C^T dI = y;  Ii += dI;  s = P dI / dt,
// with C the Cholesky factor of Z = Li + theta dt Ri.
//
// The two triangular solves read the factor once each (4 N^2 bytes per
// solve) and are HBM-bound.  They are blocked by B columns (B = 1024 at
// large N) and synchronised only by kernel boundaries (no workgroup ever
// waits on another):
//   forward,  for J = 0..NB-1:   y_J = D_J^{-1} b_J          (diag kernel)
//                                b_I -= C(I, J) y_J, I > J     (update kernel)
//   backward, for J = NB-1..0:   x_J = D_J^{-T} y_J          (diag kernel)
//                                y_I -= C(J, I)^T x_J, I < J   (update kernel)
// D_J^{-1} are the inverses of the diagonal blocks of C, formed once per
// factorisation and kept twice: column-major (backward: output c is a dot
// product with column c) and transposed (forward: output r is a dot product
// with row r), so every wave streams contiguous memory.  The update kernels
// keep 16-32 independent loads in flight per lane.  Every sum is taken in a
// fixed order, so reruns are bit-identical.  The state update Ii += dI and
// the probe partial sums are fused into the backward diagonal kernel.
//
// One step's launches read the step index from device memory, so the whole
// step is captured once into a HIP graph and replayed n_steps times.
#include "kernels.h"

namespace mm {
namespace {

constexpr int NT = 256;
constexpr int MAXB = 2048;
constexpr int BCOLS = 4;        // backward update: columns per wave

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

// b = -dt Ri I + F u^k   (k read from *kstep)
__global__ void chol_rhs_k(int64_t n0, Csr Ri, Forcing f, double theta, double dt,
                           const int64_t* kstep, const double* __restrict__ I,
                           double* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n0) return;
  const int64_t k = *kstep;
  double s = 0.0;
  for (int64_t p = Ri.rowptr[i + Ri.off]; p < Ri.rowptr[i + Ri.off + 1]; ++p) {
    const int64_t c = (int64_t)Ri.col[p] - Ri.off;
    if (c >= 0) s += Ri.val[p] * I[c];
  }
  double r = -dt * s;
  for (int j = 0; j < f.nf; ++j) r += f.F[i + (int64_t)j * n0] * forcing_u(f, j, k, theta, dt);
  b[i] = r;
}

// b += dt (V (Y^T I) + Y (V^T I)) on the rows idx: the low-rank part of
// -dt R_i I when R_i = R'' - V Y^T - Y V^T (one workgroup).
__global__ void __launch_bounds__(256) lowrank_rhs_k(RLowRank lr, double dt,
                                                     const double* __restrict__ I,
                                                     double* __restrict__ b) {
  constexpr int MAXM = 8;
  __shared__ double red[2 * MAXM][4];
  __shared__ double dv[2 * MAXM];  // [0, m): V^T I, [m, 2m): Y^T I
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int m = lr.m;
  double av[MAXM], ay[MAXM];
#pragma unroll
  for (int a = 0; a < MAXM; ++a) av[a] = ay[a] = 0.0;
  for (int j = t; j < lr.ns; j += 256) {
    const double x = I[lr.idx[j]];
#pragma unroll
    for (int a = 0; a < MAXM; ++a)
      if (a < m) {
        av[a] += lr.Vs[j + (int64_t)a * lr.ns] * x;
        ay[a] += lr.Ys[j + (int64_t)a * lr.ns] * x;
      }
  }
#pragma unroll
  for (int a = 0; a < MAXM; ++a)
    if (a < m) {
      const double v1 = wave_sum(av[a]), v2 = wave_sum(ay[a]);
      if (lane == 0) {
        red[a][wave] = v1;
        red[m + a][wave] = v2;
      }
    }
  __syncthreads();
  if (t < 2 * m) dv[t] = (red[t][0] + red[t][1]) + (red[t][2] + red[t][3]);
  __syncthreads();
  for (int j = t; j < lr.ns; j += 256) {
    double s = 0.0;
    for (int a = 0; a < m; ++a)
      s += lr.Vs[j + (int64_t)a * lr.ns] * dv[m + a] + lr.Ys[j + (int64_t)a * lr.ns] * dv[a];
    b[lr.idx[j]] += dt * s;
  }
}

__global__ void step_inc_k(int64_t* kstep) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *kstep += 1;
}

// Forward diagonal block: y_J(r) = sum_{c <= r} Dinv_J(r, c) b_J(c), one wave
// per output row, reading row r of Dinv_J contiguously from DinvT.
__global__ void __launch_bounds__(NT) fwd_diag_k(int64_t n, int B, int64_t J,
                                                 const double* __restrict__ DinvT,
                                                 const double* __restrict__ b,
                                                 double* __restrict__ y) {
  __shared__ double r[MAXB];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t J0 = J * B;
  const int jb = (int)min((int64_t)B, n - J0);
  for (int c = t; c < jb; c += NT) r[c] = b[J0 + c];
  __syncthreads();
  const int row = blockIdx.x * (NT / 64) + wave;
  if (row >= jb) return;
  const double* Dr = DinvT + J * (int64_t)B * B + (int64_t)row * B;
  double s = 0.0;
#pragma unroll 8
  for (int c = lane; c <= row; c += 64) s += Dr[c] * r[c];
  s = wave_sum(s);
  if (lane == 0) y[J0 + row] = s;
}

// Forward update: b_i -= sum_c C(i, J0 + c) y_J(c) for rows i >= J0 + B.
// Workgroup: 16 rows x B columns (four 128-byte row segments per wave load).
// Wave w owns columns [w B/4, (w+1) B/4); lane (r, g) = (lane % 16, lane / 16)
// reads row r of columns g, g+4, g+8, ... of that range.
__global__ void __launch_bounds__(NT) fwd_update_k(int64_t n, int B, int64_t J,
                                                   const double* __restrict__ C, int64_t ld,
                                                   const double* __restrict__ y,
                                                   double* __restrict__ b) {
  __shared__ double yj[MAXB];
  __shared__ double part[NT / 64][16];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int64_t J0 = J * B;
  for (int c = t; c < B; c += NT) yj[c] = y[J0 + c];  // J is not the last block
  __syncthreads();
  const int64_t row = J0 + B + (int64_t)blockIdx.x * 16 + r;
  const int cq = B / 4;
  double s = 0.0;
  if (row < n) {
    const double* Cp = C + row + (J0 + (int64_t)wave * cq + g) * ld;
    const double* yp = yj + wave * cq + g;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 16
    for (int c = 0; c < cq / 4; ++c) acc[c & 3] += Cp[(int64_t)(4 * c) * ld] * yp[4 * c];
    s = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  }
  // lanes r, r+16, r+32, r+48 hold the same row
  s += __shfl_xor(s, 16, 64);
  s += __shfl_xor(s, 32, 64);
  if (lane < 16) part[wave][lane] = s;
  __syncthreads();
  if (t < 16) {
    const int64_t rr = J0 + B + (int64_t)blockIdx.x * 16 + t;
    if (rr < n) b[rr] -= (part[0][t] + part[1][t]) + (part[2][t] + part[3][t]);
  }
}

// Backward diagonal block: x_J(c) = sum_{r >= c} Dinv_J(r, c) y_J(r), one wave
// per output (column c of Dinv_J, contiguous).  Fused: Ii += x_J and the probe
// partial sums of this workgroup's outputs.
__global__ void __launch_bounds__(NT) bwd_diag_k(int64_t n, int B, int64_t J,
                                                 const double* __restrict__ Dinv,
                                                 const double* __restrict__ y,
                                                 double* __restrict__ x, double* __restrict__ state,
                                                 const double* __restrict__ Pt, int n_probe,
                                                 double* __restrict__ pp_base,
                                                 const int64_t* kstep, int64_t parts) {
  __shared__ double r[MAXB];
  __shared__ double red[8][NT / 64];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t J0 = J * B;
  const int jb = (int)min((int64_t)B, n - J0);
  for (int c = t; c < jb; c += NT) r[c] = y[J0 + c];
  __syncthreads();
  const int c = blockIdx.x * (NT / 64) + wave;
  double out = 0.0;
  if (c < jb) {
    const double* Dc = Dinv + J * (int64_t)B * B + (int64_t)c * B;
    double s = 0.0;
#pragma unroll 8
    for (int rr = c + lane; rr < jb; rr += 64) s += Dc[rr] * r[rr];
    out = wave_sum(s);
    if (lane == 0) {
      x[J0 + c] = out;
      state[J0 + c] += out;
    }
  }
  // probe partials: one per (block J, workgroup), fixed order over the waves
  const int64_t k = *kstep;
  for (int p = 0; p < n_probe; ++p)
    if (lane == 0) red[p][wave] = (c < jb) ? Pt[(J0 + c) + (int64_t)p * n] * out : 0.0;
  __syncthreads();
  if (t < n_probe) {
    const int64_t part_idx = J * ((B + NT / 64 - 1) / (NT / 64)) + blockIdx.x;
    pp_base[(k * parts + part_idx) * n_probe + t] =
        (red[t][0] + red[t][1]) + (red[t][2] + red[t][3]);
  }
}

// Backward update: y_c -= sum_r C(J0 + r, c) x_J(r) for columns c < J0.
// Each wave handles BCOLS columns at once (contiguous segments of B rows).
__global__ void __launch_bounds__(NT) bwd_update_k(int64_t n, int B, int64_t J,
                                                   const double* __restrict__ C, int64_t ld,
                                                   const double* __restrict__ x,
                                                   double* __restrict__ y) {
  __shared__ double xj[MAXB];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t J0 = J * B;
  const int jb = (int)min((int64_t)B, n - J0);
  for (int c = t; c < jb; c += NT) xj[c] = x[J0 + c];
  __syncthreads();
  const int64_t col0 = ((int64_t)blockIdx.x * (NT / 64) + wave) * BCOLS;
  double s[BCOLS];
#pragma unroll
  for (int q = 0; q < BCOLS; ++q) s[q] = 0.0;
  // J > 0 here, so block J starts at J0 >= B and col0 + q < J0 <= n - jb:
  // every column pointer below stays inside the matrix.
  const double* Cc[BCOLS];
#pragma unroll
  for (int q = 0; q < BCOLS; ++q) Cc[q] = C + J0 + min(col0 + q, J0 - 1) * ld;
#pragma unroll 4
  for (int rr = lane; rr < jb; rr += 64) {
    const double xv = xj[rr];
#pragma unroll
    for (int q = 0; q < BCOLS; ++q) s[q] += Cc[q][rr] * xv;
  }
#pragma unroll
  for (int q = 0; q < BCOLS; ++q) {
    const double v = wave_sum(s[q]);
    if (lane == 0 && col0 + q < J0) y[col0 + q] -= v;
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

// One step's launch sequence (the step index is read from *kstep).
void enqueue_step(const CholStep& c, hipStream_t s) {
  const int64_t n = c.n0;
  const int B = c.B;
  const int64_t NB = ceil_div(n, B);
  const int64_t parts = trsv_parts(n);
  const unsigned rgrid = (unsigned)ceil_div(n, 256);
  const unsigned dgrid = (unsigned)ceil_div(B, NT / 64);
  hipLaunchKernelGGL(chol_rhs_k, dim3(rgrid), dim3(256), 0, s, n, c.Ri, c.f, c.theta, c.dt,
                     c.kstep, c.I, c.b);
  if (c.Rlr.ns > 0)
    hipLaunchKernelGGL(lowrank_rhs_k, dim3(1), dim3(256), 0, s, c.Rlr, c.dt, c.I, c.b);
  for (int64_t J = 0; J < NB; ++J) {
    hipLaunchKernelGGL(fwd_diag_k, dim3(dgrid), dim3(NT), 0, s, n, B, J, c.DinvT, c.b, c.y);
    const int64_t below = n - (J + 1) * B;
    if (below > 0)
      hipLaunchKernelGGL(fwd_update_k, dim3((unsigned)ceil_div(below, 16)), dim3(NT), 0, s, n, B,
                         J, c.Cf, c.ld, c.y, c.b);
  }
  for (int64_t J = NB - 1; J >= 0; --J) {
    hipLaunchKernelGGL(bwd_diag_k, dim3(dgrid), dim3(NT), 0, s, n, B, J, c.Dinv, c.y, c.b, c.I,
                       c.Pt, c.n_probe, c.probe_partial, c.kstep, parts);
    const int64_t J0 = J * B;
    if (J0 > 0)
      hipLaunchKernelGGL(bwd_update_k, dim3((unsigned)ceil_div(J0, (NT / 64) * BCOLS)), dim3(NT),
                         0, s, n, B, J, c.Cf, c.ld, c.b, c.y);
  }
  hipLaunchKernelGGL(step_inc_k, dim3(1), dim3(64), 0, s, c.kstep);
}

}  // namespace

int trsv_block(int64_t n) {
  return n >= 16384 ? 2048 : (n >= 8192 ? 1024 : (n >= 2048 ? 512 : 128));
}

int64_t trsv_parts(int64_t n) {
  const int B = trsv_block(n);
  return ceil_div(n, B) * ceil_div(B, NT / 64);
}

void chol_steps(const CholStep& c, int64_t k0, int64_t n_steps, hipStream_t s) {
  MM_REQUIRE(c.B >= 64 && c.B <= MAXB && c.B % 64 == 0, kInvalid, "chol_steps: block size");
  MM_REQUIRE(c.n_probe <= 8, kInvalid, "chol_steps: at most 8 probes");
  MM_REQUIRE(c.Rlr.ns == 0 || (c.Rlr.m >= 1 && c.Rlr.m <= 8), kInvalid,
             "chol_steps: low-rank resistance term of rank 1..8");
  if (n_steps <= 0) return;
  fill_i64(c.kstep, 1, k0, s);
  if (!c.use_graph || n_steps < 4) {
    for (int64_t k = 0; k < n_steps; ++k) enqueue_step(c, s);
    MM_HIP_TRY(hipGetLastError());
    return;
  }
  // Capture on a private non-blocking stream (the legacy default stream cannot
  // be captured), ordered after and before the caller's stream by events.
  hipStream_t cs = nullptr;
  hipEvent_t before = nullptr, after = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  MM_HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t e = hipEventCreateWithFlags(&before, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&after, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(before, s);
  if (e == hipSuccess) e = hipStreamWaitEvent(cs, before, 0);
  if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    enqueue_step(c, cs);
    e = hipStreamEndCapture(cs, &graph);
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  for (int64_t k = 0; e == hipSuccess && k < n_steps; ++k) e = hipGraphLaunch(exec, cs);
  if (e == hipSuccess) e = hipEventRecord(after, cs);
  if (e == hipSuccess) e = hipStreamWaitEvent(s, after, 0);
  hipError_t e2 = hipStreamSynchronize(cs);
  if (e == hipSuccess) e = e2;
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (before) (void)hipEventDestroy(before);
  if (after) (void)hipEventDestroy(after);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess)
    throw Error{kDevice, std::string("Cholesky step graph: ") + hipGetErrorString(e)};
}

namespace {
__global__ void transpose_blocks_k(const double* __restrict__ S, int B, double* __restrict__ D) {
  __shared__ double tile[32][33];
  const int64_t blk = blockIdx.z;
  const double* Sb = S + blk * (int64_t)B * B;
  double* Db = D + blk * (int64_t)B * B;
  const int bi = blockIdx.x * 32, bj = blockIdx.y * 32;
  const int tx = threadIdx.x, ty = threadIdx.y;
  for (int r = ty; r < 32; r += 8) tile[r][tx] = Sb[(bi + tx) + (int64_t)(bj + r) * B];
  __syncthreads();
  for (int r = ty; r < 32; r += 8) Db[(bj + tx) + (int64_t)(bi + r) * B] = tile[tx][r];
}
}  // namespace

void transpose_blocks(const double* Dinv, int64_t nblocks, int B, double* DinvT,
                      hipStream_t s) {
  MM_REQUIRE(B % 32 == 0, kInvalid, "transpose_blocks: B must be a multiple of 32");
  if (nblocks <= 0) return;
  hipLaunchKernelGGL(transpose_blocks_k, dim3(B / 32, B / 32, (unsigned)nblocks), dim3(32, 8), 0,
                     s, Dinv, B, DinvT);
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
