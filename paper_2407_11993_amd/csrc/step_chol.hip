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
constexpr int MAXB = 4096;
constexpr int BCOLS = 4;        // backward update: columns per wave

// Workgroups of a diagonal-block kernel: four waves, two rows or columns each.
__host__ __device__ inline int diag_groups(int B) { return (B / 2 + NT / 64 - 1) / (NT / 64); }

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

// Diagonal blocks.  Rows (forward) or columns (backward) p and jb-1-p of the
// triangular block inverse are folded onto one wave: together they hold
// jb + 1 entries, so every wave does the same work and issues all of its
// loads at once (clamped addresses, masked values).  KC load slots per lane:
// the two rows of a forward pair span at most B / 64 + 1 chunks of 64, the
// two columns of a backward pair at most B / 64 + 2 (their first chunks need
// not be aligned).  The right-hand side of the block is staged in LDS once
// per workgroup.
// Forward: y_J(r) = sum_{c <= r} Dinv_J(r, c) b_J(c), row r of Dinv_J read
// contiguously from DinvT.
template <int KC>
__global__ void __launch_bounds__(NT) fwd_diag_k(int64_t n, int B, int64_t J,
                                                 const double* __restrict__ DinvT,
                                                 const double* __restrict__ b,
                                                 double* __restrict__ y) {
  __shared__ double bs[MAXB];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t J0 = J * B;
  const int jb = (int)min((int64_t)B, n - J0);
  // a wave past the last pair computes pair 0 again and discards it, so the
  // barrier below is reached by every thread
  const int pw = blockIdx.x * (NT / 64) + wave;
  const bool live = pw < (jb + 1) / 2;
  const int p = live ? pw : 0;
  const int r1 = p, r2 = jb - 1 - p;
  const int n1 = r1 / 64 + 1, n2 = (r2 > r1) ? r2 / 64 + 1 : 0;
  const double* D1 = DinvT + J * (int64_t)B * B + (int64_t)r1 * B;
  const double* D2 = DinvT + J * (int64_t)B * B + (int64_t)r2 * B;
  double dv[KC];
#pragma unroll
  for (int v = 0; v < KC; ++v) {
    const bool sec = v >= n1;
    dv[v] = (sec ? D2 : D1)[min(64 * (sec ? v - n1 : v) + lane, sec ? r2 : r1)];
  }
  // the block's right-hand side, staged while the loads above are in flight
  for (int c = t; c < jb; c += NT) bs[c] = b[J0 + c];
  __syncthreads();
  double s1 = 0.0, s2 = 0.0;
#pragma unroll
  for (int v = 0; v < KC; ++v) {
    const bool sec = v >= n1;
    const int rr = sec ? r2 : r1;
    const int c = 64 * (sec ? v - n1 : v) + lane;
    const bool ok = v < n1 + n2 && c <= rr;
    const double val = ok ? dv[v] * bs[min(c, rr)] : 0.0;
    if (sec) s2 += val;
    else s1 += val;
  }
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  if (live && lane == 0) {
    y[J0 + r1] = s1;
    if (r2 > r1) y[J0 + r2] = s2;
  }
}

// Forward panel update  b_i -= sum_c C(i, J0 + c) y_J(c)  for the rows
// i >= J0 + B.  Workgroup: a tile of 64 rows (one per lane, so every wave
// load is one contiguous 512-byte column segment) times all B columns of the
// panel, which its UW waves take in turn, UL columns at a time: each wave
// keeps UL loads in flight.  The waves' row sums are combined in LDS in wave
// order (deterministic, no atomics).
constexpr int UW = 16;  // waves per forward-update workgroup
constexpr int UL = 16;  // column loads in flight per wave
__global__ void __launch_bounds__(64 * UW) fwd_update_k(int64_t n, int B, int64_t J,
                                                        const double* __restrict__ C, int64_t ld,
                                                        const double* __restrict__ y,
                                                        double* __restrict__ b) {
  __shared__ double red[UW][64];
  const int t = threadIdx.x, lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);  // wave-uniform: y via scalar loads
  const int64_t J0 = J * B;
  const int64_t row = J0 + B + (int64_t)blockIdx.x * 64 + lane;
  const double* Cp = C + min(row, n - 1) + J0 * ld;  // clamped: rows past n are not stored
  const double* yp = y + J0;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  // B is a multiple of UW * UL = 256 columns
  for (int q0 = wave * UL; q0 < B; q0 += UW * UL) {
    double cv[UL];
#pragma unroll
    for (int u = 0; u < UL; ++u) cv[u] = Cp[(int64_t)(q0 + u) * ld];
    __builtin_amdgcn_sched_barrier(0);  // all UL loads issue before the first use
#pragma unroll
    for (int u = 0; u < UL; ++u) acc[u & 3] += cv[u] * yp[q0 + u];
  }
  red[wave][lane] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  __syncthreads();
  if (wave != 0) return;
  double v = 0.0;
#pragma unroll
  for (int w = 0; w < UW; ++w) v += red[w][lane];
  if (row < n) b[row] -= v;
}

// Backward: x_J(c) = sum_{r >= c} Dinv_J(r, c) y_J(r), column c of Dinv_J
// read contiguously.  Fused: Ii += x_J and the probe partial sums of this
// workgroup's outputs (one per workgroup and probe, fixed order).
template <int KC>
__global__ void __launch_bounds__(NT) bwd_diag_k(int64_t n, int B, int64_t J,
                                                 const double* __restrict__ Dinv,
                                                 const double* __restrict__ y,
                                                 double* __restrict__ x, double* __restrict__ state,
                                                 const double* __restrict__ Pt, int n_probe,
                                                 double* __restrict__ pp_base,
                                                 const int64_t* kstep, int64_t parts) {
  __shared__ double ys[MAXB];
  __shared__ double red[8][NT / 64];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t J0 = J * B;
  const int jb = (int)min((int64_t)B, n - J0);
  // a wave past the last pair computes pair 0 again and discards it, so the
  // barrier below is reached by every thread
  const int pw = blockIdx.x * (NT / 64) + wave;
  const bool live = pw < (jb + 1) / 2;
  const int p = live ? pw : 0;
  const int c1 = p, c2 = jb - 1 - p;
  double o1 = 0.0, o2 = 0.0;
  {
    const int last = (jb - 1) / 64;  // chunk of the block's last row
    const int f1 = c1 / 64, f2 = c2 / 64;
    const int n1 = last - f1 + 1, n2 = (c2 > c1) ? last - f2 + 1 : 0;
    const double* D1 = Dinv + J * (int64_t)B * B + (int64_t)c1 * B;
    const double* D2 = Dinv + J * (int64_t)B * B + (int64_t)c2 * B;
    double dv[KC];
#pragma unroll
    for (int v = 0; v < KC; ++v) {
      const bool sec = v >= n1;
      const int r = 64 * (sec ? f2 + (v - n1) : f1 + v) + lane;
      dv[v] = (sec ? D2 : D1)[min(max(r, sec ? c2 : c1), jb - 1)];
    }
    // the block's right-hand side, staged while the loads above are in flight
    for (int c = t; c < jb; c += NT) ys[c] = y[J0 + c];
    __syncthreads();
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int v = 0; v < KC; ++v) {
      const bool sec = v >= n1;
      const int cc0 = sec ? c2 : c1;
      const int r = 64 * (sec ? f2 + (v - n1) : f1 + v) + lane;
      const bool ok = v < n1 + n2 && r >= cc0 && r < jb;
      const double val = ok ? dv[v] * ys[min(max(r, cc0), jb - 1)] : 0.0;
      if (sec) s2 += val;
      else s1 += val;
    }
    o1 = live ? wave_sum(s1) : 0.0;
    o2 = live ? wave_sum(s2) : 0.0;
    if (live && lane == 0) {
      x[J0 + c1] = o1;
      state[J0 + c1] += o1;
      if (c2 > c1) {
        x[J0 + c2] = o2;
        state[J0 + c2] += o2;
      }
    }
  }
  const int64_t k = *kstep;
  for (int q = 0; q < n_probe; ++q)
    if (lane == 0) {
      double v = 0.0;
      if (live) {
        v = Pt[(J0 + c1) + (int64_t)q * n] * o1;
        if (c2 > c1) v += Pt[(J0 + c2) + (int64_t)q * n] * o2;
      }
      red[q][wave] = v;
    }
  __syncthreads();
  if (t < n_probe) {
    const int64_t part_idx = J * diag_groups(B) + blockIdx.x;
    pp_base[(k * parts + part_idx) * n_probe + t] =
        (red[t][0] + red[t][1]) + (red[t][2] + red[t][3]);
  }
}

// Backward update  y_c -= sum_r C(J0 + r, c) x_J(r)  for the columns c < J0.
// Each wave owns BCOLS columns over all of block J's rows; lanes walk the
// rows, so every load is a contiguous 512-byte column segment, and RB row
// chunks of all BCOLS columns are loaded before any is used (BCOLS * RB
// loads in flight per wave).
constexpr int RB = 4;
__global__ void __launch_bounds__(NT) bwd_update_k(int64_t n, int B, int64_t J,
                                                   const double* __restrict__ C, int64_t ld,
                                                   const double* __restrict__ x,
                                                   double* __restrict__ y) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t J0 = J * B;
  const int jb = (int)min((int64_t)B, n - J0);
  const int64_t col0 = ((int64_t)blockIdx.x * (NT / 64) + wave) * BCOLS;
  double s[BCOLS];
#pragma unroll
  for (int q = 0; q < BCOLS; ++q) s[q] = 0.0;
  // J > 0 here, so block J starts at J0 >= B and col0 + q < J0 <= n - jb:
  // every (clamped) column pointer below stays inside the matrix.
  const double* Cc[BCOLS];
#pragma unroll
  for (int q = 0; q < BCOLS; ++q) Cc[q] = C + J0 + min(col0 + q, J0 - 1) * ld;
  const double* xj = x + J0;
  int rr = lane;
  for (; rr + 64 * (RB - 1) < jb; rr += 64 * RB) {
    double cv[RB][BCOLS], xv[RB];
#pragma unroll
    for (int u = 0; u < RB; ++u) {
      xv[u] = xj[rr + 64 * u];
#pragma unroll
      for (int q = 0; q < BCOLS; ++q) cv[u][q] = Cc[q][rr + 64 * u];
    }
#pragma unroll
    for (int u = 0; u < RB; ++u)
#pragma unroll
      for (int q = 0; q < BCOLS; ++q) s[q] += cv[u][q] * xv[u];
  }
  for (; rr < jb; rr += 64) {
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

template <int C64>  // C64 = B / 64
void launch_diag_b(bool fwd, unsigned grid, hipStream_t s, int64_t n, int64_t J,
                   const CholStep& c) {
  if (fwd)
    hipLaunchKernelGGL((fwd_diag_k<C64 + 1>), dim3(grid), dim3(NT), 0, s, n, c.B, J, c.DinvT,
                       c.b, c.y);
  else
    hipLaunchKernelGGL((bwd_diag_k<C64 + 2>), dim3(grid), dim3(NT), 0, s, n, c.B, J, c.Dinv,
                       c.y, c.b, c.I, c.Pt, c.n_probe, c.probe_partial, c.kstep, trsv_parts(n));
}
void launch_diag(bool fwd, int B, unsigned grid, hipStream_t s, int64_t n, int64_t J,
                 const CholStep& c) {
  switch (B) {
    case 256: launch_diag_b<4>(fwd, grid, s, n, J, c); break;
    case 512: launch_diag_b<8>(fwd, grid, s, n, J, c); break;
    case 1024: launch_diag_b<16>(fwd, grid, s, n, J, c); break;
    case 2048: launch_diag_b<32>(fwd, grid, s, n, J, c); break;
    case 4096: launch_diag_b<64>(fwd, grid, s, n, J, c); break;
    default: throw Error{kInvalid, "triangular solve: unsupported block size"};
  }
}

// One step's launch sequence (the step index is read from *kstep).
void enqueue_step(const CholStep& c, hipStream_t s) {
  const int64_t n = c.n0;
  const int B = c.B;
  const int64_t NB = ceil_div(n, B);
  const int64_t parts = trsv_parts(n);
  const unsigned rgrid = (unsigned)ceil_div(n, 256);
  const unsigned dgrid = (unsigned)diag_groups(B);
  hipLaunchKernelGGL(chol_rhs_k, dim3(rgrid), dim3(256), 0, s, n, c.Ri, c.f, c.theta, c.dt,
                     c.kstep, c.I, c.b);
  if (c.Rlr.ns > 0)
    hipLaunchKernelGGL(lowrank_rhs_k, dim3(1), dim3(256), 0, s, c.Rlr, c.dt, c.I, c.b);
  for (int64_t J = 0; J < NB; ++J) {
    launch_diag(true, B, dgrid, s, n, J, c);
    const int64_t below = n - (J + 1) * B;
    if (below > 0)
      hipLaunchKernelGGL(fwd_update_k, dim3((unsigned)ceil_div(below, 64)), dim3(64 * UW), 0, s,
                         n, B, J, c.Cf, c.ld, c.y, c.b);
  }
  for (int64_t J = NB - 1; J >= 0; --J) {
    launch_diag(false, B, dgrid, s, n, J, c);
    const int64_t J0 = J * B;
    if (J0 > 0)
      hipLaunchKernelGGL(bwd_update_k, dim3((unsigned)ceil_div(J0, (NT / 64) * BCOLS)), dim3(NT),
                         0, s, n, B, J, c.Cf, c.ld, c.b, c.y);
  }
  hipLaunchKernelGGL(step_inc_k, dim3(1), dim3(64), 0, s, c.kstep);
}

}  // namespace

int trsv_block(int64_t n) {
  // about eight diagonal blocks, at most 2048: fewer, larger launches (4096
  // measured no faster at N = 16384 and doubles the inverse blocks' memory)
  int B = 256;
  while (B < 2048 && 8 * (int64_t)(2 * B) <= n) B *= 2;
  return B;
}

int64_t trsv_parts(int64_t n) {
  const int B = trsv_block(n);
  return ceil_div(n, B) * diag_groups(B);
}

void chol_steps(const CholStep& c, int64_t k0, int64_t n_steps, hipStream_t s) {
  MM_REQUIRE(c.B == 256 || c.B == 512 || c.B == 1024 || c.B == 2048 || c.B == 4096, kInvalid,
             "chol_steps: block size must be a power of two in [256, 4096]");
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
