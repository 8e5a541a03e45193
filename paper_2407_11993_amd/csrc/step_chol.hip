// The classical theta-method (Sec. 3.3.1, eq. time_integration): per step
//   b = -dt Ri Ii + f^k;  C y = b;  C^T dI = y;  Ii += dI;  s = P dI / dt,
// with C the Cholesky factor of Z = Li + theta dt Ri.
//
// Block substitution with pre-scaled panels.  With D = blockdiag(C_JJ) (B x B
// blocks, B = 2048 at large N) the two solves are
//   forward:  y_J = D_J^{-1} b_J - sum_{K<J} W_JK y_K,      W_JK = D_J^{-1} C_JK,
//   backward: x_J = D_J^{-T} y_J - sum_{K>J} V_KJ^T x_K,    V_KJ = C_KJ D_J^{-1}.
// W and V are formed once per factorisation and stored as panels whose rows
// are contiguous: panel K of the forward solve holds, for every row i below
// block K, the B entries W(i, block K); panel K of the backward solve holds,
// for every row i above block K, the entries V^T(i, block K).  A solve is one
// block-diagonal product over all blocks at once (the block inverses' lower
// triangles, two rows folded per wave), then a chain of panel updates with no
// diagonal work between them, each a set of row dot products streaming its
// panel front to back, one wave per row.  The words read per solve equal
// those of C's lower triangle, and the solves are HBM-bound.
// Synchronisation is by kernel boundaries only (no workgroup waits on
// another); every sum has a fixed order, so reruns are bit-identical.
//
// One step's launches read the step index from device memory, so the whole
// step is captured once into a HIP graph and replayed n_steps times.
#include "kernels.h"

namespace mm {
namespace {

constexpr int NT = 256;

// Wave-wide sum, every lane gets the result: sums over quads and rows of 16
// lanes by DPP moves (xor 1, xor 2, half-row mirror, row mirror), then the
// four row sums read with readlane and added in a fixed order.
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const int2 b = __builtin_bit_cast(int2, v);
  int2 r;
  r.x = __builtin_amdgcn_update_dpp(0, b.x, CTRL, 0xF, 0xF, false);
  r.y = __builtin_amdgcn_update_dpp(0, b.y, CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, r);
}
__device__ __forceinline__ double lane_value(double v, int l) {
  const int2 b = __builtin_bit_cast(int2, v);
  int2 r;
  r.x = __builtin_amdgcn_readlane(b.x, l);
  r.y = __builtin_amdgcn_readlane(b.y, l);
  return __builtin_bit_cast(double, r);
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp<0xB1>(v);
  v += dpp<0x4E>(v);
  v += dpp<0x141>(v);
  v += dpp<0x140>(v);
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

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

// b = -dt Ri I + F u^k, k = kstep[0]; the first thread copies k to kstep[1],
// where the step's last kernel reads it, so that kernel can advance kstep[0]
__global__ void chol_rhs_k(int64_t n0, Csr Ri, Forcing f, double theta, double dt,
                           int64_t* kstep, const double* __restrict__ I,
                           double* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t k = kstep[0];
  if (i == 0) kstep[1] = k;
  if (i >= n0) return;
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

// Block-diagonal products, all blocks in one launch (blockIdx.y = block J),
// one wave per row of the triangle:
//   forward  (LOWER): out_J(r) = sum_{c <= r} Dinv_J(r, c) in_J(c), row r of
//                     Dinv_J read contiguously from DinvT;
//   backward:         out_J(c) = sum_{r >= c} Dinv_J(r, c) in_J(r), column c
//                     of Dinv_J read contiguously.
// A wave takes R pairs of rows (p, jb - 1 - p), whose lengths add up to
// jb + 1, so every wave does the same work; a row's 64-entry chunks are
// loaded at once (chunks outside the triangle skipped, wave-uniformly) and
// reduced over the wave by DPP moves.  The block's input is staged in LDS
// once per workgroup.
template <int NL, bool LOWER>
__global__ void __launch_bounds__(NT) trid_k(int64_t n, const double* __restrict__ D,
                                             const double* __restrict__ in,
                                             double* __restrict__ out, int R) {
  constexpr int B = NL * 64;
  __shared__ double xs[B];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t J = blockIdx.y;
  const int64_t J0 = J * B;
  const int jb = (int)min((int64_t)B, n - J0);
  const int np = (jb + 1) / 2;  // pairs
  for (int c = t; c < B; c += NT) xs[c] = (c < jb) ? in[J0 + c] : 0.0;
  __syncthreads();
  const double* Db = D + J * (int64_t)B * B;
  for (int rr = 0; rr < 2 * R; ++rr) {
    const int p = (blockIdx.x * R + rr / 2) * (NT / 64) + wave;
    if (p >= np) break;  // wave-uniform
    const int a = (rr & 1) ? jb - 1 - p : p;
    if ((rr & 1) && a == p) break;  // the middle row of an odd block, done already
    // chunks [m0, m1] of this row hold its entries
    const int m0 = LOWER ? 0 : a / 64, m1 = LOWER ? a / 64 : (jb - 1) / 64;
    const double* row = Db + (int64_t)a * B;
    double pv[NL];
#pragma unroll
    for (int m = 0; m < NL; ++m) pv[m] = (m >= m0 && m <= m1) ? row[64 * m + lane] : 0.0;
    double a4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int m = 0; m < NL; ++m) {
      const int e = 64 * m + lane;
      const bool ok = LOWER ? e <= a : e >= a;  // the triangle (xs is zero past jb)
      a4[m & 3] += ok ? pv[m] * xs[e] : 0.0;
    }
    const double d = wave_sum_dpp((a4[0] + a4[1]) + (a4[2] + a4[3]));
    if (lane == 0) out[J0 + a] = d;
  }
}

// Panel update, one wave per row:
//   vec(row0 + i) -= sum_{c < jb} P(c, i) vec(col0 + c),   0 <= i < nrows,
// with P (B x nrows, column-major, leading dimension B) the panel, so row i's
// B entries are contiguous.  Lane l reads entries l + 64 m (every wave load
// one contiguous 512-byte segment, all B / 64 of a row in flight at once),
// the block's values vec(col0 + c) (zero past jb) are staged in LDS once per
// workgroup, and a row's sum is reduced over the wave by DPP moves.  A
// workgroup's rows are consecutive (wave w takes rows w, w + 4, ...), so it
// streams one contiguous piece of the panel; latency is hidden by the other
// waves of the CU.
template <int NL>
__global__ void __launch_bounds__(NT) rowupd_k(int64_t row0, int64_t nrows, int64_t col0, int jb,
                                               const double* __restrict__ P,
                                               double* __restrict__ vec, int R) {
  constexpr int B = NL * 64;
  __shared__ double xs[B];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  int64_t i = (int64_t)blockIdx.x * R * (NT / 64) + wave;
  double pv[NL];
  if (i < nrows) {
#pragma unroll
    for (int m = 0; m < NL; ++m) pv[m] = P[i * B + 64 * m + lane];
  }
  for (int c = t; c < B; c += NT) xs[c] = (c < jb) ? vec[col0 + c] : 0.0;
  __syncthreads();
  for (int r = 0; r < R && i < nrows; ++r) {
    if (r > 0) {
#pragma unroll
      for (int m = 0; m < NL; ++m) pv[m] = P[i * B + 64 * m + lane];
    }
    double a4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int m = 0; m < NL; ++m) a4[m & 3] += pv[m] * xs[64 * m + lane];
    const double d = wave_sum_dpp((a4[0] + a4[1]) + (a4[2] + a4[3]));
    if (lane == 0) vec[row0 + i] -= d;
    i += NT / 64;
  }
}

// End of a step: Ii += dI (dI = x, the backward solve's result) and the probe
// partial sums of this workgroup's 256 rows (one per workgroup and probe,
// fixed order).  The step index is kstep[1]; the first thread advances
// kstep[0] (read by no other kernel of the step after chol_rhs_k).
__global__ void __launch_bounds__(NT) finish_k(int64_t n, const double* __restrict__ x,
                                               double* __restrict__ state,
                                               const double* __restrict__ Pt, int n_probe,
                                               double* __restrict__ pp_base,
                                               int64_t* kstep, int64_t parts,
                                               double* __restrict__ dI_out) {
  __shared__ double red[8][NT / 64];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t i = (int64_t)blockIdx.x * NT + t;
  const int64_t k = kstep[1];
  double d = 0.0;
  if (i < n) {
    d = x[i];
    state[i] += d;
    if (dI_out) dI_out[i + k * n] = d;
  }
  if (i == 0) kstep[0] = k + 1;
  for (int p = 0; p < n_probe; ++p) {
    const double v = wave_sum_dpp(i < n ? Pt[i + (int64_t)p * n] * d : 0.0);
    if (lane == 0) red[p][wave] = v;
  }
  __syncthreads();
  if (t < n_probe)
    pp_base[(k * parts + blockIdx.x) * n_probe + t] =
        (red[t][0] + red[t][1]) + (red[t][2] + red[t][3]);
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

// Panel offsets (in doubles): forward panel K (K < NB - 1) is B x (n - (K+1) B),
// backward panel K (K >= 1) is B x K B, each stored after the previous ones.
int64_t fwd_panel_offset(int64_t n, int B, int64_t K) {
  // sum_{K' < K} B (n - (K' + 1) B)
  return (int64_t)B * (K * n - (int64_t)B * K * (K + 1) / 2);
}
int64_t bwd_panel_offset(int B, int64_t K) {
  // sum_{1 <= K' < K} B K' B
  return (int64_t)B * B * (K * (K - 1) / 2);
}

// Rows (pairs) per wave: about five workgroups per CU in all.
int rows_per_wave(int64_t rows) {
  constexpr int64_t kSlots = 256 * 5 * (NT / 64);
  return (int)std::max<int64_t>(1, ceil_div(rows, kSlots));
}

template <int NL>
void launch_trid(bool lower, const CholStep& c, const double* in, double* out, hipStream_t s) {
  const int64_t n = c.n0;
  const int64_t NB = ceil_div(n, (int64_t)c.B);
  const int64_t pairs = (c.B + 1) / 2;
  const int R = rows_per_wave(pairs * NB);
  const dim3 grid((unsigned)ceil_div(pairs, (int64_t)R * (NT / 64)), (unsigned)NB);
  if (lower)
    hipLaunchKernelGGL((trid_k<NL, true>), grid, dim3(NT), 0, s, n, c.DinvT, in, out, R);
  else
    hipLaunchKernelGGL((trid_k<NL, false>), grid, dim3(NT), 0, s, n, c.Dinv, in, out, R);
}

template <int NL>
void launch_rowupd(int64_t row0, int64_t nrows, int64_t col0, int jb, const double* P,
                   double* vec, hipStream_t s) {
  if (nrows <= 0) return;
  const int R = rows_per_wave(nrows);
  hipLaunchKernelGGL((rowupd_k<NL>), dim3((unsigned)ceil_div(nrows, (int64_t)R * (NT / 64))),
                     dim3(NT), 0, s, row0, nrows, col0, jb, P, vec, R);
}

// One step's launch sequence (the step index is kstep[0], advanced by the
// last kernel):
//   b = rhs;  y = D^{-1} b;  for K = 0..NB-2: y(rows below K) -= W(:, K) y_K;
//   x = D^{-T} y (into b);   for K = NB-1..1: x(rows above K) -= V^T(:, K) x_K;
//   Ii += x;  probe partial sums.
template <int NL>
void enqueue_step_b(const CholStep& c, hipStream_t s) {
  const int64_t n = c.n0;
  const int B = c.B;
  const int64_t NB = ceil_div(n, (int64_t)B);
  const int64_t parts = trsv_parts(n);
  const unsigned rgrid = (unsigned)ceil_div(n, 256);
  hipLaunchKernelGGL(chol_rhs_k, dim3(rgrid), dim3(256), 0, s, n, c.Ri, c.f, c.theta, c.dt,
                     c.kstep, c.I, c.b);
  if (c.Rlr.ns > 0)
    hipLaunchKernelGGL(lowrank_rhs_k, dim3(1), dim3(256), 0, s, c.Rlr, c.dt, c.I, c.b);
  launch_trid<NL>(true, c, c.b, c.y, s);
  for (int64_t K = 0; K + 1 < NB; ++K)
    launch_rowupd<NL>((K + 1) * B, n - (K + 1) * B, K * B, B, c.pf + fwd_panel_offset(n, B, K),
                      c.y, s);
  launch_trid<NL>(false, c, c.y, c.b, s);
  for (int64_t K = NB - 1; K >= 1; --K)
    launch_rowupd<NL>(0, K * B, K * B, (int)std::min<int64_t>(B, n - K * B),
                      c.pb + bwd_panel_offset(B, K), c.b, s);
  hipLaunchKernelGGL(finish_k, dim3((unsigned)parts), dim3(NT), 0, s, n, c.b, c.I, c.Pt,
                     c.n_probe, c.probe_partial, c.kstep, parts, c.dI_out);
}

void enqueue_step(const CholStep& c, hipStream_t s) {
  switch (c.B) {
    case 256: enqueue_step_b<4>(c, s); break;
    case 512: enqueue_step_b<8>(c, s); break;
    case 1024: enqueue_step_b<16>(c, s); break;
    case 2048: enqueue_step_b<32>(c, s); break;
    default: throw Error{kInvalid, "triangular solve: unsupported block size"};
  }
}

}  // namespace

int trsv_block(int64_t n) {
  // about eight diagonal blocks, at most 2048 (4096 measured slower at
  // N = 16384: the 64-chunk rows lower the occupancy of both kernels)
  int B = 256;
  while (B < 2048 && 8 * (int64_t)(2 * B) <= n) B *= 2;
  return B;
}

int64_t trsv_parts(int64_t n) { return ceil_div(n, NT); }

void chol_steps(const CholStep& c, int64_t k0, int64_t n_steps, hipStream_t s) {
  MM_REQUIRE(c.B == 256 || c.B == 512 || c.B == 1024 || c.B == 2048, kInvalid,
             "chol_steps: block size must be a power of two in [256, 2048]");
  MM_REQUIRE(c.dI_out ? c.n_probe == 0 : c.n_probe <= 8, kInvalid,
             "chol_steps: at most 8 probes, or none with the increments written out");
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

int64_t trsv_panel_elems(int64_t n, int B) {
  const int64_t NB = ceil_div(n, (int64_t)B);
  return fwd_panel_offset(n, B, NB - 1) + bwd_panel_offset(B, NB);
}

void trsv_prescale(const double* Cf, int64_t n, int B, const double* Dinv, double* pf,
                   double* pb, hipStream_t s) {
  const int64_t NB = ceil_div(n, (int64_t)B);
  const int64_t nf = fwd_panel_offset(n, B, NB - 1);
  // the short last block leaves rows of the backward panels' columns unset
  fill(pb, bwd_panel_offset(B, NB), 0.0, s);
  for (int64_t K = 0; K + 1 < NB; ++K) {
    double* base = pf + fwd_panel_offset(n, B, K);
    for (int64_t I = K + 1; I < NB; ++I) {
      const int64_t jbI = std::min<int64_t>(B, n - I * B);
      Gemm g;  // W_IK^T = C_IK^T D_I^{-T}: row i of panel K is column i here
      g.m = B; g.n = jbI; g.k = jbI;
      g.A = Cf + I * B + K * B * n; g.lda = n; g.ta = true;
      g.B = Dinv + I * (int64_t)B * B; g.ldb = B; g.tb = true; g.b_band = 0;
      g.C = base + (I - K - 1) * (int64_t)B * B; g.ldc = B;
      gemm(g, s);
    }
  }
  (void)nf;
  for (int64_t K = 1; K < NB; ++K) {
    const int64_t jbK = std::min<int64_t>(B, n - K * B);
    double* base = pb + bwd_panel_offset(B, K);
    for (int64_t J = 0; J < K; ++J) {
      Gemm g;  // V_KJ = C_KJ D_J^{-1}: row i of panel K (in block J) is column i here
      g.m = jbK; g.n = B; g.k = B;
      g.A = Cf + K * B + J * B * n; g.lda = n;
      g.B = Dinv + J * (int64_t)B * B; g.ldb = B; g.b_lower = true;
      g.C = base + J * (int64_t)B * B; g.ldc = B;
      gemm(g, s);
    }
  }
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
