// The modal theta-method (Sec. 3.3.2): in the basis of Li-normalised
// generalized eigenvectors every mode is an independent scalar equation
//   y_n' + lam_n y_n = (W u)_n,
// stepped with  (1 + theta dt lam_n) dy_n = -dt lam_n y_n + (W u^k)_n,
// where u^k holds the source increments of step k (the same forcing as the
// Cholesky method, expressed in the modal basis), and the probe signal of
// the step is  s_p = sum_n Pt(n, p) dy_n / dt  (+ the direct electrode term).
//
// With exact = true every mode is integrated in closed form over the step,
// the waveforms taken linear between their samples: the forcing on the step
// is e1 + e2 s / dt (s in [0, dt]; e2 from the R_D i_D columns only) and
//   dy = -alpha y + beta e1 + gamma e2,   x = lam dt,
//   alpha = 1 - exp(-x), beta = alpha / x, gamma = (1 - beta) / x,
// in the same increment encoding of the forcing (e1 uses theta = 0).
//
// One launch runs all steps: a thread keeps its mode's amplitude, factor and
// weights in registers for the whole horizon, so HBM traffic is O(N + T).
// Each step reduces the probe contributions over the wave (xor butterfly)
// and the workgroup (LDS, double-buffered by step parity: one barrier per
// step) and writes one partial per workgroup; a second pass sums the
// partials in workgroup order, so the result is deterministic.
#include "kernels.h"

namespace mm {
namespace {

constexpr int NT = 256;
constexpr int MAXF = 8;
constexpr int MAXP = 8;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

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
// quads and rows of 16 by DPP (xor 1, xor 2, half-row and row mirrors), then
// the four rows' sums by readlane, added in a fixed order
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp<0xB1>(v);
  v += dpp<0x4E>(v);
  v += dpp<0x141>(v);
  v += dpp<0x140>(v);
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
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

constexpr int SM = 8;  // steps whose probe sums are reduced together

template <int NF, int NP>
__global__ void __launch_bounds__(NT) modal_step_k(ModalStep ms, int64_t n_steps) {
  __shared__ double red[2][SM][NT / 64][NP > 0 ? NP : 1];
  // waveform samples of a batch, rows k0 .. k0 + SM of [i_src | i_D], staged
  // one batch ahead (loaded while the current batch computes)
  __shared__ double wv[2][SM + 1][MAXF];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t n = (int64_t)blockIdx.x * NT + t;
  const int64_t n0 = ms.n0;
  const int nf = NF > 0 ? NF : ms.f.nf;
  const int np = ms.n_probe;  // <= NP (template capacity)
  const bool exact = ms.exact;
  const double th = exact ? 0.0 : ms.theta;
  double y = 0.0, c = 0.0, a = 0.0, g = 0.0;
  double w[MAXF], pt[NP > 0 ? NP : 1];
  for (int j = 0; j < MAXF; ++j) w[j] = 0.0;
  for (int p = 0; p < (NP > 0 ? NP : 1); ++p) pt[p] = 0.0;
  if (n < n0) {
    const double lam = ms.lam[n];
    y = ms.y[n];
    if (exact) {
      // a = alpha, c = beta, g = gamma; gamma summed as sum_k (-x)^k / (k+2)!
      // below x = 1/2, where 1 - beta cancels
      const double x = ms.dt * lam;
      a = -expm1(-x);
      if (x == 0.0) {
        c = 1.0;
        g = 0.5;
      } else {
        c = a / x;
        if (x < 0.5) {
          double term = 0.5;
          g = 0.0;
          for (int q = 0; q < 24; ++q) {
            g += term;
            term *= -x / (double)(q + 3);
          }
        } else {
          g = (1.0 - c) / x;
        }
      }
    } else {
      a = ms.dt * lam;
      c = 1.0 / (1.0 + ms.theta * ms.dt * lam);
    }
    for (int j = 0; j < nf; ++j) w[j] = ms.W[n + (int64_t)j * n0];
    for (int p = 0; p < np; ++p) pt[p] = ms.Pt[n + (int64_t)p * n0];
  }
  const int64_t G = gridDim.x;
  const int mD = ms.f.m;
  // Probe contributions of SM steps are kept per thread and reduced together:
  // one DPP wave sum each, one barrier per SM steps (LDS double-buffered by
  // batch parity), then threads t < SM np sum the four waves in order.
  const int ns = ms.f.n_src, nwc = ns + mD;  // <= nf <= MAXF waveform columns
  const bool stager = t < (SM + 1) * nwc;
  const int sr = stager ? t / nwc : 0, sc = stager ? t % nwc : 0;
  auto sample = [&](int64_t k0n) {  // row k0n + sr (clamped to the last sample)
    const int64_t k = min(k0n + sr, n_steps);
    return sc < ns ? ms.f.i_src[k * ns + sc] : ms.f.i_D[k * mD + (sc - ns)];
  };
  if (stager) wv[0][sr][sc] = sample(0);
  __syncthreads();
  for (int64_t k0 = 0; k0 < n_steps; k0 += SM) {
    const int buf = (int)((k0 / SM) & 1);
    const double next = (stager && k0 + SM < n_steps) ? sample(k0 + SM) : 0.0;
    double acc[SM][NP > 0 ? NP : 1];
#pragma unroll
    for (int i = 0; i < SM; ++i) {
      const int64_t k = k0 + i;
      double dy = 0.0;
      if (k < n_steps) {
        const double* S0 = wv[buf][i];      // samples k
        const double* S1 = wv[buf][i + 1];  // samples k + 1
        double e = 0.0, e2 = 0.0;
#pragma unroll
        for (int j = 0; j < MAXF; ++j) {
          if (j < nf) {
            double u;
            if (j < mD) {  // R_D: -dt (iD^k + theta d iD)
              const double a0 = S0[ns + j], a1 = S1[ns + j];
              u = -ms.dt * (a0 + th * (a1 - a0));
              e2 += w[j] * (-ms.dt * (a1 - a0));
            } else if (j < 2 * mD) {  // L_D: -d iD
              u = -(S1[ns + j - mD] - S0[ns + j - mD]);
            } else {  // sources: -d i0
              u = -(S1[j - 2 * mD] - S0[j - 2 * mD]);
            }
            e += w[j] * u;
          }
        }
        dy = exact ? c * e + g * e2 - a * y : c * (e - a * y);
        y += dy;
        if (ms.dy_out && n < n0) ms.dy_out[n + k * n0] = dy;
      }
#pragma unroll
      for (int p = 0; p < (NP > 0 ? NP : 1); ++p) acc[i][p] = pt[p] * dy;
    }
    if (stager && k0 + SM < n_steps) wv[buf ^ 1][sr][sc] = next;
#pragma unroll
    for (int i = 0; i < SM; ++i)
#pragma unroll
      for (int p = 0; p < (NP > 0 ? NP : 1); ++p)
        if (p < np) {
          const double v = wave_sum_dpp(acc[i][p]);
          if (lane == 0) red[buf][i][wave][p] = v;
        }
    __syncthreads();
    if (t < SM * np) {
      const int i = t / np, p = t % np;
      const int64_t k = k0 + i;
      if (k < n_steps) {
        const double s = (red[buf][i][0][p] + red[buf][i][1][p]) +
                         (red[buf][i][2][p] + red[buf][i][3][p]);
        ms.probe_partial[(k * G + blockIdx.x) * np + p] = s;
      }
    }
  }
  if (n < n0) ms.y[n] = y;
}

// ---------------------------------------------------------------------------
// Time-parallel variant for few modes and many steps.  Per mode a step is the
// affine map y -> A y + b_k (theta: A = 1 - c dt lam, b_k = c e_k; exact:
// A = exp(-lam dt), b_k = beta e1_k + gamma e2_k).  The horizon is cut into
// chunks of L steps: (1) every (mode group, chunk) workgroup runs its chunk
// from a zero state and stores the end value Z; (2) one pass per mode chains
// the chunks, y_{q+1} = A^len_q y_q + Z_q, giving every chunk's start state;
// (3) the chunks are rerun from their start states and write the per-step
// probe partials of the sequential kernel.  2 N T mode-steps instead of N T,
// spread over (N / 256) x (T / L) workgroups instead of N / 256.
// ---------------------------------------------------------------------------
struct Coef {
  double A, c, g;  // y_{k+1} = A y_k + c e_k (+ g e2_k for exact)
};

__device__ Coef mode_coef(const ModalStep& ms, double lam) {
  Coef r;
  const double x = ms.dt * lam;
  if (ms.exact) {
    const double al = -expm1(-x);
    r.A = exp(-x);
    if (x == 0.0) {
      r.c = 1.0;
      r.g = 0.5;
    } else {
      r.c = al / x;
      if (x < 0.5) {
        double term = 0.5;
        r.g = 0.0;
        for (int q = 0; q < 24; ++q) {
          r.g += term;
          term *= -x / (double)(q + 3);
        }
      } else {
        r.g = (1.0 - r.c) / x;
      }
    }
  } else {
    r.c = 1.0 / (1.0 + ms.theta * x);
    r.A = 1.0 - r.c * x;
    r.g = 0.0;
  }
  return r;
}

template <int NF, int NP, bool PROBE>
__global__ void __launch_bounds__(NT) modal_chunk_k(ModalStep ms, int64_t n_steps, int64_t L,
                                                    const double* ystart, double* Z) {
  __shared__ double red[2][SM][NT / 64][NP > 0 ? NP : 1];
  __shared__ double wv[2][SM + 1][MAXF];  // waveform samples, one batch ahead
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t n = (int64_t)blockIdx.x * NT + t;
  const int64_t n0 = ms.n0;
  const int64_t q = blockIdx.y;
  const int64_t kc0 = q * L, kc1 = min(kc0 + L, n_steps);
  const int nf = NF > 0 ? NF : ms.f.nf;
  const int np = ms.n_probe;
  const bool exact = ms.exact;
  const double th = exact ? 0.0 : ms.theta;
  const int mD = ms.f.m;
  Coef cf{1.0, 0.0, 0.0};
  double y = 0.0;
  double w[MAXF], pt[NP > 0 ? NP : 1];
  for (int j = 0; j < MAXF; ++j) w[j] = 0.0;
  for (int p = 0; p < (NP > 0 ? NP : 1); ++p) pt[p] = 0.0;
  if (n < n0) {
    cf = mode_coef(ms, ms.lam[n]);
    for (int j = 0; j < nf; ++j) w[j] = ms.W[n + (int64_t)j * n0];
    if (PROBE) {
      for (int p = 0; p < np; ++p) pt[p] = ms.Pt[n + (int64_t)p * n0];
      y = ystart[q * n0 + n];
    }
  }
  const int64_t G = gridDim.x;
  // batches of SM steps as in modal_step_k: samples staged one batch ahead,
  // probe sums of the batch reduced together
  const int ns = ms.f.n_src, nwc = ns + mD;
  const bool stager = t < (SM + 1) * nwc;
  const int sr = stager ? t / nwc : 0, sc = stager ? t % nwc : 0;
  auto sample = [&](int64_t k0n) {
    const int64_t k = min(k0n + sr, n_steps);
    return sc < ns ? ms.f.i_src[k * ns + sc] : ms.f.i_D[k * mD + (sc - ns)];
  };
  if (stager) wv[0][sr][sc] = sample(kc0);
  __syncthreads();
  for (int64_t k0 = kc0; k0 < kc1; k0 += SM) {
    const int buf = (int)(((k0 - kc0) / SM) & 1);
    const double next = (stager && k0 + SM < kc1) ? sample(k0 + SM) : 0.0;
    double acc[SM][NP > 0 ? NP : 1];
#pragma unroll
    for (int i = 0; i < SM; ++i) {
      const int64_t k = k0 + i;
      double dy = 0.0;
      if (k < kc1) {
        const double* S0 = wv[buf][i];
        const double* S1 = wv[buf][i + 1];
        double e = 0.0, e2 = 0.0;
#pragma unroll
        for (int j = 0; j < MAXF; ++j) {
          if (j < nf) {
            double u;
            if (j < mD) {
              const double a0 = S0[ns + j], a1 = S1[ns + j];
              u = -ms.dt * (a0 + th * (a1 - a0));
              e2 += w[j] * (-ms.dt * (a1 - a0));
            } else if (j < 2 * mD) {
              u = -(S1[ns + j - mD] - S0[ns + j - mD]);
            } else {
              u = -(S1[j - 2 * mD] - S0[j - 2 * mD]);
            }
            e += w[j] * u;
          }
        }
        double b = cf.c * e;
        if (exact) b += cf.g * e2;
        dy = (cf.A - 1.0) * y + b;
        y += dy;
      }
#pragma unroll
      for (int p = 0; p < (NP > 0 ? NP : 1); ++p) acc[i][p] = pt[p] * dy;
    }
    if (stager && k0 + SM < kc1) wv[buf ^ 1][sr][sc] = next;
    if (PROBE) {
#pragma unroll
      for (int i = 0; i < SM; ++i)
#pragma unroll
        for (int p = 0; p < (NP > 0 ? NP : 1); ++p)
          if (p < np) {
            const double v = wave_sum_dpp(acc[i][p]);
            if (lane == 0) red[buf][i][wave][p] = v;
          }
    }
    __syncthreads();
    if (PROBE && t < SM * np) {
      const int i = t / np, p = t % np;
      const int64_t k = k0 + i;
      if (k < kc1) {
        const double s = (red[buf][i][0][p] + red[buf][i][1][p]) +
                         (red[buf][i][2][p] + red[buf][i][3][p]);
        ms.probe_partial[(k * G + blockIdx.x) * np + p] = s;
      }
    }
  }
  if (!PROBE && n < n0) Z[q * n0 + n] = y;
}

// start states of the chunks: ystart[q n0 + n], q < Q; the final state to ms.y
__global__ void modal_chain_k(ModalStep ms, int64_t n_steps, int64_t L, int64_t Q,
                              const double* Z, double* ystart) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n0 = ms.n0;
  if (n >= n0) return;
  const Coef cf = mode_coef(ms, ms.lam[n]);
  const double AL = pow(cf.A, (double)L);
  const double Alast = pow(cf.A, (double)(n_steps - (Q - 1) * L));
  double y = ms.y[n];
  for (int64_t q = 0; q < Q; ++q) {
    ystart[q * n0 + n] = y;
    y = (q < Q - 1 ? AL : Alast) * y + Z[q * n0 + n];
  }
  ms.y[n] = y;
}

template <int NF, int NP>
void launch_scan(const ModalStep& m, int64_t n_steps, int64_t L, int64_t Q, double* Z,
                 double* ystart, hipStream_t s) {
  const dim3 grid((unsigned)modal_groups(m.n0), (unsigned)Q);
  hipLaunchKernelGGL((modal_chunk_k<NF, NP, false>), grid, dim3(NT), 0, s, m, n_steps, L,
                     (const double*)nullptr, Z);
  hipLaunchKernelGGL(modal_chain_k, dim3((unsigned)ceil_div(m.n0, 256)), dim3(256), 0, s, m,
                     n_steps, L, Q, (const double*)Z, ystart);
  hipLaunchKernelGGL((modal_chunk_k<NF, NP, true>), grid, dim3(NT), 0, s, m, n_steps, L,
                     (const double*)ystart, (double*)nullptr);
}

template <int NF>
void launch_scan_np(const ModalStep& m, int64_t n_steps, int64_t L, int64_t Q, double* Z,
                    double* ystart, hipStream_t s) {
  if (m.n_probe <= 1) launch_scan<NF, 1>(m, n_steps, L, Q, Z, ystart, s);
  else if (m.n_probe <= 2) launch_scan<NF, 2>(m, n_steps, L, Q, Z, ystart, s);
  else if (m.n_probe <= 4) launch_scan<NF, 4>(m, n_steps, L, Q, Z, ystart, s);
  else launch_scan<NF, 8>(m, n_steps, L, Q, Z, ystart, s);
}

template <int NF>
void launch_np(const ModalStep& m, int64_t n_steps, hipStream_t s, dim3 grid) {
  if (m.n_probe <= 1) hipLaunchKernelGGL((modal_step_k<NF, 1>), grid, dim3(NT), 0, s, m, n_steps);
  else if (m.n_probe <= 2) hipLaunchKernelGGL((modal_step_k<NF, 2>), grid, dim3(NT), 0, s, m, n_steps);
  else if (m.n_probe <= 4) hipLaunchKernelGGL((modal_step_k<NF, 4>), grid, dim3(NT), 0, s, m, n_steps);
  else hipLaunchKernelGGL((modal_step_k<NF, 8>), grid, dim3(NT), 0, s, m, n_steps);
}

// ---------------------------------------------------------------------------
// Batched runs: workgroup (mode group g, run r).  Each thread holds MPT modes
// (amplitude, factors, the run's forcing and probe weights) in registers for
// the whole run.  Probe contributions are accumulated per thread over S steps
// and reduced (wave by DPP moves, workgroup through LDS) once per S steps.
// ---------------------------------------------------------------------------
constexpr int S = 8;  // steps per reduction

template <int NTB, int MPT>
__global__ void __launch_bounds__(NTB) batch_step_k(BatchStep b) {
  constexpr int NW = NTB / 64;
  __shared__ double red[2][S][NW];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int g = blockIdx.x;
  const int r = b.order[blockIdx.y];
  const int64_t T = b.lens[r];
  if (T == 0) return;
  const int64_t n0 = b.n0;
  const double* Wc = b.W + (int64_t)b.wcol[r] * b.ldw;
  const double* Pc = b.Pm + (int64_t)b.pcol[r] * n0;
  double y[MPT], c[MPT], a[MPT], w[MPT], p[MPT];
#pragma unroll
  for (int i = 0; i < MPT; ++i) {
    const int64_t n = (int64_t)g * NTB * MPT + (int64_t)i * NTB + t;
    y[i] = 0.0;
    c[i] = a[i] = w[i] = p[i] = 0.0;
    if (n < n0) {
      const double lam = b.lam[n];
      a[i] = b.dt * lam;
      c[i] = 1.0 / (1.0 + b.theta * b.dt * lam);
      w[i] = Wc[n];
      p[i] = Pc[n];
    }
  }
  const double* wv = b.waves + b.woff[r];
  double* part = b.partial + b.soff[r] * b.G + g;
  for (int64_t k0 = 0, it = 0; k0 < T; k0 += S, ++it) {
    double smp[S + 1];
#pragma unroll
    for (int q = 0; q <= S; ++q) smp[q] = wv[min(k0 + q, T)];
    double acc[S];
#pragma unroll
    for (int q = 0; q < S; ++q) {
      acc[q] = 0.0;
      if (k0 + q < T) {
        const double u = -(smp[q + 1] - smp[q]);
#pragma unroll
        for (int i = 0; i < MPT; ++i) {
          const double dy = c[i] * (w[i] * u - a[i] * y[i]);
          y[i] += dy;
          acc[q] += p[i] * dy;
        }
      }
    }
    const int buf = (int)(it & 1);
#pragma unroll
    for (int q = 0; q < S; ++q) {
      const double v = wave_sum_dpp(acc[q]);
      if (lane == 0) red[buf][q][wave] = v;
    }
    __syncthreads();
    if (t < S && k0 + t < T) {
      double v = 0.0;
#pragma unroll
      for (int ww = 0; ww < NW; ++ww) v += red[buf][t][ww];
      part[(k0 + t) * b.G] = v;
    }
  }
}

// signal[e] = sum_g partial[e G + g] / dt, in group order
__global__ void batch_finish_k(const double* partial, int64_t total, int G, double dt,
                               double* signal) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const double* q = partial + e * G;
  double s = 0.0;
  for (int g = 0; g < G; ++g) s += q[g];
  signal[e] = s / dt;
}

template <int NTB, int MPT>
void launch_batch(const BatchStep& b, hipStream_t s) {
  hipLaunchKernelGGL((batch_step_k<NTB, MPT>), dim3((unsigned)b.G, (unsigned)b.n_runs),
                     dim3(NTB), 0, s, b);
}

}  // namespace

const BatchTile kBatchTiles[] = {{256, 1}, {256, 2}, {256, 4}, {128, 4}, {256, 8}, {128, 8}};
const int kNumBatchTiles = (int)(sizeof(kBatchTiles) / sizeof(kBatchTiles[0]));

int batch_groups(int64_t n0, int tile) {
  const BatchTile& bt = kBatchTiles[tile];
  return (int)std::max<int64_t>(1, ceil_div(n0, (int64_t)bt.threads * bt.modes));
}

void batch_steps(const BatchStep& b, int tile, int64_t total_steps, double* signal,
                 hipStream_t s) {
  MM_REQUIRE(tile >= 0 && tile < kNumBatchTiles, kInvalid, "batch_steps: tile");
  MM_REQUIRE(b.G == batch_groups(b.n0, tile), kInvalid, "batch_steps: group count");
  if (b.n_runs <= 0) return;
  switch (tile) {
    case 0: launch_batch<256, 1>(b, s); break;
    case 1: launch_batch<256, 2>(b, s); break;
    case 2: launch_batch<256, 4>(b, s); break;
    case 3: launch_batch<128, 4>(b, s); break;
    case 4: launch_batch<256, 8>(b, s); break;
    default: launch_batch<128, 8>(b, s); break;
  }
  MM_HIP_TRY(hipGetLastError());
  if (total_steps > 0 && signal) {
    hipLaunchKernelGGL(batch_finish_k, dim3((unsigned)ceil_div(total_steps, 256)), dim3(256), 0,
                       s, b.partial, total_steps, b.G, b.dt, signal);
    MM_HIP_TRY(hipGetLastError());
  }
}

int modal_groups(int64_t n0) { return (int)std::max<int64_t>(1, ceil_div(n0, NT)); }

int64_t scan_chunk(int64_t n0, int64_t n_steps) {
  // about 2048 workgroups, chunks of at least 32 steps, at most 65535 chunks
  const int64_t want = std::max<int64_t>(1, 2048 / modal_groups(n0));
  int64_t L = std::max<int64_t>(32, ceil_div(n_steps, want));
  L = std::max<int64_t>(L, ceil_div(n_steps, 65535));
  return L;
}

void modal_steps_scan(const ModalStep& m, int64_t n_steps, int64_t L, double* ws,
                      hipStream_t s) {
  if (n_steps <= 0) return;
  MM_REQUIRE(m.f.nf <= MAXF, kInvalid, "modal_steps: too many forcing columns");
  MM_REQUIRE(m.n_probe >= 1 && m.n_probe <= MAXP, kInvalid,
             "modal_steps: 1..8 probes per run");
  const int64_t Q = ceil_div(n_steps, L);
  MM_REQUIRE(L >= 1 && Q <= 65535, kInvalid, "modal_steps_scan: at most 65535 chunks");
  double* Z = ws;
  double* ystart = ws + Q * m.n0;
  if (m.f.nf == 1) launch_scan_np<1>(m, n_steps, L, Q, Z, ystart, s);
  else launch_scan_np<0>(m, n_steps, L, Q, Z, ystart, s);
  MM_HIP_TRY(hipGetLastError());
}

void modal_steps(const ModalStep& m, int64_t k0, int64_t n_steps, hipStream_t s) {
  (void)k0;
  if (n_steps <= 0) return;
  MM_REQUIRE(m.f.nf <= MAXF, kInvalid, "modal_steps: too many forcing columns");
  MM_REQUIRE(m.dy_out ? m.n_probe == 0 : (m.n_probe >= 1 && m.n_probe <= MAXP), kInvalid,
             "modal_steps: 1..8 probes per run, or none with the increments written out");
  dim3 grid((unsigned)modal_groups(m.n0));
  if (m.f.nf == 1) launch_np<1>(m, n_steps, s, grid);
  else launch_np<0>(m, n_steps, s, grid);
  MM_HIP_TRY(hipGetLastError());
}

}  // namespace mm
