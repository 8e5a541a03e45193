// The modal theta-method (Sec. 3.3.2): in the basis of Li-normalised
// generalized eigenvectors every mode is an independent scalar equation
//   y_n' + lam_n y_n = (W u)_n,
// stepped with  (1 + theta dt lam_n) dy_n = -dt lam_n y_n + (W u^k)_n,
// where u^k holds the source increments of step k (the same forcing as the
// Cholesky method, expressed in the modal basis), and the probe signal of
// the step is  s_p = sum_n Pt(n, p) dy_n / dt  (+ the direct electrode term).
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

template <int NF, int NP>
__global__ void __launch_bounds__(NT) modal_step_k(ModalStep ms, int64_t n_steps) {
  __shared__ double red[2][NT / 64][NP > 0 ? NP : 1];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t n = (int64_t)blockIdx.x * NT + t;
  const int64_t n0 = ms.n0;
  const int nf = NF > 0 ? NF : ms.f.nf;
  const int np = ms.n_probe;  // <= NP (template capacity)
  double y = 0.0, c = 0.0, a = 0.0;
  double w[MAXF], pt[NP > 0 ? NP : 1];
  for (int j = 0; j < MAXF; ++j) w[j] = 0.0;
  for (int p = 0; p < (NP > 0 ? NP : 1); ++p) pt[p] = 0.0;
  if (n < n0) {
    const double lam = ms.lam[n];
    y = ms.y[n];
    a = ms.dt * lam;
    c = 1.0 / (1.0 + ms.theta * ms.dt * lam);
    for (int j = 0; j < nf; ++j) w[j] = ms.W[n + (int64_t)j * n0];
    for (int p = 0; p < np; ++p) pt[p] = ms.Pt[n + (int64_t)p * n0];
  }
  const int64_t G = gridDim.x;
  for (int64_t k = 0; k < n_steps; ++k) {
    double e = 0.0;
#pragma unroll
    for (int j = 0; j < MAXF; ++j)
      if (j < nf) e += w[j] * forcing_u(ms.f, j, k, ms.theta, ms.dt);
    const double dy = c * (e - a * y);
    y += dy;
    const int buf = (int)(k & 1);
#pragma unroll
    for (int p = 0; p < (NP > 0 ? NP : 1); ++p) {
      if (p < np) {
        const double v = wave_sum(pt[p] * dy);
        if (lane == 0) red[buf][wave][p] = v;
      }
    }
    __syncthreads();
    if (t < np) {
      const double s = (red[buf][0][t] + red[buf][1][t]) + (red[buf][2][t] + red[buf][3][t]);
      ms.probe_partial[(k * G + blockIdx.x) * np + t] = s;
    }
  }
  if (n < n0) ms.y[n] = y;
}

template <int NF>
void launch_np(const ModalStep& m, int64_t n_steps, hipStream_t s, dim3 grid) {
  if (m.n_probe <= 1) hipLaunchKernelGGL((modal_step_k<NF, 1>), grid, dim3(NT), 0, s, m, n_steps);
  else if (m.n_probe <= 2) hipLaunchKernelGGL((modal_step_k<NF, 2>), grid, dim3(NT), 0, s, m, n_steps);
  else if (m.n_probe <= 4) hipLaunchKernelGGL((modal_step_k<NF, 4>), grid, dim3(NT), 0, s, m, n_steps);
  else hipLaunchKernelGGL((modal_step_k<NF, 8>), grid, dim3(NT), 0, s, m, n_steps);
}

}  // namespace

int modal_groups(int64_t n0) { return (int)std::max<int64_t>(1, ceil_div(n0, NT)); }

void modal_steps(const ModalStep& m, int64_t k0, int64_t n_steps, hipStream_t s) {
  (void)k0;
  if (n_steps <= 0) return;
  MM_REQUIRE(m.f.nf <= MAXF, kInvalid, "modal_steps: too many forcing columns");
  MM_REQUIRE(m.n_probe >= 1 && m.n_probe <= MAXP, kInvalid,
             "modal_steps: 1..8 probes per run");
  dim3 grid((unsigned)modal_groups(m.n0));
  if (m.f.nf == 1) launch_np<1>(m, n_steps, s, grid);
  else launch_np<0>(m, n_steps, s, grid);
  MM_HIP_TRY(hipGetLastError());
}

}  // namespace mm
