// Steady-state probe phasors by the modal decomposition (Sec. 3.2, eq.
// modal_decomposition_discrete; the frequency-domain comparison of Sec. 4.6).
// With sources i(t) = Re{A exp(j w t)} every decoupled mode obeys
//   (lam_n + j w) y_n = sum_j W(n, j) u_j(w),
// where the forcing columns keep the time-domain encoding with d/dt -> j w:
//   R_D columns (a < m):   u = -ID_a
//   L_D columns:           u = -j w ID_a
//   source columns:        u = -j w I0_c,
// and the phasor of the probe signal P dI/dt is
//   S_p(w) = j w (sum_n Pt(n, p) y_n + sum_a PD(p, a) ID_a).
// One frequency costs O(N) instead of the frequency-domain method's complex
// factorisation of R + j w L.
//
// Workgroup (mode group g, frequency w): one mode per thread, the mode's
// lambda, forcing and probe weights in registers; each probe's complex
// contribution is reduced over the wave (xor butterfly) and the workgroup
// (LDS) into one partial per (w, g); a second kernel sums the partials in
// group order (deterministic) and adds the direct electrode term.
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

__global__ void __launch_bounds__(NT) phasor_modes_k(ModalPhasor mp) {
  __shared__ double red[NT / 64][MAXP][2];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t n = (int64_t)blockIdx.x * NT + t;
  const int64_t w = blockIdx.y;
  const int m = mp.m, ns = mp.n_src, nf = 2 * m + ns, np = mp.n_probe;
  const double om = mp.omega[w];
  double yr = 0.0, yi = 0.0;
  if (n < mp.n0) {
    // e = sum_j W(n, j) u_j
    double er = 0.0, ei = 0.0;
    for (int j = 0; j < nf; ++j) {
      const double wv = mp.W[n + (int64_t)j * mp.n0];
      double ur, ui;
      if (j < m) {
        ur = -mp.amp_D[(w * m + j) * 2];
        ui = -mp.amp_D[(w * m + j) * 2 + 1];
      } else if (j < 2 * m) {  // -j w ID:  -j w (a + j b) = w b - j w a
        const double a = mp.amp_D[(w * m + (j - m)) * 2], b = mp.amp_D[(w * m + (j - m)) * 2 + 1];
        ur = om * b;
        ui = -om * a;
      } else {
        const int c = j - 2 * m;
        const double a = mp.amp_src[(w * ns + c) * 2], b = mp.amp_src[(w * ns + c) * 2 + 1];
        ur = om * b;
        ui = -om * a;
      }
      er += wv * ur;
      ei += wv * ui;
    }
    // y = e / (lam + j w) = e (lam - j w) / (lam^2 + w^2)
    const double lam = mp.lam[n];
    const double d = lam * lam + om * om;
    yr = (er * lam + ei * om) / d;
    yi = (ei * lam - er * om) / d;
  }
  for (int p = 0; p < np; ++p) {
    const double pt = n < mp.n0 ? mp.Pt[n + (int64_t)p * mp.n0] : 0.0;
    const double sr = wave_sum(pt * yr), si = wave_sum(pt * yi);
    if (lane == 0) {
      red[wave][p][0] = sr;
      red[wave][p][1] = si;
    }
  }
  __syncthreads();
  if (t < 2 * np) {
    const int p = t >> 1, q = t & 1;
    const double s = (red[0][p][q] + red[1][p][q]) + (red[2][p][q] + red[3][p][q]);
    mp.partial[((w * gridDim.x + blockIdx.x) * np + p) * 2 + q] = s;
  }
}

__global__ void phasor_finish_k(ModalPhasor mp, int64_t groups) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int np = mp.n_probe, m = mp.m;
  if (e >= mp.n_w * np) return;
  const int64_t w = e / np;
  const int p = (int)(e % np);
  double sr = 0.0, si = 0.0;
  for (int64_t g = 0; g < groups; ++g) {
    sr += mp.partial[((w * groups + g) * np + p) * 2];
    si += mp.partial[((w * groups + g) * np + p) * 2 + 1];
  }
  for (int a = 0; a < m; ++a) {
    const double pd = mp.PD[p + (int64_t)a * np];
    sr += pd * mp.amp_D[(w * m + a) * 2];
    si += pd * mp.amp_D[(w * m + a) * 2 + 1];
  }
  // times j w
  const double om = mp.omega[w];
  mp.out[e * 2] = -om * si;
  mp.out[e * 2 + 1] = om * sr;
}

}  // namespace

int64_t phasor_groups(int64_t n0) { return ceil_div(n0, NT); }

void modal_phasors(const ModalPhasor& mp, hipStream_t s) {
  if (mp.n_w <= 0) return;
  MM_REQUIRE(2 * mp.m + mp.n_src <= MAXF && mp.n_probe >= 1 && mp.n_probe <= MAXP, kInvalid,
             "modal_phasors: at most 8 forcing columns and 1..8 probes");
  MM_REQUIRE(mp.n_w < (int64_t)1 << 16, kInvalid, "modal_phasors: at most 65535 frequencies");
  const int64_t G = phasor_groups(mp.n0);
  hipLaunchKernelGGL(phasor_modes_k, dim3((unsigned)G, (unsigned)mp.n_w), dim3(NT), 0, s, mp);
  MM_HIP_TRY(hipGetLastError());
  const int64_t tot = mp.n_w * mp.n_probe;
  hipLaunchKernelGGL(phasor_finish_k, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, s, mp, G);
  MM_HIP_TRY(hipGetLastError());
}

}  // namespace mm
