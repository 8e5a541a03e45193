// Stage 2 of the two-stage tridiagonalisation: bulge chasing B = Q2 T Q2^T,
// and the two back-transforms Q = Q1 (Q2 Z).
//
// Band storage: AB(d, j) = B(j + d, j), 0 <= d <= 2 nb (the rows beyond nb
// hold the bulge).  Sweep s annihilates column s below the subdiagonal; its
// task k works on the row block R_k = [s+1+k nb, s+1+(k+1) nb):
//   * a Householder reflector H_{s,k} of length |R_k| maps the column it
//     eliminates (column s for k = 0, the first column of the bulge left by
//     task k-1 otherwise) onto its first entry,
//   * H is applied from the left to the block left of the diagonal block,
//     two-sided to the diagonal block R_k x R_k, and from the right to the
//     block below (which creates the next bulge).
// Tasks (s, k) with the same 3s + k touch disjoint windows of the band, and
// every task a task depends on has a smaller 3s + k, so one launch per value
// of 3s + k runs all of its tasks concurrently.
//
// Q2 = H_{0,0} H_{0,1} ... H_{1,0} ... in generation order, so Q2 Z applies
// them last-first.  Groups of 64 consecutive sweeps are applied together
// (group g descending, then k ascending, then s descending inside the
// group): every pair of reflectors whose order this changes acts on disjoint
// rows and therefore commutes.  A workgroup owns 64 columns of Z and keeps
// the group's row window in LDS while applying its reflectors.
#include "eig.h"

namespace mm {
namespace {

constexpr int NT = 256;
constexpr int GS = 64;       // sweeps per back-transform group
constexpr int ZC = 64;       // Z columns per workgroup in apply_q2
constexpr int WIN = 128;     // max window rows (nb + GS - 1)

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-wide sum (NT threads); every thread gets the result.
__device__ double block_sum(double v, double* sh) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  v = wsum(v);
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

struct Band {
  double* AB;
  int64_t ld;
  __device__ double& at(int64_t r, int64_t c) const { return AB[(r - c) + c * ld]; }  // r >= c
  __device__ double sym(int64_t r, int64_t c) const {
    return r >= c ? AB[(r - c) + c * ld] : AB[(c - r) + r * ld];
  }
};

__global__ void __launch_bounds__(NT) sb2st_stage(Band B, int64_t n, int nb, int64_t stage,
                                                  int64_t s_lo, const int64_t* off,
                                                  double* V2, double* tau2) {
  const int64_t s = s_lo + blockIdx.x;
  if (s > n - 3) return;
  const int64_t k = stage - 3 * s;
  if (k < 0) return;
  const int64_t Ks = ceil_div(n - 1 - s, nb);
  if (k >= Ks) return;
  const int t = threadIdx.x;
  const int64_t r0 = s + 1 + k * nb;
  const int len = (int)min((int64_t)nb, n - r0);
  const int64_t c0 = (k == 0) ? s : s + 1 + (k - 1) * nb;  // column to eliminate
  const int64_t cend = (k == 0) ? s + 1 : r0;              // left block columns [c0, cend)
  const int64_t rn0 = r0 + len;
  const int lenn = (int)max((int64_t)0, min((int64_t)nb, n - rn0));
  __shared__ double v[128], p[128], q[128], sh[8];
  __shared__ double s_tau, s_beta;

  if (t < len) v[t] = B.at(r0 + t, c0);
  __syncthreads();
  const double a0 = v[0];
  const double sig2 = block_sum((t >= 1 && t < len) ? v[t] * v[t] : 0.0, sh);
  if (t == 0) {
    double tv = 0.0, beta = a0;
    if (sig2 > 0.0) {
      beta = -copysign(sqrt(a0 * a0 + sig2), a0);
      tv = (beta - a0) / beta;
    }
    s_tau = tv;
    s_beta = beta;
  }
  __syncthreads();
  const double tau = s_tau;
  if (tau != 0.0 && t < len) v[t] = (t == 0) ? 1.0 : v[t] / (a0 - s_beta);
  if (tau == 0.0 && t < len) v[t] = (t == 0) ? 1.0 : 0.0;
  __syncthreads();
  // store the reflector
  const int64_t task = off[s] + k;
  if (t < nb) V2[task * nb + t] = (t < len) ? v[t] : 0.0;
  if (t == 0) tau2[task] = tau;
  if (tau == 0.0) return;

  // eliminated column: (beta, 0, ..., 0)
  if (t < len) B.at(r0 + t, c0) = (t == 0) ? s_beta : 0.0;
  // left application to the columns c0+1 .. cend-1 (k >= 1):
  //   A(R, c) -= tau v (v^T A(R, c))
  {
    const int lane = t & 63, wave = t >> 6;
    for (int64_t c = c0 + 1 + wave; c < cend; c += NT / 64) {
      double d = 0.0;
      for (int i = lane; i < len; i += 64) d += v[i] * B.at(r0 + i, c);
      d = wsum(d);
      for (int i = lane; i < len; i += 64) B.at(r0 + i, c) -= tau * v[i] * d;
    }
  }
  __syncthreads();
  // two-sided on D = A(R, R): p = tau D v, w = p - tau/2 (p^T v) v,
  // D -= v w^T + w v^T (lower triangle)
  {
    const int i = t & 127, h = t >> 7;
    double acc = 0.0;
    if (i < len)
      for (int j = h; j < len; j += 2) acc += B.sym(r0 + i, r0 + j) * v[j];
    q[t & 127] = 0.0;
    __syncthreads();
    if (h == 0 && i < len) p[i] = acc;
    __syncthreads();
    if (h == 1 && i < len) p[i] += acc;
    __syncthreads();
    if (t < len) p[t] *= tau;
    __syncthreads();
    const double pv = block_sum(t < len ? p[t] * v[t] : 0.0, sh);
    if (t < len) q[t] = p[t] - 0.5 * tau * pv * v[t];  // q = w
    __syncthreads();
    for (int e = t; e < len * len; e += NT) {
      const int ii = e % len, jj = e / len;
      if (ii >= jj) B.at(r0 + ii, r0 + jj) -= v[ii] * q[jj] + q[ii] * v[jj];
    }
  }
  __syncthreads();
  // right application to the block below: A(Rn, R) -= tau (A(Rn, R) v) v^T
  if (lenn > 0) {
    const int i = t & 127, h = t >> 7;
    double acc = 0.0;
    if (i < lenn)
      for (int j = h; j < len; j += 2) acc += B.at(rn0 + i, r0 + j) * v[j];
    if (h == 0 && i < lenn) p[i] = acc;
    __syncthreads();
    if (h == 1 && i < lenn) p[i] += acc;
    __syncthreads();
    for (int e = t; e < lenn * len; e += NT) {
      const int ii = e % lenn, jj = e / lenn;
      B.at(rn0 + ii, r0 + jj) -= tau * p[ii] * v[jj];
    }
  }
}

__global__ void band_to_tridiag(const double* AB, int64_t ld, int64_t n, double* d, double* e) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  d[j] = AB[j * ld];
  if (j + 1 < n) e[j] = AB[1 + j * ld];
}

// Z <- (group of sweeps [sa, sb)) applied to Z rows, all k, for 64 columns.
// Lane layout: column cz = wave*16 + lane/4, rows i == (lane & 3) mod 4.
__global__ void __launch_bounds__(NT) apply_q2_group(int64_t n, int nb, int64_t sa, int64_t sb,
                                                     const int64_t* off, const double* V2,
                                                     const double* tau2, double* Z, int64_t ldz,
                                                     int64_t ncols) {
  __shared__ double Zw[WIN][ZC + 1];
  __shared__ double Vs[GS][128];
  __shared__ double Ts[GS];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t col0 = (int64_t)blockIdx.x * ZC;
  const int cz = wave * 16 + (lane >> 2);
  const int quarter = lane & 3;
  const int64_t sl = min(sb, n - 2);  // sweeps beyond n-3 have no tasks
  if (sa >= sl) return;
  const int64_t kmax = ceil_div(n - 1 - sa, nb);
  for (int64_t k = 0; k < kmax; ++k) {
    const int64_t wlo = sa + 1 + k * nb;
    if (wlo >= n) break;
    const int64_t whi = min(sl + k * nb + nb, n);  // last sweep sl-1: rows up to sl + (k+1) nb
    const int wlen = (int)(whi - wlo);
    // load window and reflectors
    for (int e = t; e < wlen * ZC; e += NT) {
      const int r = e % wlen, c = e / wlen;
      Zw[r][c] = (col0 + c < ncols) ? Z[(wlo + r) + (col0 + c) * ldz] : 0.0;
    }
    for (int e = t; e < GS * nb; e += NT) {
      const int gs = e / nb, i = e % nb;
      const int64_t s = sa + gs;
      double val = 0.0;
      if (s < sl && k < ceil_div(n - 1 - s, nb)) val = V2[(off[s] + k) * nb + i];
      Vs[gs][i] = val;
    }
    for (int gs = t; gs < GS; gs += NT) {
      const int64_t s = sa + gs;
      Ts[gs] = (s < sl && k < ceil_div(n - 1 - s, nb)) ? tau2[off[s] + k] : 0.0;
    }
    __syncthreads();
    for (int64_t s = sl - 1; s >= sa; --s) {
      const int gs = (int)(s - sa);
      const double tau = Ts[gs];
      if (tau == 0.0) continue;
      const int64_t r0 = s + 1 + k * nb;
      if (r0 >= n) continue;
      const int len = (int)min((int64_t)nb, n - r0);
      const int ro = (int)(r0 - wlo);
      double d = 0.0;
      for (int i = quarter; i < len; i += 4) d += Vs[gs][i] * Zw[ro + i][cz];
      d += __shfl_xor(d, 1, 64);
      d += __shfl_xor(d, 2, 64);
      const double f = tau * d;
      for (int i = quarter; i < len; i += 4) Zw[ro + i][cz] -= f * Vs[gs][i];
    }
    __syncthreads();
    for (int e = t; e < wlen * ZC; e += NT) {
      const int r = e % wlen, c = e / wlen;
      if (col0 + c < ncols) Z[(wlo + r) + (col0 + c) * ldz] = Zw[r][c];
    }
    __syncthreads();
  }
}

}  // namespace

Sb2stPlan sb2st_plan(int64_t n, int nb) {
  Sb2stPlan p;
  p.n = n;
  p.nb = nb;
  p.offset.assign(n + 1, 0);
  int64_t acc = 0;
  for (int64_t s = 0; s < n; ++s) {
    p.offset[s] = acc;
    if (s <= n - 3) acc += ceil_div(n - 1 - s, nb);
  }
  p.offset[n] = acc;
  p.tasks = acc;
  return p;
}

void sb2st(double* AB, int64_t ldab, const Sb2stPlan& plan, const int64_t* d_offset,
           double* V2, double* tau2, double* d, double* e, hipStream_t s) {
  const int64_t n = plan.n;
  const int nb = plan.nb;
  MM_REQUIRE(nb >= 1 && nb <= 128 && ldab >= 2 * nb + 1, kInvalid, "sb2st: bad band");
  if (n >= 3) {
    const int64_t K0 = ceil_div(n - 1, nb);
    const int64_t last_stage = 3 * (n - 3) + ceil_div(n - 1 - (n - 3), nb) - 1;
    Band B{AB, ldab};
    for (int64_t st = 0; st <= std::max(last_stage, K0 - 1); ++st) {
      // s with 0 <= st - 3s < K_s <= K0
      int64_t s_lo = st - (K0 - 1) <= 0 ? 0 : ceil_div(st - (K0 - 1), 3);
      int64_t s_hi = std::min(st / 3, n - 3);
      if (s_hi < s_lo) continue;
      hipLaunchKernelGGL(sb2st_stage, dim3((unsigned)(s_hi - s_lo + 1)), dim3(NT), 0, s, B, n,
                         nb, st, s_lo, d_offset, V2, tau2);
    }
    MM_HIP_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(band_to_tridiag, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, AB,
                     ldab, n, d, e);
  MM_HIP_TRY(hipGetLastError());
}

void apply_q2(const Sb2stPlan& plan, const int64_t* d_offset, const double* V2,
              const double* tau2, double* Z, int64_t ldz, int64_t ncols, hipStream_t s) {
  const int64_t n = plan.n;
  const int nb = plan.nb;
  MM_REQUIRE(nb + GS - 1 <= WIN, kInvalid, "apply_q2: band too wide");
  if (n < 3 || ncols <= 0) return;
  const int64_t nsweeps = n - 2;  // sweeps 0..n-3
  const int64_t ngroups = ceil_div(nsweeps, GS);
  const unsigned grid = (unsigned)ceil_div(ncols, ZC);
  for (int64_t g = ngroups - 1; g >= 0; --g) {
    const int64_t sa = g * GS, sb = std::min(sa + GS, nsweeps);
    hipLaunchKernelGGL(apply_q2_group, dim3(grid), dim3(NT), 0, s, n, nb, sa, sb, d_offset,
                       V2, tau2, Z, ldz, ncols);
  }
  MM_HIP_TRY(hipGetLastError());
}

}  // namespace mm
