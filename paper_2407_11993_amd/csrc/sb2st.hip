// Stage 2 of the two-stage tridiagonalisation: bulge chasing B = Q2 T Q2^T.
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
// The back-transform by these reflectors is in q2.hip.
#include "eig.h"

namespace mm {
namespace {

constexpr int NT = 256;

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

// One task (s, k).  The three blocks it touches -- the block left of the
// diagonal block (its first column is the one eliminated), the diagonal block
// and the block below -- are staged in LDS with independent loads, updated
// there, and written back.  nb <= 64.
__global__ void __launch_bounds__(NT) sb2st_stage(Band B, int64_t n, int nb, int64_t stage,
                                                  int64_t s_lo, const int64_t* off,
                                                  double* V2, double* tau2) {
  const int64_t s = s_lo + blockIdx.x;
  if (s > n - 3) return;
  const int64_t k = stage - 3 * s;
  if (k < 0) return;
  const int64_t Ks = ceil_div(n - 1 - s, nb);
  if (k >= Ks) return;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t r0 = s + 1 + k * nb;
  const int len = (int)min((int64_t)nb, n - r0);
  const int64_t c0 = (k == 0) ? s : s + 1 + (k - 1) * nb;  // column to eliminate
  const int ncl = (int)(((k == 0) ? s + 1 : r0) - c0);       // left block columns
  const int64_t rn0 = r0 + len;
  const int lenn = (int)max((int64_t)0, min((int64_t)nb, n - rn0));
  __shared__ double Lb[64][65], Db[64][65], Bb[64][65];
  __shared__ double v[64], p[64], w[64], sh[8];
  __shared__ double s_tau, s_beta, s_scale;

  // ---- stage (column-major walks: consecutive threads, consecutive rows)
  for (int e = t; e < len * ncl; e += NT) {
    const int i = e % len, j = e / len;
    Lb[i][j] = B.at(r0 + i, c0 + j);
  }
  for (int e = t; e < len * len; e += NT) {
    const int i = e % len, j = e / len;
    if (i >= j) {
      const double a = B.at(r0 + i, r0 + j);
      Db[i][j] = a;
      Db[j][i] = a;
    }
  }
  for (int e = t; e < lenn * len; e += NT) {
    const int i = e % lenn, j = e / lenn;
    Bb[i][j] = B.at(rn0 + i, r0 + j);
  }
  __syncthreads();
  // ---- Householder reflector of the eliminated column Lb(:, 0)
  {
    double x = (t >= 1 && t < len) ? Lb[t][0] : 0.0;
    x = wsum(x * x);
    if (lane == 0) sh[wave] = x;
  }
  __syncthreads();
  if (t == 0) {
    const double a0 = Lb[0][0];
    const double sig2 = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    double tv = 0.0, beta = a0, scale = 0.0;
    if (sig2 > 0.0) {
      beta = -copysign(sqrt(a0 * a0 + sig2), a0);
      tv = (beta - a0) / beta;
      scale = 1.0 / (a0 - beta);
    }
    s_tau = tv;
    s_beta = beta;
    s_scale = scale;
  }
  __syncthreads();
  const double tau = s_tau;
  if (t < 64) v[t] = (t == 0) ? 1.0 : ((t < len) ? Lb[t][0] * s_scale : 0.0);
  __syncthreads();
  const int64_t task = off[s] + k;
  if (t < nb) V2[task * nb + t] = (t < len) ? v[t] : 0.0;
  if (t == 0) tau2[task] = tau;
  if (tau == 0.0) return;  // H = I: nothing changes (uniform branch)

  // ---- left application: Lb(:, j) -= tau v (v^T Lb(:, j)), j >= 1;
  //      the eliminated column becomes (beta, 0, ..., 0)
  {
    const int j = t >> 2, part = t & 3;  // 4 threads per column, 16 rows each
    if (j >= 1 && j < ncl) {
      double d = 0.0;
      for (int i = part; i < len; i += 4) d += v[i] * Lb[i][j];
      d += __shfl_xor(d, 1, 64);
      d += __shfl_xor(d, 2, 64);
      const double f = tau * d;
      for (int i = part; i < len; i += 4) Lb[i][j] -= f * v[i];
    }
    if (t < len) Lb[t][0] = (t == 0) ? s_beta : 0.0;
  }
  // ---- two-sided on D: p = tau D v, w = p - tau/2 (p^T v) v, D -= v w^T + w v^T
  {
    const int i = t >> 2, part = t & 3;
    double acc = 0.0;
    if (i < len)
      for (int j = part; j < len; j += 4) acc += Db[i][j] * v[j];
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    if (part == 0 && i < 64) p[i] = (i < len) ? tau * acc : 0.0;
  }
  __syncthreads();
  {
    double x = (t < len) ? p[t] * v[t] : 0.0;
    x = wsum(x);
    if (lane == 0) sh[4 + wave] = x;
  }
  __syncthreads();
  {
    const double pv = (sh[4] + sh[5]) + (sh[6] + sh[7]);
    if (t < 64) w[t] = (t < len) ? p[t] - 0.5 * tau * pv * v[t] : 0.0;
  }
  __syncthreads();
  for (int e = t; e < len * len; e += NT) {
    const int i = e % len, j = e / len;
    if (i >= j) Db[i][j] -= v[i] * w[j] + w[i] * v[j];
  }
  // ---- right application to the block below: Bb -= tau (Bb v) v^T
  if (lenn > 0) {
    const int i = t >> 2, part = t & 3;
    double acc = 0.0;
    if (i < lenn)
      for (int j = part; j < len; j += 4) acc += Bb[i][j] * v[j];
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    const double f = tau * acc;
    if (i < lenn)
      for (int j = part; j < len; j += 4) Bb[i][j] -= f * v[j];
  }
  __syncthreads();
  // ---- write back
  for (int e = t; e < len * ncl; e += NT) {
    const int i = e % len, j = e / len;
    B.at(r0 + i, c0 + j) = Lb[i][j];
  }
  for (int e = t; e < len * len; e += NT) {
    const int i = e % len, j = e / len;
    if (i >= j) B.at(r0 + i, r0 + j) = Db[i][j];
  }
  for (int e = t; e < lenn * len; e += NT) {
    const int i = e % lenn, j = e / lenn;
    B.at(rn0 + i, r0 + j) = Bb[i][j];
  }
}

__global__ void band_to_tridiag(const double* AB, int64_t ld, int64_t n, double* d, double* e) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  d[j] = AB[j * ld];
  if (j + 1 < n) e[j] = AB[1 + j * ld];
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
  MM_REQUIRE(nb >= 1 && nb <= 64 && ldab >= 2 * nb + 1, kInvalid, "sb2st: band must be 1..64");
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

}  // namespace mm
