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
// there, and written back.  nb <= 64, so a block row or column fits one
// wave: the four waves split the other dimension.
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
  const int64_t task = off[s] + k;
  __shared__ double Lb[64][65], Db[64][65], Bb[64][65];
  __shared__ double v[64], p4[4][64], w_s[64];
  __shared__ double s_tau, s_beta;

  // ---- stage: every thread issues all of its loads before the first LDS
  // store (addresses are clamped into the block, the value is selected), so
  // the three blocks arrive in one memory latency
  {
    const int li = min(lane, len - 1), lb = min(lane, max(lenn, 1) - 1);
    double rl[16], rd[16], rb[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int j = wave + 4 * q;
      rl[q] = B.at(r0 + li, c0 + min(j, ncl - 1));
      const int jd = min(j, len - 1);
      rd[q] = B.sym(r0 + li, r0 + jd);
      rb[q] = (lenn > 0) ? B.at(rn0 + lb, r0 + jd) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int j = wave + 4 * q;
      if (lane < len && j < ncl) Lb[lane][j] = rl[q];
      if (lane < len && j < len) Db[lane][j] = rd[q];
      if (lane < lenn && j < len) Bb[lane][j] = rb[q];
    }
  }
  __syncthreads();
  // ---- Householder reflector of the eliminated column Lb(:, 0) (wave 0)
  if (wave == 0) {
    const double x = (lane < len) ? Lb[lane][0] : 0.0;
    const double sig2 = wsum((lane >= 1) ? x * x : 0.0);
    const double a0 = __shfl(x, 0, 64);
    double tv = 0.0, beta = a0, scale = 0.0;
    if (sig2 > 0.0) {
      beta = -copysign(sqrt(a0 * a0 + sig2), a0);
      tv = (beta - a0) / beta;
      scale = 1.0 / (a0 - beta);
    }
    v[lane] = (lane == 0) ? 1.0 : ((lane < len) ? x * scale : 0.0);
    if (lane == 0) {
      s_tau = tv;
      s_beta = beta;
    }
    if (lane < nb) V2[task * nb + lane] = (lane < len) ? v[lane] : 0.0;
    if (lane == 0) tau2[task] = tv;
  }
  __syncthreads();
  const double tau = s_tau;
  if (tau == 0.0) return;  // H = I: nothing changes (uniform branch)
  const double vl = v[lane];

  // ---- left application: Lb(:, j) -= tau v (v^T Lb(:, j)), j >= 1; lane =
  //      column, each wave sums a quarter of the rows; the eliminated column
  //      becomes (beta, 0, ..., 0)
  if (ncl > 1) {
    const int i0 = 16 * wave, i1 = min(i0 + 16, len);
    double acc = 0.0;
    if (lane < ncl)
      for (int i = i0; i < i1; ++i) acc += v[i] * Lb[i][lane];
    p4[wave][lane] = acc;
    __syncthreads();
    const double d = (p4[0][lane] + p4[1][lane]) + (p4[2][lane] + p4[3][lane]);
    if (lane >= 1 && lane < ncl)
      for (int i = i0; i < i1; ++i) Lb[i][lane] -= tau * v[i] * d;
    __syncthreads();  // p4 is reused below
  }
  if (wave == 0 && lane < len) Lb[lane][0] = (lane == 0) ? s_beta : 0.0;
  // ---- two-sided on D: p = tau D v, w = p - tau/2 (p^T v) v, D -= v w^T + w v^T
  {
    double acc = 0.0;
    if (lane < len)
      for (int j = wave; j < len; j += 4) acc += Db[lane][j] * v[j];
    p4[wave][lane] = acc;
  }
  __syncthreads();
  const double pl = (lane < len) ? tau * ((p4[0][lane] + p4[1][lane]) + (p4[2][lane] + p4[3][lane]))
                                 : 0.0;
  const double pv = wsum(pl * vl);
  const double wl = pl - 0.5 * tau * pv * vl;  // w for row `lane`
  // every wave needs w_j for its columns j: publish w in LDS
  __syncthreads();  // all reads of p4 above are done
  if (wave == 0) w_s[lane] = wl;
  __syncthreads();
  for (int j = wave; j < len; j += 4)
    if (lane < len && lane >= j) Db[lane][j] -= vl * w_s[j] + wl * v[j];
  // ---- right application to the block below: Bb -= tau (Bb v) v^T
  if (lenn > 0) {
    double acc = 0.0;
    if (lane < lenn)
      for (int j = wave; j < len; j += 4) acc += Bb[lane][j] * v[j];
    p4[wave][lane] = acc;  // p4 was last read before the barrier above
    __syncthreads();
    const double q = (lane < lenn) ? (p4[0][lane] + p4[1][lane]) + (p4[2][lane] + p4[3][lane])
                                   : 0.0;
    for (int j = wave; j < len; j += 4)
      if (lane < lenn) Bb[lane][j] -= tau * q * v[j];
  }
  __syncthreads();
  // ---- write back
  for (int j = wave; j < ncl; j += 4)
    if (lane < len) B.at(r0 + lane, c0 + j) = Lb[lane][j];
  for (int j = wave; j < len; j += 4)
    if (lane < len && lane >= j) B.at(r0 + lane, r0 + j) = Db[lane][j];
  for (int j = wave; j < len; j += 4)
    if (lane < lenn) B.at(rn0 + lane, r0 + j) = Bb[lane][j];
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
