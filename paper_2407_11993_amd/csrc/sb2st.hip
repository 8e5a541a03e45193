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
// The back-transform by these reflectors is in q2.hip.  Optionally a few
// columns Y (n x ny, ny <= 4 YQ) are taken along: every task applies its
// reflector to the rows R_k of Y, so Y leaves as Q2^T Y (two reflectors
// whose rows overlap are applied in the order they were generated, by the
// same argument as for the band).
#include "eig.h"

namespace mm {
namespace {

constexpr int NT = 256;
constexpr int YQ = 8;  // columns of Y per wave

// Wave-wide sum, every lane gets the result: sums over quads and rows of 16
// lanes by DPP moves (xor 1, xor 2, half-row mirror, row mirror), then the
// four row sums are read with readlane.
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
__device__ __forceinline__ double wsum(double v) {
  v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp<0x141>(v);  // row_half_mirror
  v += dpp<0x140>(v);  // row_mirror
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
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
// and the block below -- are staged in LDS as zero-padded 64 x 64 tiles with
// independent loads, updated there, and written back.  nb <= 64, so a block
// row or column fits one wave and the four waves split the other dimension;
// the zero padding lets every loop run a fixed 16 iterations, unrolled.
__global__ void __launch_bounds__(NT) sb2st_stage(Band B, int n, int nb, int stage, int s_lo,
                                                  const int64_t* off, double* V2,
                                                  double* tau2, double* Y, int64_t ldy,
                                                  int ny) {
  const int s = s_lo + (int)blockIdx.x;
  if (s > n - 3) return;
  const int k = stage - 3 * s;
  if (k < 0) return;
  const int Ks = (n - 2 - s + nb) / nb;  // ceil((n - 1 - s) / nb)
  if (k >= Ks) return;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t r0 = s + 1 + (int64_t)k * nb;
  const int len = (int)min((int64_t)nb, n - r0);
  const int64_t c0 = (k == 0) ? s : s + 1 + (int64_t)(k - 1) * nb;  // column to eliminate
  const int ncl = (int)(((k == 0) ? s + 1 : r0) - c0);                // left block columns
  const int64_t rn0 = r0 + len;
  const int lenn = (int)max((int64_t)0, min((int64_t)nb, n - rn0));
  const int64_t task = off[s] + k;
  // The diagonal block (D) and the block below (Bb, rows rn0.., columns r0..)
  // take only updates in which a thread reads and writes its own 16 entries
  // (row lane, columns wave + 4 q) and exchanges one row sum per wave through
  // p4: both stay in registers from load to store.  Only the left block,
  // whose update needs column sums, is staged in LDS.
  __shared__ double Lb[64][65];
  __shared__ double v[64], p4[4][64], w_s[64];
  __shared__ double s_tau, s_beta;
  double yv[YQ];  // rows R_k of Y (lane = row), columns wave + 4 q
  double rd[16];  // D(lane, wave + 4 q), zero outside the block
  double rb[16];  // Bb(lane, wave + 4 q), zero outside the block

  // ---- stage: all loads are issued before the first LDS store (addresses
  // clamped into the block, values selected)
  {
    const int li = min(lane, len - 1), lb = min(lane, max(lenn, 1) - 1);
#pragma unroll
    for (int q = 0; q < YQ; ++q) {
      const int c = wave + 4 * q;
      yv[q] = (c < ny) ? Y[(r0 + li) + c * ldy] : 0.0;
    }
    double rl[16];
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
      Lb[lane][j] = (lane < len && j < ncl) ? rl[q] : 0.0;
      if (!(lane < len && j < len)) rd[q] = 0.0;
      if (!(lane < lenn && j < len)) rb[q] = 0.0;
    }
  }
  __syncthreads();
  // ---- Householder reflector of the eliminated column Lb(:, 0) (wave 0)
  if (wave == 0) {
    const double x = Lb[lane][0];
    const double sig2 = wsum((lane >= 1) ? x * x : 0.0);
    const double a0 = lane_value(x, 0);
    double tv = 0.0, beta = a0, scale = 0.0;
    if (sig2 > 0.0) {
      beta = -copysign(sqrt(a0 * a0 + sig2), a0);
      tv = (beta - a0) / beta;
      scale = 1.0 / (a0 - beta);
    }
    const double vv = (lane == 0) ? 1.0 : x * scale;  // zero beyond len
    v[lane] = vv;
    if (lane == 0) {
      s_tau = tv;
      s_beta = beta;
    }
    if (V2) {  // kept for the back-transform (not when only Q2^T Y is wanted)
      if (lane < nb) store_dev(&V2[task * nb + lane], vv);
      if (lane == 0) store_dev(&tau2[task], tv);
    }
  }
  __syncthreads();
  const double tau = s_tau;
  if (tau == 0.0) return;  // H = I: nothing changes (uniform branch)
  const double vl = v[lane];
  // ---- Y(R_k, c) -= tau v (v^T Y(R_k, c)); v is zero past len
#pragma unroll
  for (int q = 0; q < YQ; ++q)
    if (wave + 4 * q < ny) yv[q] -= tau * vl * wsum(vl * yv[q]);

  // ---- left application: Lb(:, j) -= tau v (v^T Lb(:, j)), j >= 1; lane =
  //      column, each wave sums a quarter of the rows; the eliminated column
  //      becomes (beta, 0, ..., 0)
  if (ncl > 1) {
    const int i0 = 16 * wave;
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) acc += v[i0 + q] * Lb[i0 + q][lane];
    p4[wave][lane] = acc;
    __syncthreads();
    const double d = (lane >= 1) ? tau * ((p4[0][lane] + p4[1][lane]) + (p4[2][lane] + p4[3][lane]))
                                 : 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) Lb[i0 + q][lane] -= v[i0 + q] * d;
    __syncthreads();  // p4 is reused below
  }
  if (wave == 0) Lb[lane][0] = (lane == 0) ? s_beta : 0.0;
  // ---- two-sided on D: p = tau D v, w = p - tau/2 (p^T v) v, D -= v w^T + w v^T
  {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) acc += rd[q] * v[wave + 4 * q];
    p4[wave][lane] = acc;
  }
  __syncthreads();
  const double pl = tau * ((p4[0][lane] + p4[1][lane]) + (p4[2][lane] + p4[3][lane]));
  const double pv = wsum(pl * vl);
  const double wl = pl - 0.5 * tau * pv * vl;  // w for row `lane`
  __syncthreads();  // all reads of p4 above are done
  if (wave == 0) w_s[lane] = wl;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int j = wave + 4 * q;
    rd[q] -= vl * w_s[j] + wl * v[j];
  }
  // ---- right application to the block below: Bb -= tau (Bb v) v^T
  if (lenn > 0) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) acc += rb[q] * v[wave + 4 * q];
    p4[wave][lane] = acc;  // p4 was last read before the barriers above
    __syncthreads();
    const double tq = tau * ((p4[0][lane] + p4[1][lane]) + (p4[2][lane] + p4[3][lane]));
#pragma unroll
    for (int q = 0; q < 16; ++q) rb[q] -= tq * v[wave + 4 * q];
  }
  __syncthreads();
  // ---- write back: read every value first, then store (written through:
  //      the next stage reads these blocks, on whichever XCD its tasks run)
  {
    double rl[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int j = wave + 4 * q;
      rl[q] = Lb[lane][j];
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int j = wave + 4 * q;
      if (lane < len && j < ncl) store_dev(&B.at(r0 + lane, c0 + j), rl[q]);
      if (lane < len && j <= lane) store_dev(&B.at(r0 + lane, r0 + j), rd[q]);
      if (lane < lenn && j < len) store_dev(&B.at(rn0 + lane, r0 + j), rb[q]);
    }
#pragma unroll
    for (int q = 0; q < YQ; ++q) {
      const int c = wave + 4 * q;
      if (c < ny && lane < len) store_dev(&Y[(r0 + lane) + c * ldy], yv[q]);
    }
  }
}

__global__ void band_to_tridiag(const double* AB, int64_t ld, int64_t n, double* d, double* e) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  d[j] = AB[j * ld];
  if (j + 1 < n) e[j] = AB[1 + j * ld];
}

}  // namespace

int sb2st_max_cols() { return 4 * YQ; }

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
           double* V2, double* tau2, double* d, double* e, hipStream_t s, double* Y,
           int64_t ldy, int ny) {
  const int64_t n = plan.n;
  const int nb = plan.nb;
  MM_REQUIRE(nb >= 1 && nb <= 64 && ldab >= 2 * nb + 1, kInvalid, "sb2st: band must be 1..64");
  MM_REQUIRE(ny >= 0 && ny <= sb2st_max_cols() && (ny == 0 || (Y && ldy >= n)), kInvalid,
             "sb2st: at most 32 columns carried along");
  MM_REQUIRE(n < (int64_t)1 << 29, kInvalid, "sb2st: order too large");
  if (n >= 3) {
    const int64_t K0 = ceil_div(n - 1, nb);
    const int64_t last_stage = 3 * (n - 3) + ceil_div(n - 1 - (n - 3), nb) - 1;
    Band B{AB, ldab};
    for (int64_t st = 0; st <= std::max(last_stage, K0 - 1); ++st) {
      // s with 0 <= st - 3s < K_s <= K0
      int64_t s_lo = st - (K0 - 1) <= 0 ? 0 : ceil_div(st - (K0 - 1), 3);
      int64_t s_hi = std::min(st / 3, n - 3);
      if (s_hi < s_lo) continue;
      hipLaunchKernelGGL(sb2st_stage, dim3((unsigned)(s_hi - s_lo + 1)), dim3(NT), 0, s, B,
                         (int)n, nb, (int)st, (int)s_lo, d_offset, V2, tau2, Y, ldy, ny);
    }
    MM_HIP_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(band_to_tridiag, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, AB,
                     ldab, n, d, e);
  MM_HIP_TRY(hipGetLastError());
}

}  // namespace mm
