// Adjoint of the probe-signal misfit over runs that share one waveform,
// evaluated in the modal basis (the modal recursion of Sec. 3.3.2 run
// backward).
//
// The modal theta-method is the theta-method of Sec. 3.3.1 seen through the
// congruence V = G^{-T} Q (V^T L V = I, V^T R V = Lam), so the adjoint of the
// physical recursion
//     Z dI_k = -dt R I_k + M_c u_k,  Z = L + theta dt R,  u_k = -(i_{k+1} - i_k)
//     J = sum_c sum_k (P_c^T dI_k / dt - obs_c[k])^2
// is exact in modal coordinates, where Z^{-1} = V (I + theta dt Lam)^{-1} V^T:
//     l_k = (r_k w_c - dt Lam nu_k) / (1 + theta dt Lam),  nu_{k-1} = nu_k + l_k,
//     r_k = 2 (s_c[k] - obs_c[k]) / dt  (the probe weights of run c enter s),
//     dJ/du_k = sum_c w_c^T l_k,   dJ/dR = -V S V^T,
//     S = sum_{c,k} l_k zeta_k^T,  zeta_k = dt (theta dy_k + y_k).
// Memory stays bounded at long horizons: the forward pass keeps y every K
// steps; the backward pass walks the K-step segments last first, recomputes
// the segment's zeta from its checkpoint, runs the recursion over it and
// adds the segment's  L Z^T  to S on the matrix cores.
#include "kernels.h"

namespace mm {
namespace {

constexpr int NT = 256;
constexpr int MPT = 4;    // modes per thread
constexpr int SB = 8;     // steps per reduction block

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
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp<0xB1>(v);
  v += dpp<0x4E>(v);
  v += dpp<0x141>(v);
  v += dpp<0x140>(v);
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

struct Modes {
  double c[MPT], a[MPT], w[MPT], p[MPT];
};

__device__ __forceinline__ void load_modes(const AdjointStep& s, int r, int g, int t,
                                           Modes& m) {
  const double* Wc = s.W + (int64_t)s.wcol[r] * s.ldw;
  const double* Pc = s.Pm + (int64_t)s.pcol[r] * s.n0;
#pragma unroll
  for (int i = 0; i < MPT; ++i) {
    const int64_t n = (int64_t)g * NT * MPT + (int64_t)i * NT + t;
    m.c[i] = m.a[i] = m.w[i] = m.p[i] = 0.0;
    if (n < s.n0) {
      const double lam = s.lam[n];
      m.a[i] = s.dt * lam;
      m.c[i] = 1.0 / (1.0 + s.theta * s.dt * lam);
      m.w[i] = Wc[n];
      m.p[i] = Pc[n];
    }
  }
}

// Partial sums of SB steps: one value per (step, workgroup), written by the
// first SB threads (fixed order over the waves).
__device__ __forceinline__ void block_partials(double (&acc)[SB], double (*red)[SB][NT / 64],
                                               int buf, double* out, int64_t stride,
                                               int64_t k0, int64_t kend, int dir) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
#pragma unroll
  for (int q = 0; q < SB; ++q) {
    const double v = wave_sum(acc[q]);
    if (lane == 0) red[buf][q][wave] = v;
  }
  __syncthreads();
  if (t < SB) {
    const int64_t k = k0 + dir * t;
    if (dir > 0 ? k < kend : k >= kend)
      out[k * stride] = (red[buf][t][0] + red[buf][t][1]) + (red[buf][t][2] + red[buf][t][3]);
  }
}

// Forward: all steps of run r; y saved every K steps (before step k, k % K
// == 0); signal partials per (step, group).
__global__ void __launch_bounds__(NT) adj_forward_k(AdjointStep s) {
  __shared__ double red[2][SB][NT / 64];
  const int t = threadIdx.x, g = blockIdx.x, r = blockIdx.y;
  Modes m;
  load_modes(s, r, g, t, m);
  double y[MPT];
#pragma unroll
  for (int i = 0; i < MPT; ++i) y[i] = 0.0;
  const int64_t T = s.T, K = s.K, n0 = s.n0;
  double* part = s.part_sig + (int64_t)r * T * s.G + g;
  for (int64_t k0 = 0, it = 0; k0 < T; k0 += SB, ++it) {
    double acc[SB];
#pragma unroll
    for (int q = 0; q < SB; ++q) {
      acc[q] = 0.0;
      const int64_t k = k0 + q;
      if (k < T) {
        if (k % K == 0) {
          double* ck = s.ckpt + ((int64_t)r * s.n_ckpt + k / K) * n0;
#pragma unroll
          for (int i = 0; i < MPT; ++i) {
            const int64_t n = (int64_t)g * NT * MPT + (int64_t)i * NT + t;
            if (n < n0) ck[n] = y[i];
          }
        }
        const double u = -(s.wave[k + 1] - s.wave[k]);
#pragma unroll
        for (int i = 0; i < MPT; ++i) {
          const double dy = m.c[i] * (m.w[i] * u - m.a[i] * y[i]);
          y[i] += dy;
          acc[q] += m.p[i] * dy;
        }
      }
    }
    block_partials(acc, red, (int)(it & 1), part, s.G, k0, T, +1);
  }
}

// Recompute zeta_k = dt (theta dy_k + y_k) over segment [k0, k1) of run r
// from its checkpoint; zeta is stored column-major n0 x (runs * K), column
// r * K + (k - k0).
__global__ void __launch_bounds__(NT) adj_recompute_k(AdjointStep s, int64_t k0, int64_t k1,
                                                      double* Zb) {
  const int t = threadIdx.x, g = blockIdx.x, r = blockIdx.y;
  Modes m;
  load_modes(s, r, g, t, m);
  const int64_t n0 = s.n0;
  const double* ck = s.ckpt + ((int64_t)r * s.n_ckpt + k0 / s.K) * n0;
  double y[MPT];
  int64_t nidx[MPT];
#pragma unroll
  for (int i = 0; i < MPT; ++i) {
    nidx[i] = (int64_t)g * NT * MPT + (int64_t)i * NT + t;
    y[i] = nidx[i] < n0 ? ck[nidx[i]] : 0.0;
  }
  for (int64_t k = k0; k < k1; ++k) {
    const double u = -(s.wave[k + 1] - s.wave[k]);
    double* col = Zb + ((int64_t)r * s.K + (k - k0)) * n0;
#pragma unroll
    for (int i = 0; i < MPT; ++i) {
      const double dy = m.c[i] * (m.w[i] * u - m.a[i] * y[i]);
      if (nidx[i] < n0) col[nidx[i]] = s.dt * (s.theta * dy + y[i]);
      y[i] += dy;
    }
  }
}

// Backward over segment [k0, k1) of run r, last step first:
// l_k = c (r_k w - a nu), nu += l_k; l_k stored like zeta; partial sums of
// w^T l_k per (step, group).  nu (n0 per run) carries over the segments.
__global__ void __launch_bounds__(NT) adj_backward_k(AdjointStep s, int64_t k0, int64_t k1,
                                                     double* Lb) {
  __shared__ double red[2][SB][NT / 64];
  const int t = threadIdx.x, g = blockIdx.x, r = blockIdx.y;
  Modes m;
  load_modes(s, r, g, t, m);
  const int64_t n0 = s.n0;
  double* nu_r = s.nu + (int64_t)r * n0;
  double nu[MPT];
  int64_t nidx[MPT];
#pragma unroll
  for (int i = 0; i < MPT; ++i) {
    nidx[i] = (int64_t)g * NT * MPT + (int64_t)i * NT + t;
    nu[i] = nidx[i] < n0 ? nu_r[nidx[i]] : 0.0;
  }
  const double* res = s.resid + (int64_t)r * s.T;
  double* part = s.part_u + (int64_t)r * s.T * s.G + g;
  for (int64_t kb = k1 - 1, it = 0; kb >= k0; kb -= SB, ++it) {
    double acc[SB];
#pragma unroll
    for (int q = 0; q < SB; ++q) {
      acc[q] = 0.0;
      const int64_t k = kb - q;
      if (k >= k0) {
        const double rk = res[k];
        double* col = Lb + ((int64_t)r * s.K + (k - k0)) * n0;
#pragma unroll
        for (int i = 0; i < MPT; ++i) {
          const double l = m.c[i] * (rk * m.w[i] - m.a[i] * nu[i]);
          if (nidx[i] < n0) col[nidx[i]] = l;
          nu[i] += l;
          acc[q] += m.w[i] * l;
        }
      }
    }
    block_partials(acc, red, (int)(it & 1), part, s.G, kb, k0, -1);
  }
#pragma unroll
  for (int i = 0; i < MPT; ++i)
    if (nidx[i] < n0) nu_r[nidx[i]] = nu[i];
}

// resid[e] = 2 (s - obs) / dt with s = sum_g part_sig[e G + g] / dt;
// sq[e] = (s - obs)^2.
__global__ void adj_resid_k(const double* part_sig, int64_t total, int G, double dt,
                            const double* obs, double* resid, double* sq) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  double s = 0.0;
  for (int g = 0; g < G; ++g) s += part_sig[e * G + g];
  const double d = s / dt - obs[e];
  resid[e] = 2.0 * d / dt;
  sq[e] = d * d;
}

// J = sum of sq in a fixed order (one workgroup).
__global__ void __launch_bounds__(NT) adj_sum_k(const double* sq, int64_t total, double* J) {
  __shared__ double red[NT / 64];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  double s = 0.0;
  for (int64_t e = t; e < total; e += NT) s += sq[e];
  s = wave_sum(s);
  if (lane == 0) red[wave] = s;
  __syncthreads();
  if (t == 0) *J = (red[0] + red[1]) + (red[2] + red[3]);
}

// dJ/du_k = sum_r sum_g part_u[(r T + k) G + g];  dJ/di_j = dJ/du_j - dJ/du_{j-1}.
__global__ void adj_dudi_k(const double* part_u, int64_t T, int n_runs, int G, double* du,
                           double* di) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j > T) return;
  auto dudk = [&](int64_t k) {
    double s = 0.0;
    for (int r = 0; r < n_runs; ++r) {
      const double* q = part_u + ((int64_t)r * T + k) * G;
      for (int g = 0; g < G; ++g) s += q[g];
    }
    return s;
  };
  const double cur = j < T ? dudk(j) : 0.0;
  const double prev = j > 0 ? dudk(j - 1) : 0.0;
  if (j < T) du[j] = cur;
  di[j] = cur - prev;
}

// dJ/dR at the stored entries of R: -Phi(i, j).
__global__ void adj_gather_k(Csr R, const double* Phi, int64_t ld, double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= R.rows) return;
  for (int64_t p = R.rowptr[i]; p < R.rowptr[i + 1]; ++p)
    out[p] = -Phi[i + (int64_t)R.col[p] * ld];
}

unsigned blocks(int64_t count) { return (unsigned)std::max<int64_t>(1, ceil_div(count, 256)); }

}  // namespace

int adjoint_groups(int64_t n0) { return (int)std::max<int64_t>(1, ceil_div(n0, NT * MPT)); }

void adjoint_forward(const AdjointStep& s, double* J, double* sq, hipStream_t st) {
  MM_REQUIRE(s.G == adjoint_groups(s.n0), kInvalid, "adjoint: group count");
  MM_REQUIRE(s.K >= 1 && s.n_ckpt == ceil_div(s.T, s.K), kInvalid, "adjoint: checkpoints");
  hipLaunchKernelGGL(adj_forward_k, dim3((unsigned)s.G, (unsigned)s.n_runs), dim3(NT), 0, st, s);
  const int64_t total = (int64_t)s.n_runs * s.T;
  hipLaunchKernelGGL(adj_resid_k, dim3(blocks(total)), dim3(256), 0, st, s.part_sig, total, s.G,
                     s.dt, s.obs, s.resid, sq);
  hipLaunchKernelGGL(adj_sum_k, dim3(1), dim3(NT), 0, st, sq, total, J);
  MM_HIP_TRY(hipGetLastError());
}

void adjoint_segment(const AdjointStep& s, int64_t k0, int64_t k1, double* Zb, double* Lb,
                     hipStream_t st) {
  MM_REQUIRE(k0 % s.K == 0 && k1 > k0 && k1 - k0 <= s.K, kInvalid, "adjoint: segment");
  hipLaunchKernelGGL(adj_recompute_k, dim3((unsigned)s.G, (unsigned)s.n_runs), dim3(NT), 0, st,
                     s, k0, k1, Zb);
  hipLaunchKernelGGL(adj_backward_k, dim3((unsigned)s.G, (unsigned)s.n_runs), dim3(NT), 0, st,
                     s, k0, k1, Lb);
  MM_HIP_TRY(hipGetLastError());
}

void adjoint_waveform_grad(const AdjointStep& s, double* du, double* di, hipStream_t st) {
  hipLaunchKernelGGL(adj_dudi_k, dim3(blocks(s.T + 1)), dim3(256), 0, st, s.part_u, s.T,
                     s.n_runs, s.G, du, di);
  MM_HIP_TRY(hipGetLastError());
}

void adjoint_gather(const Csr& R, const double* Phi, int64_t ld, double* out, hipStream_t st) {
  hipLaunchKernelGGL(adj_gather_k, dim3(blocks(R.rows)), dim3(256), 0, st, R, Phi, ld, out);
  MM_HIP_TRY(hipGetLastError());
}

}  // namespace mm
