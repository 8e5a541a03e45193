// The classical theta-method (Sec. 3.3.1, eq. time_integration): per step
//   b = -dt Ri Ii + f^k;  C y = b;  C^T dI = y;  Ii += dI;  s = P dI / dt,
// with C the Cholesky factor of Z = Li + theta dt Ri.
//
// The two triangular solves read the whole factor once each (4 N^2 bytes
// per solve), so they are HBM-bound.  Each solve is one persistent kernel:
// the factor is cut into 128 x 128 tiles, and workgroups take work items
// from an atomic ticket in column-sweep order (diagonal block J, then the
// tiles below it).  A tile item forms its 128-long partial product as soon
// as the solution block it needs is published; a diagonal item sums the
// partials of its block row in a fixed order (so reruns are bit-identical)
// and applies the precomputed inverse of the diagonal block.  Every item
// waits only on items with smaller tickets, which are already held by
// running workgroups, so the dataflow cannot deadlock; the waits are still
// bounded and raise an error word instead of spinning forever.
#include "kernels.h"

namespace mm {
namespace {

constexpr int TB = TRSV_NB;
constexpr int NT = 256;
constexpr long kSpinLimit = 1L << 26;

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

// One thread waits until *p >= target (acquire); false on error/timeout.
__device__ bool wait_geq(unsigned* p, unsigned target, unsigned* err) {
  long spins = 0;
  while (__hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) return false;
    if (++spins > kSpinLimit) {
      atomicOr(err, 1u);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  return true;
}

__device__ __forceinline__ int64_t group_offset(int64_t g, int64_t NB) {
  return g * NB - g * (g - 1) / 2;
}

// Items come in groups g = 0..NB-1 of NB-g items each; returns (g, index).
__device__ void decode(int64_t item, int64_t NB, int64_t& g, int64_t& idx) {
  int64_t lo = 0, hi = NB - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) / 2;
    if (group_offset(mid, NB) <= item) lo = mid; else hi = mid - 1;
  }
  g = lo;
  idx = item - group_offset(lo, NB);
}

__device__ __forceinline__ int64_t tri(int64_t hi, int64_t lo) {  // hi > lo
  return hi * (hi - 1) / 2 + lo;
}

// b = -dt Ri I + F u^k;  also clears the dataflow words of both solves.
__global__ void chol_rhs_k(int64_t n0, Csr Ri, Forcing f, double theta, double dt,
                           int64_t k, const double* __restrict__ I,
                           double* __restrict__ b, unsigned* sync, int64_t nsync) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nsync) sync[1 + i] = 0u;  // sync[0] is the sticky error word
  if (i >= n0) return;
  double s = 0.0;
  for (int64_t p = Ri.rowptr[i]; p < Ri.rowptr[i + 1]; ++p) s += Ri.val[p] * I[Ri.col[p]];
  double r = -dt * s;
  for (int j = 0; j < f.nf; ++j) r += f.F[i + (int64_t)j * n0] * forcing_u(f, j, k, theta, dt);
  b[i] = r;
}

// y_J = Dinv_J r  for a 128 x 128 column-major Dinv_J; r, out in LDS.
__device__ void block_gemv(const double* __restrict__ D, const double* r, double* red,
                           double* out) {
  const int t = threadIdx.x, i = t & (TB - 1), h = t >> 7;
  double s = 0.0;
  const double* Dc = D + (int64_t)(h * 64) * TB + i;
#pragma unroll 8
  for (int c = 0; c < 64; ++c) s += Dc[(int64_t)c * TB] * r[h * 64 + c];
  red[t] = s;
  __syncthreads();
  if (t < TB) out[t] = red[t] + red[t + TB];
  __syncthreads();
}

// Forward solve C y = b in place (x holds b on entry, y on exit).
__global__ void __launch_bounds__(NT) trsv_fwd_k(int64_t n, const double* __restrict__ C,
                                                 int64_t ld, const double* __restrict__ Dinv,
                                                 double* x, double* partial,
                                                 unsigned* sync, unsigned* err) {
  const int64_t NB = ceil_div(n, TB);
  const int64_t total = group_offset(NB, NB);
  unsigned* ticket = sync;
  unsigned* count = sync + 1;
  unsigned* ready = sync + 1 + NB;
  __shared__ int64_t s_item;
  __shared__ int s_ok;
  __shared__ double vec[TB], res[TB], red[NT];
  const int t = threadIdx.x;
  for (;;) {
    if (t == 0) s_item = (int64_t)atomicAdd(ticket, 1u);
    __syncthreads();
    const int64_t item = s_item;
    if (item >= total) return;
    int64_t J, idx;
    decode(item, NB, J, idx);
    const int64_t J0 = J * TB;
    if (idx == 0) {
      // diagonal item: r = b_J - sum_{J' < J} partial(J, J') in J' order
      if (t == 0) s_ok = wait_geq(&count[J], (unsigned)J, err);
      __syncthreads();
      const int i = t & (TB - 1), h = t >> 7;
      const int64_t half = (J + 1) / 2;
      const int64_t a0 = h ? half : 0, a1 = h ? J : half;
      double acc = 0.0;
      if (s_ok)
        for (int64_t q = a0; q < a1; ++q) acc += partial[tri(J, q) * TB + i];
      red[t] = acc;
      __syncthreads();
      if (t < TB) {
        const double bi = (J0 + t < n) ? x[J0 + t] : 0.0;
        vec[t] = (J0 + t < n) ? bi - (red[t] + red[t + TB]) : 0.0;
      }
      __syncthreads();
      block_gemv(Dinv + J * TB * TB, vec, red, res);
      if (t < TB && J0 + t < n) x[J0 + t] = res[t];
      __syncthreads();
      if (t == 0) {
        __threadfence();
        __hip_atomic_store(&ready[J], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    } else {
      // tile item (I, J), I > J: partial(I, J) = C(I, J) y_J
      const int64_t I = J + idx, I0 = I * TB;
      if (t == 0) s_ok = wait_geq(&ready[J], 1u, err);
      __syncthreads();
      if (t < TB) vec[t] = s_ok ? x[J0 + t] : 0.0;  // J < NB-1: full block
      __syncthreads();
      const int i = t & (TB - 1), h = t >> 7;
      double s = 0.0;
      if (I0 + i < n) {
        const double* Cp = C + (I0 + i) + (J0 + h * 64) * ld;
#pragma unroll 8
        for (int c = 0; c < 64; ++c) s += Cp[(int64_t)c * ld] * vec[h * 64 + c];
      }
      red[t] = s;
      __syncthreads();
      if (t < TB) partial[tri(I, J) * TB + t] = red[t] + red[t + TB];
      __syncthreads();
      if (t == 0) {
        __threadfence();
        __hip_atomic_fetch_add(&count[I], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

// Backward solve C^T x = y in place; also Ii += x and the probe partials
// pp(J, p) = sum_{i in block J} Pt(i, p) x_i for this step.
__global__ void __launch_bounds__(NT) trsv_bwd_k(int64_t n, const double* __restrict__ C,
                                                 int64_t ld, const double* __restrict__ DinvT,
                                                 double* x, double* partial,
                                                 unsigned* sync, unsigned* err,
                                                 double* state, const double* __restrict__ Pt,
                                                 int n_probe, double* pp) {
  const int64_t NB = ceil_div(n, TB);
  const int64_t total = group_offset(NB, NB);
  unsigned* ticket = sync;
  unsigned* count = sync + 1;
  unsigned* ready = sync + 1 + NB;
  __shared__ int64_t s_item;
  __shared__ int s_ok;
  __shared__ double vec[TB], res[TB], red[NT];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  for (;;) {
    if (t == 0) s_item = (int64_t)atomicAdd(ticket, 1u);
    __syncthreads();
    const int64_t item = s_item;
    if (item >= total) return;
    int64_t g, idx;
    decode(item, NB, g, idx);
    const int64_t J = NB - 1 - g, J0 = J * TB;
    if (idx == 0) {
      // diagonal item: r = y_J - sum_{J2 > J} partial(J2, J) in J2 order
      if (t == 0) s_ok = wait_geq(&count[J], (unsigned)(NB - 1 - J), err);
      __syncthreads();
      const int i = t & (TB - 1), h = t >> 7;
      const int64_t cnt = NB - 1 - J, half = (cnt + 1) / 2;
      const int64_t a0 = J + 1 + (h ? half : 0), a1 = h ? NB : J + 1 + half;
      double acc = 0.0;
      if (s_ok)
        for (int64_t q = a0; q < a1; ++q) acc += partial[tri(q, J) * TB + i];
      red[t] = acc;
      __syncthreads();
      if (t < TB) vec[t] = (J0 + t < n) ? x[J0 + t] - (red[t] + red[t + TB]) : 0.0;
      __syncthreads();
      block_gemv(DinvT + J * TB * TB, vec, red, res);
      if (t < TB && J0 + t < n) {
        x[J0 + t] = res[t];
        state[J0 + t] += res[t];
      }
      // probe partials of this block
      for (int p = 0; p < n_probe; ++p) {
        double v = 0.0;
        if (t < TB && J0 + t < n) v = Pt[(J0 + t) + (int64_t)p * n] * res[t];
        v = wave_sum(v);
        if (lane == 0) red[wave] = v;
        __syncthreads();
        if (t == 0) pp[J * n_probe + p] = (red[0] + red[1]) + (red[2] + red[3]);
        __syncthreads();
      }
      if (t == 0) {
        __threadfence();
        __hip_atomic_store(&ready[J], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
      __syncthreads();
    } else {
      // tile item (I, J), I < J: partial(J, I) = C(J, I)^T x_J
      const int64_t I = J - idx, I0 = I * TB;
      if (t == 0) s_ok = wait_geq(&ready[J], 1u, err);
      __syncthreads();
      if (t < TB) vec[t] = (s_ok && J0 + t < n) ? x[J0 + t] : 0.0;
      __syncthreads();
      const bool r0 = J0 + lane < n, r1 = J0 + 64 + lane < n;
      const double x0 = vec[lane], x1 = vec[64 + lane];
      for (int cc = 0; cc < TB / 4; ++cc) {
        const int c = wave * (TB / 4) + cc;
        const double* Cc = C + J0 + (I0 + c) * ld;
        double v = 0.0;
        if (r0) v += Cc[lane] * x0;
        if (r1) v += Cc[64 + lane] * x1;
        v = wave_sum(v);
        if (lane == 0) res[c] = v;
      }
      __syncthreads();
      if (t < TB) partial[tri(J, I) * TB + t] = res[t];
      __syncthreads();
      if (t == 0) {
        __threadfence();
        __hip_atomic_fetch_add(&count[I], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
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

}  // namespace

int64_t trsv_partial_elems(int64_t n) {
  const int64_t NB = ceil_div(n, TB);
  return std::max<int64_t>(1, NB * (NB - 1) / 2) * TB;
}

// [0] error word; then per solve: ticket, count[NB], ready[NB]
int64_t trsv_sync_words(int64_t n) {
  const int64_t NB = ceil_div(n, TB);
  return 1 + 2 * (1 + 2 * NB);
}

int64_t trsv_error_offset(int64_t) { return 0; }

void chol_steps(const CholStep& c, int64_t k0, int64_t n_steps, hipStream_t s) {
  const int64_t n = c.n0;
  const int64_t NB = ceil_div(n, TB);
  const int64_t per = 1 + 2 * NB;
  const int64_t nsync = 2 * per;
  unsigned* err = c.sync;
  unsigned* fsync = c.sync + 1;
  unsigned* bsync = c.sync + 1 + per;
  const int64_t items = NB * (NB + 1) / 2;
  const unsigned grid = (unsigned)std::min<int64_t>(items, 1024);
  const unsigned rgrid = (unsigned)ceil_div(std::max(n, nsync), 256);
  for (int64_t k = k0; k < k0 + n_steps; ++k) {
    hipLaunchKernelGGL(chol_rhs_k, dim3(rgrid), dim3(256), 0, s, n, c.Ri, c.f, c.theta,
                       c.dt, k, c.I, c.b, c.sync, nsync);
    hipLaunchKernelGGL(trsv_fwd_k, dim3(grid), dim3(NT), 0, s, n, c.Cf, c.ld, c.Dinv, c.b,
                       c.partial, fsync, err);
    hipLaunchKernelGGL(trsv_bwd_k, dim3(grid), dim3(NT), 0, s, n, c.Cf, c.ld,
                       c.Dinv + NB * TB * TB, c.b, c.partial, bsync, err, c.I, c.Pt,
                       c.n_probe, c.probe_partial + (k - k0) * NB * c.n_probe);
  }
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
