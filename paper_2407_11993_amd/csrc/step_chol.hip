// The classical theta-method (Sec. 3.3.1, eq. time_integration): per step
//   b = -dt Ri Ii + f^k;  C y = b;  C^T dI = y;  Ii += dI;  s = P dI / dt,
// with C the Cholesky factor of Z = Li + theta dt Ri.
//
// Block substitution with pre-scaled panels.  With D = blockdiag(C_JJ) (B x B
// blocks, B = 2048 at large N) the two solves are
//   forward:  y_J = D_J^{-1} b_J - sum_{K<J} W_JK y_K,      W_JK = D_J^{-1} C_JK,
//   backward: x_J = D_J^{-T} y_J - sum_{K>J} V_KJ^T x_K,    V_KJ = C_KJ D_J^{-1},
// so once per factorisation W replaces C's blocks below the diagonal blocks
// and V^T fills the (otherwise unused) blocks above them.  A solve is then
// one block-diagonal product over all blocks at once, followed by a chain of
// panel updates with no diagonal work between them, and both solves read
// column panels.  The bytes read per solve are those of C's lower triangle
// (D^{-1}'s lower triangles plus the panels), and the solves stay HBM-bound.
// A panel update is split into 256-column chunks, each accumulating into its
// own copy of the partial sums, so that short panels still fill the chip and
// no two workgroups write the same word.  Synchronisation is by kernel
// boundaries only (no workgroup waits on another); every sum has a fixed
// order, so reruns are bit-identical.
//
// One step's launches read the step index from device memory, so the whole
// step is captured once into a HIP graph and replayed n_steps times.
#include "kernels.h"

namespace mm {
namespace {

constexpr int NT = 256;
constexpr int MAXB = 4096;
constexpr int UW = 16;  // waves per panel-update workgroup
constexpr int UL = 16;  // column loads in flight per wave (UW * UL = 256 columns per chunk)

// Workgroups of a diagonal-block kernel: four waves, two rows or columns each.
constexpr int DT = 512;  // block-diagonal kernels: 8 waves, 16 rows or columns per workgroup
__host__ __device__ inline int diag_groups(int B) { return (B / 2 + DT / 64 - 1) / (DT / 64); }

// base[byte_off / 8] with a 32-bit byte offset, so the load can take the
// scalar base + 32-bit vector offset form (one address register per load)
__device__ __forceinline__ double ld_off(const double* base, unsigned byte_off) {
  return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(base) + byte_off);
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

// Block-diagonal products.  Rows (forward) or columns (backward) p and
// jb-1-p of a triangular block inverse are folded onto one wave: together
// they hold jb + 1 entries, so every wave does the same work and issues all
// of its loads at once (clamped addresses, masked values).  KC load slots per
// lane: the two rows of a forward pair span at most B / 64 + 1 chunks of 64,
// the two columns of a backward pair at most B / 64 + 2 (their first chunks
// need not be aligned).  blockIdx.y is the block; its right-hand side is
// staged in LDS once per workgroup.  The workgroups of block J also clear
// the accumulators (S x n) on the block's rows for the panel updates that
// follow.
// Forward: z_J(r) = sum_{c <= r} Dinv_J(r, c) b_J(c), row r of Dinv_J read
// contiguously from DinvT.
template <int KC>
__global__ void __launch_bounds__(DT) fwd_bd_k(int64_t n, int B, const double* __restrict__ DinvT,
                                               const double* __restrict__ b,
                                               double* __restrict__ z, double* __restrict__ acc,
                                               int S) {
  __shared__ double bs[MAXB];
  const int t = threadIdx.x, lane = t & 63;
  const int wave = t >> 6;
  const int64_t J = blockIdx.y;
  const int64_t J0 = J * B;
  const int jb = (int)min((int64_t)B, n - J0);
  // a wave past the last pair computes pair 0 again and discards it, so the
  // barrier below is reached by every thread
  const int pw = blockIdx.x * (DT / 64) + wave;
  const bool live = pw < (jb + 1) / 2;
  const int p = live ? pw : 0;
  const int r1 = p, r2 = jb - 1 - p;
  const int n1 = r1 / 64 + 1, n2 = (r2 > r1) ? r2 / 64 + 1 : 0;
  // one base per block and 32-bit byte offsets (8 B * B < 2^32)
  const double* Db = DinvT + J * (int64_t)B * B;
  double dv[KC];
#pragma unroll
  for (int v = 0; v < KC; ++v) {
    const bool sec = v >= n1;
    const int rr = sec ? r2 : r1;
    dv[v] = ld_off(Db, 8u * (unsigned)(rr * B + min(64 * (sec ? v - n1 : v) + lane, rr)));
  }
  // the block's right-hand side, staged while the loads above are in flight
  for (int c = t; c < jb; c += DT) bs[c] = b[J0 + c];
  for (int64_t e = (int64_t)blockIdx.x * DT + t; e < (int64_t)jb * S; e += (int64_t)gridDim.x * DT)
    acc[(e / jb) * n + J0 + e % jb] = 0.0;
  __syncthreads();
  double s1 = 0.0, s2 = 0.0;
#pragma unroll
  for (int v = 0; v < KC; ++v) {
    const bool sec = v >= n1;
    const int rr = sec ? r2 : r1;
    const int c = 64 * (sec ? v - n1 : v) + lane;
    const bool ok = v < n1 + n2 && c <= rr;
    const double val = ok ? dv[v] * bs[min(c, rr)] : 0.0;
    if (sec) s2 += val;
    else s1 += val;
  }
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  if (live && lane == 0) {
    z[J0 + r1] = s1;
    if (r2 > r1) z[J0 + r2] = s2;
  }
}

// Backward: x_J(c) = sum_{r >= c} Dinv_J(r, c) y_J(r), column c of Dinv_J
// read contiguously, y the forward solve's result.
template <int KC>
__global__ void __launch_bounds__(DT) bwd_bd_k(int64_t n, int B, const double* __restrict__ Dinv,
                                               const double* __restrict__ y, int S,
                                               double* __restrict__ x, double* __restrict__ accb) {
  __shared__ double ys[MAXB];
  const int t = threadIdx.x, lane = t & 63;
  const int wave = t >> 6;
  const int64_t J = blockIdx.y;
  const int64_t J0 = J * B;
  const int jb = (int)min((int64_t)B, n - J0);
  const int pw = blockIdx.x * (DT / 64) + wave;
  const bool live = pw < (jb + 1) / 2;
  const int p = live ? pw : 0;
  const int c1 = p, c2 = jb - 1 - p;
  const int last = (jb - 1) / 64;  // chunk of the block's last row
  const int f1 = c1 / 64, f2 = c2 / 64;
  const int n1 = last - f1 + 1, n2 = (c2 > c1) ? last - f2 + 1 : 0;
  // one base per block and 32-bit byte offsets (8 B * B < 2^32)
  const double* Db = Dinv + J * (int64_t)B * B;
  double dv[KC];
#pragma unroll
  for (int v = 0; v < KC; ++v) {
    const bool sec = v >= n1;
    const int cc = sec ? c2 : c1;
    const int r = 64 * (sec ? f2 + (v - n1) : f1 + v) + lane;
    dv[v] = ld_off(Db, 8u * (unsigned)(cc * B + min(max(r, cc), jb - 1)));
  }
  for (int c = t; c < jb; c += DT) ys[c] = y[J0 + c];
  for (int64_t e = (int64_t)blockIdx.x * DT + t; e < (int64_t)jb * S; e += (int64_t)gridDim.x * DT)
    accb[(e / jb) * n + J0 + e % jb] = 0.0;
  __syncthreads();
  double s1 = 0.0, s2 = 0.0;
#pragma unroll
  for (int v = 0; v < KC; ++v) {
    const bool sec = v >= n1;
    const int cc0 = sec ? c2 : c1;
    const int r = 64 * (sec ? f2 + (v - n1) : f1 + v) + lane;
    const bool ok = v < n1 + n2 && r >= cc0 && r < jb;
    const double val = ok ? dv[v] * ys[min(max(r, cc0), jb - 1)] : 0.0;
    if (sec) s2 += val;
    else s1 += val;
  }
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  if (live && lane == 0) {
    x[J0 + c1] = s1;
    if (c2 > c1) x[J0 + c2] = s2;
  }
}

// Panel update with the pre-scaled panel M (W below the diagonal blocks for
// the forward solve, V^T above them for the backward one):
//   acc_g(i) += sum_{c in chunks g, g+G, ...} M(i, col0 + c) v(c),   row0 <= i < row0 + nrows,
// where a chunk is UW * UL = 256 columns of the panel, g = blockIdx.y < G,
// and v(c) = z(col0 + c) - sum_q acc_q(col0 + c) are the block's final values
// (every earlier panel's contribution is in the accumulators), staged in LDS
// once per workgroup for all of its chunks.  Workgroup: a tile of 64 rows
// (one per lane, so every wave load is one contiguous 512-byte column
// segment) walking its chunks, UL columns per wave and chunk, the loads of a
// chunk issued before the first use; the waves' row sums are combined in LDS
// in wave order.  Column group g owns accumulator copy g, so no two
// workgroups write the same word and every sum has a fixed order (no
// atomics).
template <int S>
__global__ void __launch_bounds__(64 * UW) upd_k(int64_t n, int64_t row0, int64_t nrows,
                                                 int64_t col0, int jb,
                                                 const double* __restrict__ M, int64_t ld,
                                                 const double* __restrict__ z,
                                                 double* __restrict__ acc, int G) {
  constexpr int CH = UW * UL;  // columns per chunk
  __shared__ double red[UW][64];
  __shared__ double vs[S * CH];
  const int t = threadIdx.x, lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int g = blockIdx.y;
  const int64_t row = row0 + (int64_t)blockIdx.x * 64 + lane;
  const bool rok = row < row0 + nrows;
  const double* Mp = M + min(row, row0 + nrows - 1);  // clamped row
  int ch = g;
  double cv[UL];
#pragma unroll
  for (int u = 0; u < UL; ++u) cv[u] = Mp[(col0 + min(ch * CH + wave * UL + u, jb - 1)) * ld];
  __builtin_amdgcn_sched_barrier(0);  // the first chunk's loads issue first
  double old = 0.0;
  if (wave == 0 && rok) old = acc[(int64_t)g * n + row];
  const int P = (S - g + G - 1) / G;  // chunks of this workgroup
  for (int e = t; e < P * CH; e += 64 * UW) {
    const int c = (g + (e / CH) * G) * CH + e % CH;
    double v = 0.0;  // zero past the panel's last column
    if (c < jb) {
      v = z[col0 + c];
#pragma unroll
      for (int q = 0; q < S; ++q) v -= acc[(int64_t)q * n + col0 + c];
    }
    vs[e] = v;
  }
  __syncthreads();
  double a4[4] = {0.0, 0.0, 0.0, 0.0};
  for (int p = 0;; ++p) {
#pragma unroll
    for (int u = 0; u < UL; ++u) a4[u & 3] += cv[u] * vs[p * CH + wave * UL + u];
    ch += G;
    if (ch >= S) break;
#pragma unroll
    for (int u = 0; u < UL; ++u) cv[u] = Mp[(col0 + min(ch * CH + wave * UL + u, jb - 1)) * ld];
  }
  red[wave][lane] = (a4[0] + a4[1]) + (a4[2] + a4[3]);
  __syncthreads();
  if (wave != 0) return;
  double sum = 0.0;
#pragma unroll
  for (int w = 0; w < UW; ++w) sum += red[w][lane];
  if (rok) acc[(int64_t)g * n + row] = old + sum;
}

// y = z - sum_q acc_q (the forward solve's result, in place of z).
__global__ void combine_k(int64_t n, double* __restrict__ z, const double* __restrict__ acc,
                          int S) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = z[i];
  for (int q = 0; q < S; ++q) v -= acc[(int64_t)q * n + i];
  z[i] = v;
}

// End of a step: dI = x - sum_q accb_q, Ii += dI, and the probe partial sums
// of this workgroup's 256 rows (one per workgroup and probe, fixed order).
// The step index is kstep[1]; the first thread advances kstep[0] (read by
// no other kernel of the step after chol_rhs_k).
__global__ void __launch_bounds__(NT) finish_k(int64_t n, const double* __restrict__ x,
                                               const double* __restrict__ accb, int S,
                                               double* __restrict__ state,
                                               const double* __restrict__ Pt, int n_probe,
                                               double* __restrict__ pp_base,
                                               int64_t* kstep, int64_t parts) {
  __shared__ double red[8][NT / 64];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t i = (int64_t)blockIdx.x * NT + t;
  double d = 0.0;
  if (i < n) {
    d = x[i];
    for (int q = 0; q < S; ++q) d -= accb[(int64_t)q * n + i];
    state[i] += d;
  }
  const int64_t k = kstep[1];
  if (i == 0) kstep[0] = k + 1;
  for (int p = 0; p < n_probe; ++p) {
    const double v = wave_sum(i < n ? Pt[i + (int64_t)p * n] * d : 0.0);
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

template <int C64>  // C64 = B / 64
void launch_bd_b(bool fwd, unsigned grid, unsigned nb, hipStream_t s, int64_t n,
                 const CholStep& c) {
  if (fwd)
    hipLaunchKernelGGL((fwd_bd_k<C64 + 1>), dim3(grid, nb), dim3(DT), 0, s, n, c.B, c.DinvT, c.b,
                       c.y, c.accf, c.B / (UW * UL));
  else
    hipLaunchKernelGGL((bwd_bd_k<C64 + 2>), dim3(grid, nb), dim3(DT), 0, s, n, c.B, c.Dinv, c.y,
                       c.B / (UW * UL), c.b, c.accb);
}
void launch_bd(bool fwd, int B, unsigned grid, unsigned nb, hipStream_t s, int64_t n,
               const CholStep& c) {
  switch (B) {
    case 256: launch_bd_b<4>(fwd, grid, nb, s, n, c); break;
    case 512: launch_bd_b<8>(fwd, grid, nb, s, n, c); break;
    case 1024: launch_bd_b<16>(fwd, grid, nb, s, n, c); break;
    case 2048: launch_bd_b<32>(fwd, grid, nb, s, n, c); break;
    case 4096: launch_bd_b<64>(fwd, grid, nb, s, n, c); break;
    default: throw Error{kInvalid, "triangular solve: unsupported block size"};
  }
}

// Column groups G of a panel update of `tiles` row tiles and S chunks.  With
// one workgroup per CU at a time (the kernel's register use), a workgroup of
// P = S / G chunks costs about P + 1/2 chunk-times (the 1/2: staging the
// block values and combining the waves), so the estimate is
// ceil(tiles G / CUs) (S / G + 1/2); the smallest G of least estimate wins.
int upd_groups(int64_t tiles, int S) {
  constexpr int64_t kCUs = 256;
  int best = 1;
  double best_cost = 1e300;
  for (int G = 1; G <= S; G *= 2) {
    const double cost = (double)ceil_div(tiles * G, kCUs) * ((double)S / G + 0.5);
    if (cost < best_cost) {
      best_cost = cost;
      best = G;
    }
  }
  return best;
}

void launch_upd(int64_t n, int64_t row0, int64_t nrows, int64_t col0, int jb, const CholStep& c,
                const double* z, double* acc, hipStream_t s) {
  if (nrows <= 0) return;
  const int S = c.B / (UW * UL);
  const int64_t tiles = ceil_div(nrows, 64);
  const int G = upd_groups(tiles, S);
  const dim3 grid((unsigned)tiles, (unsigned)G);
  switch (S) {
    case 1: hipLaunchKernelGGL((upd_k<1>), grid, dim3(64 * UW), 0, s, n, row0, nrows, col0, jb, c.Cf, c.ld, z, acc, G); break;
    case 2: hipLaunchKernelGGL((upd_k<2>), grid, dim3(64 * UW), 0, s, n, row0, nrows, col0, jb, c.Cf, c.ld, z, acc, G); break;
    case 4: hipLaunchKernelGGL((upd_k<4>), grid, dim3(64 * UW), 0, s, n, row0, nrows, col0, jb, c.Cf, c.ld, z, acc, G); break;
    case 8: hipLaunchKernelGGL((upd_k<8>), grid, dim3(64 * UW), 0, s, n, row0, nrows, col0, jb, c.Cf, c.ld, z, acc, G); break;
    case 16: hipLaunchKernelGGL((upd_k<16>), grid, dim3(64 * UW), 0, s, n, row0, nrows, col0, jb, c.Cf, c.ld, z, acc, G); break;
    default: throw Error{kInvalid, "triangular solve: unsupported block size"};
  }
}

// One step's launch sequence (the step index is kstep[0], advanced by the last kernel):
//   b = rhs;  z = D^{-1} b;  for J = 0..NB-2: accf += W(:, J) (z - accf)_J, rows below J;
//   y = z - accf;  x = D^{-T} y;  for J = NB-1..1: accb += V^T(:, J) (x - accb)_J, rows above J;
//   dI = x - accb;  Ii += dI;  probe partial sums.
void enqueue_step(const CholStep& c, hipStream_t s) {
  const int64_t n = c.n0;
  const int B = c.B;
  const int64_t NB = ceil_div(n, B);
  const int64_t parts = trsv_parts(n);
  const unsigned rgrid = (unsigned)ceil_div(n, 256);
  const unsigned dgrid = (unsigned)diag_groups(B);
  hipLaunchKernelGGL(chol_rhs_k, dim3(rgrid), dim3(256), 0, s, n, c.Ri, c.f, c.theta, c.dt,
                     c.kstep, c.I, c.b);
  if (c.Rlr.ns > 0)
    hipLaunchKernelGGL(lowrank_rhs_k, dim3(1), dim3(256), 0, s, c.Rlr, c.dt, c.I, c.b);
  launch_bd(true, B, dgrid, (unsigned)NB, s, n, c);
  for (int64_t J = 0; J + 1 < NB; ++J)
    launch_upd(n, (J + 1) * B, n - (J + 1) * B, J * B, B, c, c.y, c.accf, s);
  if (NB > 1)
    hipLaunchKernelGGL(combine_k, dim3(rgrid), dim3(256), 0, s, n, c.y, c.accf, B / (UW * UL));
  launch_bd(false, B, dgrid, (unsigned)NB, s, n, c);
  for (int64_t J = NB - 1; J >= 1; --J)
    launch_upd(n, 0, J * B, J * B, (int)std::min<int64_t>(B, n - J * B), c, c.b, c.accb, s);
  hipLaunchKernelGGL(finish_k, dim3((unsigned)parts), dim3(NT), 0, s, n, c.b, c.accb,
                     B / (UW * UL), c.I, c.Pt, c.n_probe, c.probe_partial, c.kstep, parts);
}

}  // namespace

int trsv_block(int64_t n) {
  // about eight diagonal blocks, at most 2048: fewer, larger launches (4096
  // measured no faster at N = 16384 and doubles the inverse blocks' memory)
  int B = 256;
  while (B < 2048 && 8 * (int64_t)(2 * B) <= n) B *= 2;
  return B;
}

int64_t trsv_parts(int64_t n) { return ceil_div(n, NT); }

void chol_steps(const CholStep& c, int64_t k0, int64_t n_steps, hipStream_t s) {
  MM_REQUIRE(c.B == 256 || c.B == 512 || c.B == 1024 || c.B == 2048 || c.B == 4096, kInvalid,
             "chol_steps: block size must be a power of two in [256, 4096]");
  MM_REQUIRE(c.n_probe <= 8, kInvalid, "chol_steps: at most 8 probes");
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

void trsv_prescale(double* Cf, int64_t n, int B, const double* Dinv, double* T,
                   hipStream_t s) {
  const int64_t NB = ceil_div(n, B);
  // V^T first: it reads C's blocks below the diagonal before W overwrites them
  for (int64_t J = 0; J < NB; ++J) {
    const int64_t J0 = J * B, jb = std::min<int64_t>(B, n - J0), m = n - J0 - jb;
    if (m <= 0) continue;
    Gemm g;  // (V_{below,J})^T = D_J^{-T} C_{below,J}^T, into the blocks right of D_J
    g.m = jb; g.n = m; g.k = jb;
    g.A = Dinv + J * (int64_t)B * B; g.lda = B; g.ta = true; g.a_upper = true;
    g.B = Cf + (J0 + jb) + J0 * n; g.ldb = n; g.tb = true;
    g.C = Cf + J0 + (J0 + jb) * n; g.ldc = n;
    gemm(g, s);
  }
  for (int64_t J = 1; J < NB; ++J) {
    const int64_t J0 = J * B, jb = std::min<int64_t>(B, n - J0);
    Gemm g;  // W_{J,left} = D_J^{-1} C_{J,left}, through T (B x n)
    g.m = jb; g.n = J0; g.k = jb;
    g.A = Dinv + J * (int64_t)B * B; g.lda = B; g.a_lower = true;
    g.B = Cf + J0; g.ldb = n;
    g.C = T; g.ldc = jb;
    gemm(g, s);
    copy_matrix(T, jb, Cf + J0, n, jb, J0, s);
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
