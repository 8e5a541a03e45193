// Back-transform by the bulge-chase reflectors: Z <- Q2 Z.
//
// Q2 = H_{0,0} H_{0,1} ... H_{1,0} ... in generation order (sweep s, then
// block k), so Q2 Z applies them last-first.  Reflectors are grouped by 64
// consecutive sweeps: for group g (sweeps [sa, sl)) and block k the product
// H_{sa,k} H_{sa+1,k} ... H_{sl-1,k} acts on the row window
// [sa + 1 + k nb, sl + (k+1) nb) (at most nb + 63 <= 128 rows) and equals
// I - V T V^T with V the window's 64 shifted reflectors (columns) and T upper
// triangular (the forward compact-WY factor).  The order "g descending, k
// ascending" is valid: every pair of reflectors whose relative order it
// changes acts on disjoint rows and commutes.
//
// Pass 1 (one workgroup per (g, k)): build V (128 x 64) in LDS, its Gram
// matrix, T by the recurrence T(c,c) = tau_c, T(0:c, c) = -tau_c T(0:c,0:c)
// (V^T V)(0:c, c), and VT = V T; write V and VT.
// Pass 2 (one launch): each workgroup owns 64 columns of Z and walks the
// (g, k) blocks in order; per block it stages the 128 x 64 window of Z in
// LDS and applies  W = V^T Zw,  Zw -= VT W  on the matrix cores.
// Workgroups never wait on one another.  Pairs are processed in batches
// sized to the workspace.
#include "eig.h"

#include <vector>

namespace mm {
namespace {

constexpr int NT = 256;
constexpr int GS = 64;    // sweeps per group = columns of V
constexpr int WR = 128;   // window rows (>= nb + GS - 1)
constexpr int ZC = 64;    // Z columns per workgroup
constexpr int LP = 1;     // LDS padding

struct Pair {
  int64_t sa, sl, k, wlo, wlen;
};

// ---------------------------------------------------------------------------
// pass 1: V, T, VT of one (g, k) block
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(NT) q2_build_k(const Pair* pairs, int64_t p0, int64_t n,
                                                 int nb, const int64_t* off, const double* V2,
                                                 const double* tau2, double* Vout,
                                                 double* VTout) {
  __shared__ double V[WR][GS + LP];
  __shared__ double S[GS][GS + LP];
  __shared__ double T[GS][GS + LP];
  __shared__ double tau[GS];
  __shared__ double col[GS];
  const int t = threadIdx.x;
  const Pair pr = pairs[p0 + blockIdx.x];
  // V: column gs is the reflector of sweep sa+gs at block k, placed at row
  // offset (sweep - sa) of the window (zero when the sweep has no such task)
  for (int e = t; e < WR * GS; e += NT) {
    const int i = e % WR, gs = e / WR;
    const int64_t s = pr.sa + gs;
    double v = 0.0;
    if (s < pr.sl && pr.k < ceil_div(n - 1 - s, nb)) {
      const int ro = (int)(s - pr.sa);
      const int64_t r0 = s + 1 + pr.k * nb;
      const int len = (int)min((int64_t)nb, n - r0);
      if (i >= ro && i < ro + len) v = V2[(off[s] + pr.k) * nb + (i - ro)];
    }
    V[i][gs] = v;
  }
  for (int gs = t; gs < GS; gs += NT) {
    const int64_t s = pr.sa + gs;
    tau[gs] = (s < pr.sl && pr.k < ceil_div(n - 1 - s, nb)) ? tau2[off[s] + pr.k] : 0.0;
  }
  __syncthreads();
  // S = V^T V
  for (int e = t; e < GS * GS; e += NT) {
    const int a = e % GS, b = e / GS;
    double acc = 0.0;
    for (int i = 0; i < WR; ++i) acc += V[i][a] * V[i][b];
    S[a][b] = acc;
    T[a][b] = 0.0;
  }
  __syncthreads();
  // forward recurrence for T (upper)
  for (int c = 0; c < GS; ++c) {
    const double tc = tau[c];
    if (t < c) {
      double acc = 0.0;
      for (int q = t; q < c; ++q) acc += T[t][q] * S[q][c];
      col[t] = -tc * acc;
    }
    __syncthreads();
    if (t < c) T[t][c] = col[t];
    if (t == 0) T[c][c] = tc;
    __syncthreads();
  }
  // VT = V T.  Both are written in the MFMA operand order of pass 2:
  //   F1[(h*2 + x)*32 + kk][lane] = V(4kk + lane/16, 32h + 16x + lane%16)
  //   F2[(wv*2 + x)*16 + kk][lane] = VT(32wv + 16x + lane%16, 4kk + lane/16)
  // so that every operand load there is one contiguous 512-byte wave load.
  __syncthreads();
  double* F1 = Vout + (int64_t)blockIdx.x * WR * GS;
  double* F2 = VTout + (int64_t)blockIdx.x * WR * GS;
  for (int e = t; e < WR * GS; e += NT) {
    const int ln = e & 63, f = e >> 6;          // f = (h*2 + x)*32 + kk
    const int kk = f & 31, x = (f >> 5) & 1, h = f >> 6;
    F1[e] = V[4 * kk + (ln >> 4)][32 * h + 16 * x + (ln & 15)];
  }
  for (int e = t; e < WR * GS; e += NT) {
    const int ln = e & 63, f = e >> 6;          // f = (wv*2 + x)*16 + kk
    const int kk = f & 15, x = (f >> 4) & 1, wv = f >> 5;
    const int i = 32 * wv + 16 * x + (ln & 15), j = 4 * kk + (ln >> 4);
    double acc = 0.0;
    for (int q = 0; q <= j; ++q) acc += V[i][q] * T[q][j];
    F2[e] = acc;
  }
}

// ---------------------------------------------------------------------------
// pass 2: apply the blocks of pairs [p0, p1) to 64 columns of Z per workgroup
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(NT) q2_apply_k(const Pair* pairs, int64_t p0, int64_t p1,
                                                 const double* Vall, const double* VTall,
                                                 double* Z, int64_t ldz, int64_t ncols) {
  __shared__ double Zw[WR][ZC + LP];
  __shared__ double W[GS][ZC + LP];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t col0 = (int64_t)blockIdx.x * ZC;
  const int ncl = (int)min((int64_t)ZC, ncols - col0);
  for (int64_t p = p0; p < p1; ++p) {
    const Pair pr = pairs[p];
    const int wlen = (int)pr.wlen;
    const double* F1 = Vall + (p - p0) * WR * GS;
    const double* F2 = VTall + (p - p0) * WR * GS;
    // stage the window (zero rows beyond wlen, zero columns beyond ncols)
    for (int e = t; e < WR * ZC; e += NT) {
      const int i = e % WR, j = e / WR;
      Zw[i][j] = (i < wlen && j < ncl) ? Z[(pr.wlo + i) + (col0 + j) * ldz] : 0.0;
    }
    __syncthreads();
    // W = V^T Zw  (64 x 64, K = 128): wave quadrant (wm, wn) of 32 x 32
    {
      const int h = wave & 1, wm = h * 32, wn = (wave >> 1) * 32;
      v4d acc[2][2];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = v4d{0.0, 0.0, 0.0, 0.0};
      double fa[2][WR / 4];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int kk = 0; kk < WR / 4; ++kk) fa[x][kk] = F1[((h * 2 + x) * 32 + kk) * 64 + lane];
#pragma unroll
      for (int kk = 0; kk < WR / 4; ++kk) {
        const int k0 = 4 * kk;
        double av[2], bv[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) av[x] = fa[x][kk];
#pragma unroll
        for (int y = 0; y < 2; ++y) bv[y] = Zw[k0 + lk][wn + 16 * y + lr];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
            acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[y], av[x], acc[x][y], 0, 0, 0);
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int q = 0; q < 4; ++q) W[wm + 16 * x + lr][wn + 16 * y + lk + 4 * q] = acc[x][y][q];
    }
    __syncthreads();
    // Zw -= VT W  (128 x 64, K = 64): wave owns rows [32 wave, 32 wave + 32)
    {
      const int rm = wave * 32;
      v4d acc[2][4];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = v4d{0.0, 0.0, 0.0, 0.0};
      double fb[2][GS / 4];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int kk = 0; kk < GS / 4; ++kk) fb[x][kk] = F2[((wave * 2 + x) * 16 + kk) * 64 + lane];
#pragma unroll
      for (int kk = 0; kk < GS / 4; ++kk) {
        const int k0 = 4 * kk;
        double av[2], bv[4];
#pragma unroll
        for (int x = 0; x < 2; ++x) av[x] = fb[x][kk];
#pragma unroll
        for (int y = 0; y < 4; ++y) bv[y] = W[k0 + lk][16 * y + lr];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y)
            acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[y], av[x], acc[x][y], 0, 0, 0);
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int i = rm + 16 * x + lr, j = 16 * y + lk + 4 * q;
            if (i < wlen && j < ncl) Z[(pr.wlo + i) + (col0 + j) * ldz] = Zw[i][j] - acc[x][y][q];
          }
    }
    __syncthreads();
  }
}

}  // namespace

void apply_q2(const Sb2stPlan& plan, const int64_t* d_offset, const double* V2,
              const double* tau2, double* Z, int64_t ldz, int64_t ncols, double* ws,
              int64_t ws_elems, hipStream_t s) {
  const int64_t n = plan.n;
  const int nb = plan.nb;
  MM_REQUIRE(nb + GS - 1 <= WR, kInvalid, "apply_q2: band too wide");
  if (n < 3 || ncols <= 0) return;
  const int64_t nsweeps = n - 2;  // sweeps 0..n-3 carry reflectors
  const int64_t ngroups = ceil_div(nsweeps, GS);
  std::vector<Pair> pairs;
  for (int64_t g = ngroups - 1; g >= 0; --g) {
    const int64_t sa = g * GS, sl = std::min(sa + GS, nsweeps);
    const int64_t kmax = ceil_div(n - 1 - sa, nb);
    for (int64_t k = 0; k < kmax; ++k) {
      const int64_t wlo = sa + 1 + k * nb;
      if (wlo >= n) break;
      const int64_t whi = std::min(sl + (k + 1) * nb, n);
      pairs.push_back(Pair{sa, sl, k, wlo, whi - wlo});
    }
  }
  const int64_t npairs = (int64_t)pairs.size();
  const int64_t per_pair = 2 * (int64_t)WR * GS;
  const int64_t pair_words = (int64_t)((sizeof(Pair) * npairs + 7) / 8);
  MM_REQUIRE(ws_elems > pair_words + per_pair, kInvalid, "apply_q2: workspace too small");
  Pair* d_pairs = reinterpret_cast<Pair*>(ws);
  double* buf = ws + pair_words;
  const int64_t batch = std::min<int64_t>(npairs, (ws_elems - pair_words) / per_pair);
  MM_HIP_TRY(hipMemcpyAsync(d_pairs, pairs.data(), sizeof(Pair) * npairs,
                            hipMemcpyHostToDevice, s));
  double* Vb = buf;
  double* VTb = buf + batch * WR * GS;
  const unsigned grid = (unsigned)ceil_div(ncols, ZC);
  for (int64_t p0 = 0; p0 < npairs; p0 += batch) {
    const int64_t p1 = std::min(npairs, p0 + batch);
    hipLaunchKernelGGL(q2_build_k, dim3((unsigned)(p1 - p0)), dim3(NT), 0, s, d_pairs, p0, n, nb,
                       d_offset, V2, tau2, Vb, VTb);
    hipLaunchKernelGGL(q2_apply_k, dim3(grid), dim3(NT), 0, s, d_pairs, p0, p1, Vb, VTb, Z, ldz,
                       ncols);
    MM_HIP_TRY(hipGetLastError());
  }
  // the host vector must outlive the copy
  MM_HIP_TRY(hipStreamSynchronize(s));
}

}  // namespace mm
