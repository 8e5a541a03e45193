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
// Zero structure used (valid for any nb <= 64): column gs of V is non-zero
// only on window rows [gs, gs + 64), so W = V^T Zw for V columns
// [16x, 16x + 16) needs window rows [16x, 16x + 80) only; VT = V T has row i
// non-zero only in columns j >= i - 63, so row block r of VT (rows
// [16r, 16r + 16)) needs k-steps kk >= ks(r) = max(0, 4r - 16).
// Consecutive blocks k, k + 1 of one group (nb = 64) have windows offset by
// 64 rows: the lower half of block k's window stays in LDS as the upper half
// of block k + 1's, and only 64 new rows are loaded, prefetched into
// registers while the matrix cores work on block k.
__device__ constexpr int ks_of(int r) { return r < 4 ? 0 : 4 * r - 16; }
__device__ constexpr int koff_of(int r) {  // compact fragment offset of row block r
  return r <= 5 ? 16 * r : (r == 6 ? 92 : 100);
}
constexpr int NVT = 104;  // non-zero VT fragments (16 x 4 each)

__global__ void __launch_bounds__(NT) q2_apply_k(const Pair* pairs, int64_t p0, int64_t p1,
                                                 const double* Vall, const double* VTall,
                                                 double* Z, int64_t ldz, int64_t n,
                                                 int64_t ncols) {
  __shared__ double Zh[2][64][ZC + LP];  // window halves; Zh[a] holds rows [0, 64)
  __shared__ double W[GS][ZC + LP];
  __shared__ double VTs[NVT * 64];       // compact VT fragments of the current block
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t col0 = (int64_t)blockIdx.x * ZC;
  const int ncl = (int)min((int64_t)ZC, ncols - col0);
  int a = 0;
  bool resident = false;  // the window's upper half is already in LDS
  for (int64_t p = p0; p < p1; ++p) {
    const Pair pr = pairs[p];
    bool cont = false;
    if (p + 1 < p1) {
      const Pair nx = pairs[p + 1];
      cont = nx.sa == pr.sa && nx.k == pr.k + 1 && nx.wlo == pr.wlo + 64;
    }
    const double* F1 = Vall + (p - p0) * WR * GS;
    const double* F2 = VTall + (p - p0) * WR * GS;
    // issue this block's VT fragments (26 per thread) and the next block's
    // new rows (16 per thread)
    double vt[NVT / 4];
#pragma unroll
    for (int u = 0; u < NVT / 4; ++u) {
      const int e = t + NT * u, fc = e >> 6;
      const int g = fc < 80 ? fc : fc < 92 ? fc + 4 : fc < 100 ? fc + 12 : fc + 24;
      vt[u] = F2[g * 64 + (e & 63)];
    }
    double zn[16];
    if (cont) {
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = t + NT * u, i = e & 63, j = e >> 6;
        const int64_t row = pr.wlo + 128 + i;
        zn[u] = (row < n && j < ncl) ? Z[row + (col0 + j) * ldz] : 0.0;
      }
    }
    if (!resident) {
      // the whole window (rows beyond n and columns beyond ncols are zero)
#pragma unroll 4
      for (int u = 0; u < 32; ++u) {
        const int e = t + NT * u, i = e & 127, j = e >> 7;
        const int64_t row = pr.wlo + i;
        Zh[a ^ (i >> 6)][i & 63][j] = (row < n && j < ncl) ? Z[row + (col0 + j) * ldz] : 0.0;
      }
      __syncthreads();
    }
    // ---- W = V^T Zw: wave owns W rows [16 wave, 16 wave + 16), k-steps
    //      kk = 4 wave + s (window rows 16 wave + 4 s + lk), s < 20
    {
      double fa[20];
#pragma unroll
      for (int s2 = 0; s2 < 20; ++s2) fa[s2] = F1[(wave * 32 + 4 * wave + s2) * 64 + lane];
      v4d acc[4];
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[y] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s2 = 0; s2 < 20; ++s2) {
        const int i = 16 * wave + 4 * s2 + lk;
        const double* zr = &Zh[a ^ (i >> 6)][i & 63][0];
        double bv[4];
#pragma unroll
        for (int y = 0; y < 4; ++y) bv[y] = zr[16 * y + lr];
#pragma unroll
        for (int y = 0; y < 4; ++y)
          acc[y] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[y], fa[s2], acc[y], 0, 0, 0);
      }
#pragma unroll
      for (int y = 0; y < 4; ++y)
#pragma unroll
        for (int q = 0; q < 4; ++q) W[16 * wave + lr][16 * y + lk + 4 * q] = acc[y][q];
    }
#pragma unroll
    for (int u = 0; u < NVT / 4; ++u) VTs[t + NT * u] = vt[u];
    __syncthreads();
    // ---- Zw -= VT W: wave owns columns [16 wave, 16 wave + 16), all rows
    {
      double wb[16];
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) wb[kk] = W[4 * kk + lk][16 * wave + lr];
      v4d acc[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) acc[r] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < 16; ++kk)
#pragma unroll
        for (int r = 0; r < 8; ++r)
          if (kk >= ks_of(r))
            acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                wb[kk], VTs[(koff_of(r) + kk - ks_of(r)) * 64 + lane], acc[r], 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int i = 16 * r + lr;
        double* zr = &Zh[a ^ (r >> 2)][i & 63][0];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int j = 16 * wave + lk + 4 * q;
          const double zv = zr[j] - acc[r][q];
          if (cont && r >= 4) {
            zr[j] = zv;
          } else {
            const int64_t row = pr.wlo + i;
            if (row < n && j < ncl) Z[row + (col0 + j) * ldz] = zv;
          }
        }
      }
    }
    __syncthreads();
    if (cont) {
      // the lower half becomes the upper half; the new rows fill the other
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = t + NT * u;
        Zh[a][e & 63][e >> 6] = zn[u];
      }
      a ^= 1;
      __syncthreads();
    }
    resident = cont;
  }
}

// ---------------------------------------------------------------------------
// Y <- Q2^T Y for a few columns (one launch per stage of a wavefront)
// ---------------------------------------------------------------------------
// Q2^T = (B_0 ... B_last)^T with the blocks B in the order of q2_pairs, so
// Q2^T Y applies the blocks in the reverse order (g ascending, k descending),
// each as its reflectors in generation order (sweep ascending; the block's
// transpose I - V T^T V^T).  The blocks of one launch share no row.  Each
// workgroup applies one block to 64 columns: the 128-row window staged in
// LDS, the block's reflectors one after the other (wave w sums and updates
// reflector rows [16 w, 16 w + 16), lane = column).
__global__ void __launch_bounds__(NT) q2t_apply_k(const Pair* pairs, int64_t p0, int64_t n,
                                                  int nb, const int64_t* off, const double* V2,
                                                  const double* tau2, double* Y, int64_t ldy,
                                                  int64_t ncols) {
  __shared__ double Yw[WR][ZC + LP];
  __shared__ double Vs[GS][GS + LP];  // Vs[gs][i]: element i of sweep sa + gs's reflector
  __shared__ double ts[GS];
  __shared__ double red[4][ZC];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const Pair pr = pairs[p0 + blockIdx.x];
  const int64_t col0 = (int64_t)blockIdx.y * ZC;
  const int ncl = (int)min((int64_t)ZC, ncols - col0);
  for (int e = t; e < WR * ZC; e += NT) {
    const int i = e % WR, j = e / WR;
    const int64_t row = pr.wlo + i;
    Yw[i][j] = (row < n && j < ncl) ? Y[row + (col0 + j) * ldy] : 0.0;
  }
  for (int e = t; e < GS * GS; e += NT) {
    const int i = e % GS, gs = e / GS;
    const int64_t s = pr.sa + gs;
    const bool ok = s < pr.sl && pr.k < ceil_div(n - 1 - s, nb) && i < nb;
    Vs[gs][i] = ok ? V2[(off[s] + pr.k) * nb + i] : 0.0;
  }
  for (int gs = t; gs < GS; gs += NT) {
    const int64_t s = pr.sa + gs;
    ts[gs] = (s < pr.sl && pr.k < ceil_div(n - 1 - s, nb)) ? tau2[off[s] + pr.k] : 0.0;
  }
  __syncthreads();
  // the reflector of sweep sa + gs starts at window row gs
  for (int gs = 0; gs < GS; ++gs) {
    const double tau = ts[gs];
    if (tau == 0.0) continue;  // uniform: H = I
    const int i0 = 16 * wave;
    double yr[16];
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      yr[q] = Yw[gs + i0 + q][lane];
      acc += Vs[gs][i0 + q] * yr[q];
    }
    red[wave][lane] = acc;
    __syncthreads();
    const double d = tau * ((red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]));
#pragma unroll
    for (int q = 0; q < 16; ++q) Yw[gs + i0 + q][lane] = yr[q] - Vs[gs][i0 + q] * d;
    __syncthreads();
  }
  for (int e = t; e < WR * ZC; e += NT) {
    const int i = e % WR, j = e / WR;
    const int64_t row = pr.wlo + i;
    if (row < n && j < ncl) Y[row + (col0 + j) * ldy] = Yw[i][j];
  }
}

// the (g, k) blocks in application order: g descending, k ascending
std::vector<Pair> q2_pairs(int64_t n, int nb) {
  std::vector<Pair> pairs;
  if (n < 3) return pairs;
  const int64_t nsweeps = n - 2;  // sweeps 0..n-3 carry reflectors
  const int64_t ngroups = ceil_div(nsweeps, GS);
  for (int64_t g = ngroups - 1; g >= 0; --g) {
    const int64_t sa = g * GS, sl = std::min(sa + GS, nsweeps);
    const int64_t kmax = ceil_div(n - 1 - sa, nb);
    for (int64_t k = 0; k < kmax; ++k) {
      const int64_t wlo = sa + 1 + k * nb;
      if (wlo >= n) break;
      const int64_t whi = std::min(wlo + WR, n);
      pairs.push_back(Pair{sa, sl, k, wlo, whi - wlo});
    }
  }
  return pairs;
}

constexpr int64_t kPerPair = 2 * (int64_t)WR * GS;  // V and VT of one block

int64_t pair_list_words(int64_t npairs) { return (int64_t)((sizeof(Pair) * npairs + 7) / 8); }

}  // namespace

int64_t apply_q2_ws_elems(int64_t n, int nb) {
  const int64_t npairs = (int64_t)q2_pairs(n, nb).size();
  return pair_list_words(npairs) + kPerPair * std::max<int64_t>(1, npairs) + 1;
}

void apply_q2(const Sb2stPlan& plan, const int64_t* d_offset, const double* V2,
              const double* tau2, double* Z, int64_t ldz, int64_t ncols, double* ws,
              int64_t ws_elems, hipStream_t s) {
  const int64_t n = plan.n;
  const int nb = plan.nb;
  MM_REQUIRE(nb + GS - 1 <= WR, kInvalid, "apply_q2: band too wide");
  if (n < 3 || ncols <= 0) return;
  const std::vector<Pair> pairs = q2_pairs(n, nb);
  const int64_t npairs = (int64_t)pairs.size();
  const int64_t per_pair = kPerPair;
  const int64_t pair_words = pair_list_words(npairs);
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
                       n, ncols);
    MM_HIP_TRY(hipGetLastError());
  }
  // the host vector must outlive the copy
  MM_HIP_TRY(hipStreamSynchronize(s));
}

int64_t apply_q2t_ws_elems(int64_t n, int nb) {
  return pair_list_words((int64_t)q2_pairs(n, nb).size()) + 1;
}

void apply_q2t(const Sb2stPlan& plan, const int64_t* d_offset, const double* V2,
               const double* tau2, double* Y, int64_t ldy, int64_t ncols, double* ws,
               int64_t ws_elems, hipStream_t s) {
  const int64_t n = plan.n;
  const int nb = plan.nb;
  MM_REQUIRE(nb + GS - 1 <= WR, kInvalid, "apply_q2t: band too wide");
  if (n < 3 || ncols <= 0) return;
  const std::vector<Pair> fwd = q2_pairs(n, nb);
  const int64_t npairs = (int64_t)fwd.size();
  MM_REQUIRE(ws_elems >= pair_list_words(npairs), kInvalid, "apply_q2t: workspace too small");
  // Stages.  With nb = GS the window of block (g, k) starts at row
  // GS (g + k) + 1, so the blocks before it (in the order g ascending,
  // k descending) that share rows with it have windows g' + k' within one of
  // g + k and g' - k' < g - k; blocks with equal g - k are 2 GS rows apart.
  // Stage g - k (shifted to start at 0) is therefore a valid wavefront.
  // Otherwise (nb < GS: at most GS + 1 unknowns, a handful of blocks) every
  // block is a stage of its own.
  std::vector<Pair> order;
  std::vector<int64_t> start;
  if (nb == GS) {
    int64_t kmax = 0, gmax = 0;
    for (const Pair& p : fwd) {
      kmax = std::max(kmax, p.k);
      gmax = std::max(gmax, p.sa / GS);
    }
    const int64_t nst = gmax + kmax + 1;
    std::vector<int64_t> cnt(nst + 1, 0);
    for (const Pair& p : fwd) ++cnt[p.sa / GS - p.k + kmax + 1];
    for (int64_t i = 0; i < nst; ++i) cnt[i + 1] += cnt[i];
    start = cnt;
    order.resize(npairs);
    for (const Pair& p : fwd) order[cnt[p.sa / GS - p.k + kmax]++] = p;
  } else {
    order.assign(fwd.rbegin(), fwd.rend());
    start.resize(npairs + 1);
    for (int64_t i = 0; i <= npairs; ++i) start[i] = i;
  }
  Pair* d_pairs = reinterpret_cast<Pair*>(ws);
  MM_HIP_TRY(hipMemcpyAsync(d_pairs, order.data(), sizeof(Pair) * npairs,
                            hipMemcpyHostToDevice, s));
  const unsigned cgrid = (unsigned)ceil_div(ncols, ZC);
  for (size_t st = 0; st + 1 < start.size(); ++st) {
    const int64_t p0 = start[st], p1 = start[st + 1];
    if (p1 == p0) continue;
    hipLaunchKernelGGL(q2t_apply_k, dim3((unsigned)(p1 - p0), cgrid), dim3(NT), 0, s, d_pairs,
                       p0, n, nb, d_offset, V2, tau2, Y, ldy, ncols);
  }
  MM_HIP_TRY(hipGetLastError());
  // the host vector must outlive the copy
  MM_HIP_TRY(hipStreamSynchronize(s));
}

}  // namespace mm
