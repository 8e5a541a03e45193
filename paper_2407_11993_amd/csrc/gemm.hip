// FP64 GEMM on the gfx950 matrix cores (v_mfma_f64_16x16x4_f64).
//
// C = alpha op(A) op(B) + beta C, column-major.  One workgroup of four
// 64-wide waves computes a BM x BN tile; each wave owns a (BM/2) x (BN/2)
// quarter made of 16x16 MFMA blocks.  op(A) and op(B) are staged through LDS
// in k-slices of 16 (double buffered, one barrier per slice).  The operands
// are fed to the MFMA with B first so that each lane's four results lie in
// one column of C on consecutive rows, which makes the column-major stores
// contiguous per 16 lanes.
//
// Tiles are walked in groups of 8 tile-rows for L2 reuse, and dealt to the
// XCDs in chunks of consecutive tiles (the dispatcher deals workgroups
// round-robin over the 8 XCDs, each with its own L2): workgroup b runs tile
// t = ((b/8) / CH * 8 + b%8) * CH + (b/8) % CH, so each XCD walks its own
// chunks in order and shares operands within a chunk, while every XCD gets
// chunks from all over the tile grid.  The last matters for triangular
// launches (lower C, triangular operands), whose work per tile row grows
// down the grid: contiguous eighths of the grid per XCD leave the last XCD
// with most of the work.
#include "common.h"

namespace mm {
namespace {

constexpr int BK = 16;    // k-slice per LDS stage
constexpr int PAD = 2;    // LDS row padding (doubles): conflict-free k-major stores
constexpr int GROUP_M = 8;

struct KArgs {
  int64_t m, n, k;
  double alpha, beta;
  const double* A;
  int64_t lda;
  const double* B;
  int64_t ldb;
  double* C;
  int64_t ldc;
  int lower, a_lower, a_upper, b_lower, a_sym;
  int64_t b_band;
  int64_t sA, sB, sC;
  int splits;
  double* ws;
  const GemmGroup* groups;
  int tiles_m, tiles_n;  // tile grid the launch covers
  int ch_log2;           // log2 of the tiles per chunk dealt to one XCD
};

// The tile of workgroup bid; false for the padding of the grid (a multiple of
// 8 chunks).
__device__ __forceinline__ bool tile_of(int bid, int tiles_m, int tiles_n, int ch_log2,
                                        int& ti, int& tj) {
  const int T = tiles_m * tiles_n;
  const int xcd = bid & 7, local = bid >> 3;
  const int chunk = ((local >> ch_log2) << 3) + xcd;
  const int t = (chunk << ch_log2) + (local & ((1 << ch_log2) - 1));
  if (t >= T) return false;
  // grouped ordering along M
  const int per_group = GROUP_M * tiles_n;
  const int g = t / per_group;
  const int first_m = g * GROUP_M;
  const int gsz = min(tiles_m - first_m, GROUP_M);
  const int w = t - g * per_group;
  ti = first_m + w % gsz;
  tj = w / gsz;
  return true;
}

// Chunk size for T tiles: the largest power of two up to 16 that still gives
// every XCD at least 16 chunks (a partial last round of chunks then costs an
// XCD at most 1/16 of its share).  16 rather than 64: the finer deal lifts a
// lower-triangular rank-512 update from 52 to 57 TFLOP/s and leaves full
// products unchanged.
int chunk_log2(int64_t T) {
  int c = 4;
  while (c > 0 && ((int64_t)8 * 16) << c > T) --c;
  return c;
}

// Workgroups of a launch over T tiles: T rounded up to 8 chunks.
int64_t padded_tiles(int64_t T, int ch_log2) {
  const int64_t q = (int64_t)8 << ch_log2;
  return ceil_div(T, q) * q;
}

#ifndef MM_GEMM_WPE
#define MM_GEMM_WPE 2
#endif
template <int BM, int BN, int WGM, int WGN, bool TA, bool TB, bool GROUPED>
__global__ void __launch_bounds__(64 * WGM * WGN)
    __attribute__((amdgpu_waves_per_eu(MM_GEMM_WPE))) gemm_kernel(KArgs a) {
  constexpr int NT = 64 * WGM * WGN;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int LA = BM * BK / NT;  // A elements loaded per thread per slice
  constexpr int LB = BN * BK / NT;
  __shared__ double As[2][BK][BM + PAD];
  __shared__ double Bs[2][BK][BN + PAD];

  int64_t M, N, K, lda, ldb, ldc;
  const double* A;
  const double* B;
  double* C;
  if constexpr (GROUPED) {
    const GemmGroup g = a.groups[blockIdx.y];
    M = g.m; N = g.n; K = g.k; lda = g.lda; ldb = g.ldb; ldc = g.ldc;
    A = g.A; B = g.B; C = g.C;
  } else {
    M = a.m; N = a.n; K = a.k; lda = a.lda; ldb = a.ldb; ldc = a.ldc;
    A = a.A + (int64_t)blockIdx.y * a.sA;
    B = a.B + (int64_t)blockIdx.y * a.sB;
    C = a.C + (int64_t)blockIdx.y * a.sC;
  }
  int ti, tj;
  if (!tile_of(blockIdx.x, a.tiles_m, a.tiles_n, a.ch_log2, ti, tj)) return;
  const int64_t i0 = (int64_t)ti * BM, j0 = (int64_t)tj * BN;
  if (i0 >= M || j0 >= N) return;
  if (a.lower && i0 + BM <= j0) return;  // tile strictly above the diagonal

  int64_t kb = 0, ke = K;
  if (a.a_lower) ke = min(ke, i0 + BM);
  if (a.b_band >= 0) ke = min(ke, j0 + BN + a.b_band);
  if (a.a_upper) kb = max(kb, i0);
  if (a.b_lower) kb = max(kb, j0);
  kb = (kb / BK) * BK;
  if (a.splits > 1) {
    const int64_t span = ke > kb ? ke - kb : 0;
    const int64_t chunk = ceil_div(ceil_div(span, a.splits), BK) * BK;
    const int64_t s0 = kb + (int64_t)blockIdx.z * chunk;
    kb = s0;
    ke = min(ke, s0 + chunk);
  }

  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm0 = (wave % WGM) * WM, wn0 = (wave / WGM) * WN;
  const int lr = lane & 15, lk = lane >> 4;

  v4d acc[FM][FN];
#pragma unroll
  for (int x = 0; x < FM; ++x)
#pragma unroll
    for (int y = 0; y < FN; ++y) acc[x][y] = v4d{0.0, 0.0, 0.0, 0.0};

  double ra[LA], rb[LB];

  // Operand loads.  With e = t + r NT the element of load r is a per-lane
  // base plus r times a wave-uniform stride in every layout, so interior
  // slices load unguarded from one base pointer; edge slices are guarded.
  constexpr int64_t RA = TA ? (NT / BK) : (NT / BM);  // op(A) rows/cols per r
  constexpr int64_t RB = TB ? (NT / BN) : (NT / BK);
  constexpr bool FAST = BM >= 128;  // the small tile keeps the guarded loads
  // A symmetric in its lower triangle (not TA): a slice that reaches above the
  // diagonal is read from the transposed position.  Slices wholly above it
  // load k-contiguous (the TA pattern, recorded in ltr for the LDS store);
  // slices that cross the diagonal pick per element.
  bool ltr = false;
  auto load = [&](int64_t kt) {
    bool sym_done = false;
    if constexpr (!TA) {
      if (a.a_sym && kt + BK - 1 > i0) {
        sym_done = true;
        if (kt >= i0 + BM - 1 && i0 + BM <= M && kt + BK <= ke) {
          ltr = true;
          const double* Ap = A + (kt + t % BK) + (i0 + t / BK) * lda;
#pragma unroll
          for (int r = 0; r < LA; ++r) ra[r] = Ap[(int64_t)r * (NT / BK) * lda];
        } else {
          ltr = false;
#pragma unroll
          for (int r = 0; r < LA; ++r) {
            const int e = t + r * NT;
            const int64_t gi = i0 + e % BM, gk = kt + e / BM;
            double v = 0.0;
            if (gi < M && gk < ke) v = gi >= gk ? A[gi + gk * lda] : A[gk + gi * lda];
            ra[r] = v;
          }
        }
      }
    }
    if (sym_done) {
    } else if (FAST && i0 + BM <= M && kt + BK <= ke) {
      ltr = false;
      const double* Ap = TA ? A + (kt + t % BK) + (i0 + t / BK) * lda
                            : A + (i0 + t % BM) + (kt + t / BM) * lda;
#pragma unroll
      for (int r = 0; r < LA; ++r) ra[r] = Ap[r * RA * lda];
    } else {
      ltr = false;
#pragma unroll
      for (int r = 0; r < LA; ++r) {
        const int e = t + r * NT;
        int ii, kk;
        if constexpr (!TA) { ii = e % BM; kk = e / BM; }
        else { kk = e % BK; ii = e / BK; }
        const int64_t gi = i0 + ii, gk = kt + kk;
        double v = 0.0;
        if (gi < M && gk < ke)
          v = TA ? A[gk + gi * lda] : A[gi + gk * lda];
        ra[r] = v;
      }
    }
    if (FAST && j0 + BN <= N && kt + BK <= ke) {
      const double* Bp = TB ? B + (j0 + t % BN) + (kt + t / BN) * ldb
                            : B + (kt + t % BK) + (j0 + t / BK) * ldb;
#pragma unroll
      for (int r = 0; r < LB; ++r) rb[r] = Bp[r * RB * ldb];
    } else {
#pragma unroll
      for (int r = 0; r < LB; ++r) {
        const int e = t + r * NT;
        int jj, kk;
        if constexpr (!TB) { kk = e % BK; jj = e / BK; }
        else { jj = e % BN; kk = e / BN; }
        const int64_t gj = j0 + jj, gk = kt + kk;
        double v = 0.0;
        if (gj < N && gk < ke)
          v = TB ? B[gj + gk * ldb] : B[gk + gj * ldb];
        rb[r] = v;
      }
    }
  };
  auto store = [&](int buf) {
    if (!TA && ltr) {
#pragma unroll
      for (int r = 0; r < LA; ++r) {
        const int e = t + r * NT;
        As[buf][e % BK][e / BK] = ra[r];
      }
    } else {
#pragma unroll
      for (int r = 0; r < LA; ++r) {
        const int e = t + r * NT;
        int ii, kk;
        if constexpr (!TA) { ii = e % BM; kk = e / BM; }
        else { kk = e % BK; ii = e / BK; }
        As[buf][kk][ii] = ra[r];
      }
    }
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      const int e = t + r * NT;
      int jj, kk;
      if constexpr (!TB) { kk = e % BK; jj = e / BK; }
      else { jj = e % BN; kk = e / BN; }
      Bs[buf][kk][jj] = rb[r];
    }
  };

  if (ke > kb) {
    load(kb);
    store(0);
    __syncthreads();
    int cur = 0;
    for (int64_t kt = kb; kt < ke; kt += BK) {
      const bool more = kt + BK < ke;
      if (more) load(kt + BK);
#pragma unroll
      for (int kk = 0; kk < BK / 4; ++kk) {
        double av[FM], bv[FN];
#pragma unroll
        for (int x = 0; x < FM; ++x) av[x] = As[cur][kk * 4 + lk][wm0 + x * 16 + lr];
#pragma unroll
        for (int y = 0; y < FN; ++y) bv[y] = Bs[cur][kk * 4 + lk][wn0 + y * 16 + lr];
#pragma unroll
        for (int x = 0; x < FM; ++x)
#pragma unroll
          for (int y = 0; y < FN; ++y)
            acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[y], av[x], acc[x][y], 0, 0, 0);
      }
      if (more) store(cur ^ 1);
      __syncthreads();
      cur ^= 1;
    }
  }

  // Epilogue.  v_mfma_f64_16x16x4 leaves D(l/16 + 4q, l%16) in result q of
  // lane l; with B fed first, D is the transposed tile, so lane l holds
  // C(i0 + wm0 + 16x + lr, j0 + wn0 + 16y + lk + 4q), q < 4.
  if (a.splits > 1) {
    double* W = a.ws + (int64_t)blockIdx.z * M * N;
#pragma unroll
    for (int x = 0; x < FM; ++x)
#pragma unroll
      for (int y = 0; y < FN; ++y)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t gi = i0 + wm0 + x * 16 + lr;
          const int64_t gj = j0 + wn0 + y * 16 + lk + 4 * q;
          if (gi < M && gj < N) W[gi + gj * M] = a.alpha * acc[x][y][q];
        }
    return;
  }
  // C = alpha acc + beta C.  Interior tiles: the C values of half the wave's
  // tile are loaded together before any is used (two memory latencies per
  // tile, not one per element), addressed from one per-lane base pointer and
  // wave-uniform offsets.  Edge tiles take the guarded element-wise path.
  const bool full = i0 + BM <= M && j0 + BN <= N && (!a.lower || i0 >= j0 + BN - 1);
  const double alpha = a.alpha, beta = a.beta;
  if (full) {
    double* Cb = C + (i0 + wm0 + lr) + (j0 + wn0 + lk) * ldc;
#pragma unroll
    for (int xh = 0; xh < FM; xh += FM / 2) {
      __builtin_amdgcn_sched_barrier(0);
      double cv[FM / 2][FN][4];
      if (beta != 0.0) {
#pragma unroll
        for (int x = 0; x < FM / 2; ++x)
#pragma unroll
          for (int y = 0; y < FN; ++y)
#pragma unroll
            for (int q = 0; q < 4; ++q)
              cv[x][y][q] = Cb[(xh + x) * 16 + (int64_t)(y * 16 + 4 * q) * ldc];
      }
#pragma unroll
      for (int x = 0; x < FM / 2; ++x)
#pragma unroll
        for (int y = 0; y < FN; ++y)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            double v = alpha * acc[xh + x][y][q];
            if (beta != 0.0) v += beta * cv[x][y][q];
            Cb[(xh + x) * 16 + (int64_t)(y * 16 + 4 * q) * ldc] = v;
          }
    }
    return;
  }
#pragma unroll
  for (int x = 0; x < FM; ++x)
#pragma unroll
    for (int y = 0; y < FN; ++y)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t gi = i0 + wm0 + x * 16 + lr;
        const int64_t gj = j0 + wn0 + y * 16 + lk + 4 * q;
        if (gi < M && gj < N && (!a.lower || gi >= gj)) {
          double v = alpha * acc[x][y][q];
          if (beta != 0.0) v += beta * C[gi + gj * ldc];
          C[gi + gj * ldc] = v;
        }
      }
}

// ---------------------------------------------------------------------------
// Large tiles: 128 x 128 per workgroup of four waves, 64 x 64 per wave (16
// MFMA accumulators, so each operand value read from LDS feeds four MFMAs),
// or 128 x 64 with 64 x 32 per wave for products with at most 64 columns.
// Every operand and C access is a buffer instruction on a uniform base (the
// slice's or the tile's corner) with one 32-bit per-lane offset and a uniform
// per-element offset, so that addresses take no 64-bit vector registers.
// Interior slices load unguarded; edge slices clamp their addresses to the
// matrix and zero the entries at k >= ke.
//
// Load patterns of one 128 x 16 slice (256 threads, 8 elements each; a
// 64 x 16 slice of B likewise with 4):
//   column pattern: thread t holds row t%128 of k = t/128 + 2r (r < 8);
//   row pattern:    thread t holds k = t%16 of row t/16 + 16r.
// op(A) untransposed and op(B) transposed are read column-wise, the others
// row-wise; with a_sym, a slice wholly above the diagonal is read row-wise
// from the transposed position and one that crosses it element by element.
// ---------------------------------------------------------------------------
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int kRsrcFlags = 0x00020000;  // gfx9 buffer resource word 3

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_of(const double* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(p), (short)0, 0x7fffffff,
                                           kRsrcFlags);
}
__device__ __forceinline__ double bld(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void bst(double v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
}

// An R x 16 slice (R = 128 or 64) of a matrix X read column-wise by 256
// threads: element (i, k) at X0 + i + k ld; thread t holds i = t % R of
// k = t / R + (256 / R) q.  ni valid rows, nk valid k (the rest clamped and,
// past nk, zeroed).
template <int R>
__device__ __forceinline__ void load_col(double* r, const double* X0, int ld, int ni, int nk,
                                         int t) {
  constexpr int S = 256 / R, NL = R / 16;
  const __amdgpu_buffer_rsrc_t rs = rsrc_of(X0);
  const int ci0 = t % R, ck0 = t / R;
  if (ni == R && nk == BK) {
    const int v = (ci0 + ck0 * ld) * 8;
#pragma unroll
    for (int q = 0; q < NL; ++q) r[q] = bld(rs, v, q * S * ld * 8);
  } else {
    const int ci = min(ci0, ni - 1);
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int k = ck0 + S * q;
      const double x = bld(rs, (ci + min(k, nk - 1) * ld) * 8, 0);
      r[q] = k < nk ? x : 0.0;
    }
  }
}
// The same slice read row-wise: element (i, k) at X0 + k + i ld; thread t
// holds k = t % 16 of row t / 16 + 16 q.
template <int R>
__device__ __forceinline__ void load_row(double* r, const double* X0, int ld, int ni, int nk,
                                         int t) {
  constexpr int NL = R / 16;
  const __amdgpu_buffer_rsrc_t rs = rsrc_of(X0);
  const int rk = t & 15, ri = t >> 4;
  if (ni == R && nk == BK) {
    const int v = (rk + ri * ld) * 8;
#pragma unroll
    for (int q = 0; q < NL; ++q) r[q] = bld(rs, v, q * 16 * ld * 8);
  } else {
    const int ck = min(rk, nk - 1);
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int i = min(ri + 16 * q, ni - 1);
      const double x = bld(rs, (ck + i * ld) * 8, 0);
      r[q] = rk < nk ? x : 0.0;
    }
  }
}
// LDS image S[k][i] of a slice held in the column or the row pattern
template <int R>
__device__ __forceinline__ void store_col(double (*S)[R + PAD], const double* r, int t) {
  constexpr int ST = 256 / R, NL = R / 16;
#pragma unroll
  for (int q = 0; q < NL; ++q) S[t / R + ST * q][t % R] = r[q];
}
template <int R>
__device__ __forceinline__ void store_row(double (*S)[R + PAD], const double* r, int t) {
  constexpr int NL = R / 16;
#pragma unroll
  for (int q = 0; q < NL; ++q) S[t & 15][(t >> 4) + 16 * q] = r[q];
}

// BN = 128: four waves of 64 x 64 (two workgroups per CU); BN = 64: four
// waves of 64 x 32 (three per CU), for products with at most 64 columns.
template <int BN, bool TA, bool TB, bool SYM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BN == 64 ? 3 : 2)))
    gemm_big_kernel(KArgs a) {
  constexpr int BM = 128, FN = BN / 32, LA = BM / 16, LB = BN / 16;
  __shared__ double As[2][BK][BM + PAD];
  __shared__ double Bs[2][BK][BN + PAD];
  const int64_t M = a.m, N = a.n, K = a.k, lda = a.lda, ldb = a.ldb, ldc = a.ldc;
  const double* A = a.A + (int64_t)blockIdx.y * a.sA;
  const double* B = a.B + (int64_t)blockIdx.y * a.sB;
  double* C = a.C + (int64_t)blockIdx.y * a.sC;
  int ti, tj;
  if (!tile_of(blockIdx.x, a.tiles_m, a.tiles_n, a.ch_log2, ti, tj)) return;
  const int64_t i0 = (int64_t)ti * BM, j0 = (int64_t)tj * BN;
  if (i0 >= M || j0 >= N) return;
  if (a.lower && i0 + BM <= j0) return;  // tile strictly above the diagonal
  int64_t kb = 0, ke = K;
  if (a.a_lower) ke = min(ke, i0 + BM);
  if (a.b_band >= 0) ke = min(ke, j0 + BN + a.b_band);
  if (a.a_upper) kb = max(kb, i0);
  if (a.b_lower) kb = max(kb, j0);
  kb = (kb / BK) * BK;
  if (a.splits > 1) {  // this workgroup's share of k (blockIdx.z)
    const int64_t span = ke > kb ? ke - kb : 0;
    const int64_t chunk = ceil_div(ceil_div(span, a.splits), BK) * BK;
    const int64_t s0 = kb + (int64_t)blockIdx.z * chunk;
    kb = s0;
    ke = min(ke, s0 + chunk);
  }

  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm0 = (wave & 1) * 64, wn0 = (wave >> 1) * (BN / 2);
  const int lr = lane & 15, lk = lane >> 4;
  const int iM = (int)min<int64_t>(BM, M - i0);  // rows of the tile inside C
  const int jN = (int)min<int64_t>(BN, N - j0);
  const int la = (int)lda, lb = (int)ldb;

  v4d acc[4][FN];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < FN; ++y) acc[x][y] = v4d{0.0, 0.0, 0.0, 0.0};

  double ra[LA], rb[LB];
  bool a_row = TA;  // pattern of the A slice in ra

  auto load = [&](int64_t kt) {
    const int nk = (int)min<int64_t>(BK, ke - kt);
    if constexpr (SYM) {
      if (kt + BK - 1 <= i0) {  // below the diagonal
        a_row = false;
        load_col<BM>(ra, A + i0 + kt * lda, la, iM, nk, t);
      } else if (kt >= i0 + BM - 1) {  // above it: A(k, i)
        a_row = true;
        load_row<BM>(ra, A + kt + i0 * lda, la, iM, nk, t);
      } else {  // crossing it: per element, from the corner b = min(i0, kt)
        a_row = false;
        const int64_t b = min(i0, kt);
        const __amdgpu_buffer_rsrc_t rs = rsrc_of(A + b + b * lda);
        const int gi = (int)(i0 - b) + min(t & 127, iM - 1);
#pragma unroll
        for (int q = 0; q < LA; ++q) {
          const int k = (t >> 7) + 2 * q;
          const int gk = (int)(kt - b) + min(k, nk - 1);
          const int rr = gi >= gk ? gi : gk, cc = gi >= gk ? gk : gi;
          const double x = bld(rs, (rr + cc * la) * 8, 0);
          ra[q] = k < nk ? x : 0.0;
        }
      }
    } else if constexpr (TA) {
      load_row<BM>(ra, A + kt + i0 * lda, la, iM, nk, t);
    } else {
      load_col<BM>(ra, A + i0 + kt * lda, la, iM, nk, t);
    }
    if constexpr (TB) load_col<BN>(rb, B + j0 + kt * ldb, lb, jN, nk, t);
    else load_row<BN>(rb, B + kt + j0 * ldb, lb, jN, nk, t);
  };
  auto store = [&](int buf) {
    if (a_row) store_row<BM>(As[buf], ra, t);
    else store_col<BM>(As[buf], ra, t);
    if constexpr (TB) store_col<BN>(Bs[buf], rb, t);
    else store_row<BN>(Bs[buf], rb, t);
  };

  if (ke > kb) {
    load(kb);
    store(0);
    __syncthreads();
    int cur = 0;
    for (int64_t kt = kb; kt < ke; kt += BK) {
      const bool more = kt + BK < ke;
      if (more) load(kt + BK);
#pragma unroll
      for (int kk = 0; kk < BK / 4; ++kk) {
        double av[4], bv[FN];
#pragma unroll
        for (int x = 0; x < 4; ++x) av[x] = As[cur][kk * 4 + lk][wm0 + x * 16 + lr];
#pragma unroll
        for (int y = 0; y < FN; ++y) bv[y] = Bs[cur][kk * 4 + lk][wn0 + y * 16 + lr];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < FN; ++y)
            acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[y], av[x], acc[x][y], 0, 0, 0);
      }
      if (more) store(cur ^ 1);
      __syncthreads();
      cur ^= 1;
    }
  }

  // Epilogue: lane l holds C(i0 + wm0 + 16x + lr, j0 + wn0 + 16y + lk + 4q).
  const double alpha = a.alpha, beta = a.beta;
  if (a.splits > 1) {  // partial sums W_z (M x N, ld M), reduced afterwards
    const __amdgpu_buffer_rsrc_t rw = rsrc_of(a.ws + (int64_t)blockIdx.z * M * N + i0 + j0 * M);
    const int lm = (int)M;
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < FN; ++y)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int li = wm0 + x * 16 + lr, lj = wn0 + y * 16 + lk + 4 * q;
          if (li < iM && lj < jN) bst(alpha * acc[x][y][q], rw, (li + lj * lm) * 8, 0);
        }
    return;
  }
  const __amdgpu_buffer_rsrc_t rc = rsrc_of(C + i0 + j0 * ldc);
  const int lc = (int)ldc;
  const int vc = ((wm0 + lr) + (wn0 + lk) * lc) * 8;
  const bool full = iM == BM && jN == BN && (!a.lower || i0 >= j0 + BN - 1);
  if (full) {
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      double cv[FN][4];
      if (beta != 0.0) {
#pragma unroll
        for (int y = 0; y < FN; ++y)
#pragma unroll
          for (int q = 0; q < 4; ++q) cv[y][q] = bld(rc, vc, (x * 16 + (y * 16 + 4 * q) * lc) * 8);
      }
#pragma unroll
      for (int y = 0; y < FN; ++y)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          double v = alpha * acc[x][y][q];
          if (beta != 0.0) v += beta * cv[y][q];
          bst(v, rc, vc, (x * 16 + (y * 16 + 4 * q) * lc) * 8);
        }
    }
    return;
  }
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < FN; ++y)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int li = wm0 + x * 16 + lr, lj = wn0 + y * 16 + lk + 4 * q;
        if (li < iM && lj < jN && (!a.lower || i0 + li >= j0 + lj)) {
          const int off = (li + lj * lc) * 8;
          double v = alpha * acc[x][y][q];
          if (beta != 0.0) v += beta * bld(rc, off, 0);
          bst(v, rc, off, 0);
        }
      }
}

// split-K of the 128-row-tile products: enough shares for this many rounds
// of resident workgroups, at most MM_GEMM_SPLIT_MAX, each at least
// MM_GEMM_SPLIT_MINK of k
#ifndef MM_GEMM_SPLIT_ROUNDS
#define MM_GEMM_SPLIT_ROUNDS 12
#endif
#ifndef MM_GEMM_SPLIT_MAX
#define MM_GEMM_SPLIT_MAX 32
#endif
#ifndef MM_GEMM_SPLIT_MINK
#define MM_GEMM_SPLIT_MINK 2048
#endif

template <int BN>
void launch_big(const KArgs& ka, bool ta, bool tb, bool sym, dim3 grid, hipStream_t s) {
  const dim3 block(256);
  if (sym) hipLaunchKernelGGL((gemm_big_kernel<BN, false, false, true>), grid, block, 0, s, ka);
  else if (!ta && !tb) hipLaunchKernelGGL((gemm_big_kernel<BN, false, false, false>), grid, block, 0, s, ka);
  else if (!ta && tb) hipLaunchKernelGGL((gemm_big_kernel<BN, false, true, false>), grid, block, 0, s, ka);
  else if (ta && !tb) hipLaunchKernelGGL((gemm_big_kernel<BN, true, false, false>), grid, block, 0, s, ka);
  else hipLaunchKernelGGL((gemm_big_kernel<BN, true, true, false>), grid, block, 0, s, ka);
}

// C = beta C + sum_z W_z in a fixed order (deterministic split-K): 64
// consecutive outputs per workgroup (lane = output, coalesced reads), wave w
// sums the partials z = w, w + 4, ... in ascending z, and the four wave sums
// are added in wave order.
__global__ void __launch_bounds__(256) splitk_reduce(int64_t M, int64_t N, int splits,
                                                     const double* W, double beta, double* C,
                                                     int64_t ldc, int lower) {
  __shared__ double part[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t idx = (int64_t)blockIdx.x * 64 + lane;
  const int64_t MN = M * N;
  double s = 0.0;
  if (idx < MN) {
    int z = wave;
    for (; z + 12 < splits; z += 16) {  // four loads in flight
      const double a = W[(int64_t)z * MN + idx], b = W[(int64_t)(z + 4) * MN + idx];
      const double c = W[(int64_t)(z + 8) * MN + idx], d = W[(int64_t)(z + 12) * MN + idx];
      s = (((s + a) + b) + c) + d;
    }
    for (; z < splits; z += 4) s += W[(int64_t)z * MN + idx];
  }
  part[wave][lane] = s;
  __syncthreads();
  if (wave != 0 || idx >= MN) return;
  const int64_t i = idx % M, j = idx / M;
  if (lower && i < j) return;
  double r = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
  if (beta != 0.0) r += beta * C[i + j * ldc];
  C[i + j * ldc] = r;
}

template <int BM, int BN, int WGM, int WGN, bool GROUPED>
void launch(const KArgs& ka, bool ta, bool tb, dim3 grid, hipStream_t s) {
  const dim3 block(64 * WGM * WGN);
  if (!ta && !tb) hipLaunchKernelGGL((gemm_kernel<BM, BN, WGM, WGN, false, false, GROUPED>), grid, block, 0, s, ka);
  else if (!ta && tb) hipLaunchKernelGGL((gemm_kernel<BM, BN, WGM, WGN, false, true, GROUPED>), grid, block, 0, s, ka);
  else if (ta && !tb) hipLaunchKernelGGL((gemm_kernel<BM, BN, WGM, WGN, true, false, GROUPED>), grid, block, 0, s, ka);
  else hipLaunchKernelGGL((gemm_kernel<BM, BN, WGM, WGN, true, true, GROUPED>), grid, block, 0, s, ka);
}

// Tile of the large configuration.
#ifndef MM_GEMM_BIG
#define MM_GEMM_BIG 128, 64, 4, 2
#endif
template <int BM_, int BN_, int WGM_, int WGN_>
struct Cfg {
  static constexpr int BM = BM_, BN = BN_, WGM = WGM_, WGN = WGN_;
};
using Big = Cfg<MM_GEMM_BIG>;

}  // namespace

void gemm(const Gemm& g, hipStream_t stream, double* ws, int64_t ws_elems) {
  if (g.m <= 0 || g.n <= 0 || g.batch <= 0) return;
  MM_REQUIRE(g.A != nullptr || g.k == 0, kInvalid, "gemm: null A");
  MM_REQUIRE(g.C != nullptr, kInvalid, "gemm: null C");
  KArgs ka{};
  ka.m = g.m; ka.n = g.n; ka.k = g.k;
  ka.alpha = g.alpha; ka.beta = g.beta;
  ka.A = g.A; ka.lda = g.lda; ka.B = g.B; ka.ldb = g.ldb;
  ka.C = g.C; ka.ldc = g.ldc;
  ka.lower = g.lower; ka.a_lower = g.a_lower; ka.a_upper = g.a_upper;
  ka.b_lower = g.b_lower; ka.b_band = g.b_band;
  ka.a_sym = g.a_sym;
  MM_REQUIRE(!g.a_sym || (!g.ta && !g.tb && !g.a_lower && !g.a_upper && g.m == g.k), kInvalid,
             "gemm: a_sym takes A and B untransposed and no triangle flags for A");
  ka.sA = g.sA; ka.sB = g.sB; ka.sC = g.sC;
  ka.splits = 1; ka.ws = nullptr; ka.groups = nullptr;
  if (g.k <= 0) {
    ka.k = 0;  // C = beta C through the epilogue
  }
  const bool big = g.m * g.n >= (int64_t)256 * 128 * 128;
  const int bm = big ? Big::BM : 64, bn = big ? Big::BN : 64;
  ka.tiles_m = (int)ceil_div(g.m, bm);
  ka.tiles_n = (int)ceil_div(g.n, bn);
  const int64_t tiles = (int64_t)ka.tiles_m * ka.tiles_n;
  ka.ch_log2 = chunk_log2(tiles);
  const int64_t wgs = padded_tiles(tiles, ka.ch_log2);
  MM_REQUIRE(wgs < (int64_t)1 << 31, kInvalid, "gemm: too many tiles");
  // split-K for few output tiles over a long k (never together with batching):
  // at least 128 of k per workgroup (eight slices: each workgroup's slices
  // are latency-bound, so many short shares beat few long ones)
  int splits = 1;
  if (ws && g.batch == 1 && tiles * 4 < 1024 && g.k >= 2048) {
    splits = (int)std::min<int64_t>(ceil_div(1024, tiles), g.k / 128);
    const int64_t cap = ws_elems / (g.m * g.n);
    splits = (int)std::min<int64_t>(splits, cap);
    if (splits < 2) splits = 1;
  }
  ka.splits = splits;
  ka.ws = splits > 1 ? ws : nullptr;
  // 128-row tiles (128 x 128, or 128 x 64 for at most 64 columns): at least
  // a million outputs, and 32-bit byte offsets across 256 rows or columns of
  // every operand (and of the split-K partials)
  const int64_t ldmax = std::max(std::max(std::max(g.lda, g.ldb), g.ldc), g.m);
  if (g.m >= 128 && g.n >= 64 && g.m * g.n >= ((int64_t)1 << 20) &&
      ldmax * 256 * 8 < ((int64_t)1 << 31)) {
    // 128 x 64 also for short updates (k <= 256): three workgroups per CU
    // overlap one another's C traffic better (3 % faster at k = 128)
    const int bnb = (g.n <= 64 || g.k <= 256) ? 64 : 128;
    ka.tiles_m = (int)ceil_div(g.m, 128);
    ka.tiles_n = (int)ceil_div(g.n, bnb);
    const int64_t tb = (int64_t)ka.tiles_m * ka.tiles_n;
    // split-K when a long-k product has fewer tiles than twelve rounds of
    // resident workgroups (three 128 x 64 or two 128 x 128 per CU): tall,
    // narrow products with k = m, such as the band reduction's A22 V.  Many
    // shares of at least 2048 of k each run faster than few long ones (the
    // paper-scale band reduction: 28.1 s with two rounds, 26.7 s with twelve),
    // their workgroups reading A at many distant places at once.
    const int64_t slots = MM_GEMM_SPLIT_ROUNDS * (bnb == 64 ? 768 : 512);
    int sp = 1;
    if (ws && g.batch == 1 && g.k >= 4096 && tb < slots) {
      sp = (int)std::min<int64_t>(std::min<int64_t>(ceil_div(slots, tb), g.k / MM_GEMM_SPLIT_MINK),
                                  std::min<int64_t>(ws_elems / (g.m * g.n), MM_GEMM_SPLIT_MAX));
      if (sp < 2) sp = 1;
    }
    ka.splits = sp;
    ka.ws = sp > 1 ? ws : nullptr;
    ka.ch_log2 = chunk_log2(tb);
    const dim3 gb((unsigned)padded_tiles(tb, ka.ch_log2), (unsigned)g.batch, (unsigned)sp);
    if (bnb == 64) launch_big<64>(ka, g.ta, g.tb, g.a_sym, gb, stream);
    else launch_big<128>(ka, g.ta, g.tb, g.a_sym, gb, stream);
    MM_HIP_TRY(hipGetLastError());
    if (sp > 1) {
      const int64_t total = g.m * g.n;
      hipLaunchKernelGGL(splitk_reduce, dim3((unsigned)ceil_div(total, 64)), dim3(256), 0, stream,
                         g.m, g.n, sp, ws, g.beta, g.C, g.ldc, (int)g.lower);
      MM_HIP_TRY(hipGetLastError());
    }
    return;
  }
  dim3 grid((unsigned)wgs, (unsigned)g.batch, (unsigned)splits);
  if (big) launch<Big::BM, Big::BN, Big::WGM, Big::WGN, false>(ka, g.ta, g.tb, grid, stream);
  else launch<64, 64, 2, 2, false>(ka, g.ta, g.tb, grid, stream);
  MM_HIP_TRY(hipGetLastError());
  if (splits > 1) {
    const int64_t total = g.m * g.n;
    hipLaunchKernelGGL(splitk_reduce, dim3((unsigned)ceil_div(total, 64)), dim3(256), 0, stream,
                       g.m, g.n, splits, ws, g.beta, g.C, g.ldc, (int)g.lower);
    MM_HIP_TRY(hipGetLastError());
  }
}

void gemm_grouped(const GemmGroup* d_groups, int64_t n_groups, int64_t max_m,
                  int64_t max_n, bool ta, bool tb, double alpha, double beta,
                  hipStream_t stream) {
  if (n_groups <= 0 || max_m <= 0 || max_n <= 0) return;
  KArgs ka{};
  ka.alpha = alpha; ka.beta = beta; ka.splits = 1; ka.b_band = -1;
  ka.groups = d_groups;
  const bool big = max_m * max_n >= (int64_t)64 * 128 * 128;
  const int bm = big ? Big::BM : 64, bn = big ? Big::BN : 64;
  ka.tiles_m = (int)ceil_div(max_m, bm);
  ka.tiles_n = (int)ceil_div(max_n, bn);
  const int64_t tiles = (int64_t)ka.tiles_m * ka.tiles_n;
  ka.ch_log2 = chunk_log2(tiles);
  const int64_t wgs = padded_tiles(tiles, ka.ch_log2);
  MM_REQUIRE(wgs < (int64_t)1 << 31, kInvalid, "gemm_grouped: too many tiles");
  dim3 grid((unsigned)wgs, (unsigned)n_groups, 1);
  if (big) launch<Big::BM, Big::BN, Big::WGM, Big::WGN, true>(ka, ta, tb, grid, stream);
  else launch<64, 64, 2, 2, true>(ka, ta, tb, grid, stream);
  MM_HIP_TRY(hipGetLastError());
}

}  // namespace mm
