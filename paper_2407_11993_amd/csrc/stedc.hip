// Divide and conquer for the symmetric tridiagonal eigenproblem T = Z Lam Z^T
// (Cuppen's method with the stable eigenvectors of Gu & Eisenstat).
//
// Tearing.  Every node of a balanced binary tree over [0, n) is cut at its
// midpoint m:  T = diag(T1, T2) + rho u u^T  with  rho = |e_{m-1}|,
// u = e_{m-1} + sign(e_{m-1}) e_m, and the two diagonal entries next to the
// cut lowered by rho.  Leaves (<= 32 rows) are solved by cyclic Jacobi in LDS.
//
// Merging (one level of the tree per round, all merges of a level batched):
//   z = [last row of Z1, sign(e) first row of Z2] / sqrt(2),  rho <- 2 rho,
//   D = eig(T1) U eig(T2) sorted;  deflation (sequential scan, one thread per
//   merge): tiny rho|z_i| or a negligible coupling after a Givens rotation of
//   two close entries; the roots of 1/rho + sum z_i^2/(d_i - x) = 0 are found
//   one per thread (shift to the nearer pole, bisection guarded by a two-pole
//   rational model); z is recomputed from the roots (Lowner: the computed
//   roots are exact for a nearby z, which keeps the vectors orthogonal);
//   U(i,j) = zhat_i / (d_i - lam_j) normalised;  Z_new = Z_kept U (matrix
//   cores);  and the merged spectrum is sorted into place.
//
// Every node keeps, row q for its q-th eigenvector, two boundary columns
// Z_node^T e_first, Z_node^T e_last (its eigenvectors' first and last
// entries, which the parent's z needs) and, in projected mode
// (stedc_project), the projections Z_node^T Y_node for a few columns Y.  A
// merge applies its rotations to rows, U^T to the kept rows, copies the
// deflated ones and sorts rows into place.
//
// Eigenvector mode (stedc) never stores the tree's eigenvectors Z.  Z is the
// product Z_leaves M_{D-1} ... M_0 of the leaves' block-diagonal eigenvectors
// and one block-diagonal factor per level (a merge's rotations, its U on the
// kept columns and the sort), so X <- X Z is taken from the left: X receives
// Z_leaves, a caller hook may transform it (the eigensolver applies Q1 Q2
// there, so that X ends as Q1 Q2 Z), and every level's merges are applied to
// X's columns in chunks of rows (gather the node's columns in merge order,
// one grouped product with U, scatter them to their sorted places).  Besides
// X this needs U (n^2, the caller's scratch) and two row chunks.
#include "eig.h"

#include <functional>
#include <vector>

namespace mm {
namespace {

constexpr int LEAF = 32;
constexpr int NT = 256;
constexpr double EPS = 2.220446049250313e-16;

struct Merge {
  int64_t lo, mid, hi;  // children [lo, mid), [mid, hi)
};

// ---------------------------------------------------------------------------
// tearing: lower the diagonal next to every cut
// ---------------------------------------------------------------------------
__global__ void tear_k(const double* d, const double* e, int64_t n, const int64_t* cuts,
                       int64_t ncuts, double* dw) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    double v = d[i];
    // a position is next to at most two cuts (at i and at i+1)
    for (int64_t q = 0; q < ncuts; ++q) {
      const int64_t m = cuts[q];
      if (m == i || m - 1 == i) v -= fabs(e[m - 1]);
    }
    dw[i] = v;
  }
}

// ---------------------------------------------------------------------------
// leaves: cyclic Jacobi on the (torn) tridiagonal block, one workgroup each
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) leaf_jacobi(const double* dw, const double* e,
                                                  const int64_t* leaf_lo, const int64_t* leaf_hi,
                                                  double* lam, double* Z, int64_t ldz,
                                                  const double* Y, int64_t ldy, int ny,
                                                  double* PY, int64_t ldpy) {
  __shared__ double A[LEAF][LEAF + 1];
  __shared__ double V[LEAF][LEAF + 1];
  __shared__ double cs[2];
  __shared__ int rot;
  const int64_t lo = leaf_lo[blockIdx.x], hi = leaf_hi[blockIdx.x];
  const int m = (int)(hi - lo);
  const int t = threadIdx.x;
  for (int q = t; q < LEAF * LEAF; q += 64) {
    const int i = q % LEAF, j = q / LEAF;
    double a = 0.0;
    if (i < m && j < m) {
      if (i == j) a = dw[lo + i];
      else if (i == j + 1) a = e[lo + j];
      else if (j == i + 1) a = e[lo + i];
    }
    A[i][j] = a;
    V[i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (t == 0) rot = 0;
    __syncthreads();
    for (int p = 0; p < m - 1; ++p) {
      for (int q = p + 1; q < m; ++q) {
        if (t == 0) {
          const double apq = A[p][q], app = A[p][p], aqq = A[q][q];
          double c = 1.0, s = 0.0;
          if (apq != 0.0 && fabs(apq) > EPS * sqrt(fabs(app * aqq))) {
            const double th = (aqq - app) / (2.0 * apq);
            const double tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
            rot = 1;
          }
          cs[0] = c;
          cs[1] = s;
        }
        __syncthreads();
        const double c = cs[0], s = cs[1];
        if (s != 0.0) {
          if (t < m) {  // columns p, q
            const double akp = A[t][p], akq = A[t][q];
            A[t][p] = c * akp - s * akq;
            A[t][q] = s * akp + c * akq;
            const double vkp = V[t][p], vkq = V[t][q];
            V[t][p] = c * vkp - s * vkq;
            V[t][q] = s * vkp + c * vkq;
          }
          __syncthreads();
          if (t < m) {  // rows p, q
            const double apk = A[p][t], aqk = A[q][t];
            A[p][t] = c * apk - s * aqk;
            A[q][t] = s * apk + c * aqk;
          }
          __syncthreads();
          if (t == 0) { A[p][q] = 0.0; A[q][p] = 0.0; }
        }
        __syncthreads();
      }
    }
    if (rot == 0) break;
    __syncthreads();
  }
  // sort ascending (rank by value, ties by index) and write out
  __shared__ int rank[LEAF];
  if (t < m) {
    const double v = A[t][t];
    int r = 0;
    for (int j = 0; j < m; ++j) {
      const double w = A[j][j];
      if (w < v || (w == v && j < t)) ++r;
    }
    rank[t] = r;
  }
  __syncthreads();
  if (t < m) lam[lo + rank[t]] = A[t][t];
  if (PY) {
    // projected mode: row rank[j] gets V(:, j)^T [Y, e_first, e_last]
    for (int q = t; q < m * (ny + 2); q += 64) {
      const int j = q % m, c = q / m;
      double acc = 0.0;
      if (c < ny) {
        for (int i = 0; i < m; ++i) acc += V[i][j] * Y[(lo + i) + (int64_t)c * ldy];
      } else {
        acc = V[c == ny ? 0 : m - 1][j];
      }
      PY[(lo + rank[j]) + (int64_t)c * ldpy] = acc;
    }
  }
  if (!Z) return;
  for (int q = t; q < m * m; q += 64) {
    const int i = q % m, j = q / m;
    Z[(lo + i) + (lo + rank[j]) * ldz] = V[i][j];
  }
}

// ---------------------------------------------------------------------------
// merge step 1: z, sort, deflation (one workgroup per merge)
// Per merge, position-indexed arrays live at [lo, hi):
//   ds, zs, cols : sorted values, z, global column (after deflation updates)
//   kind         : 1 kept, 0 deflated
//   kept[lo + j] : sorted position of the j-th kept entry
// rot arrays     : Givens rotations (col_a, col_b, c, s) in application order
// meta[4*m]      : k (kept), ndfl, nrot, rho (as bits)
// ---------------------------------------------------------------------------
struct MergeBufs {
  double* ds; double* zs; int64_t* cols; int* kind; int64_t* kept;
  int64_t* rot_a; int64_t* rot_b; double* rot_c; double* rot_s;
  int64_t* meta;   // per merge: k, nrot
  double* rho;     // per merge
  int64_t* origin; double* tau; double* lamk; double* zhat;
  double* vals; int64_t* src;  // final values and their source (>=0 kept index, <0 -(col+1))
  int64_t* dfl;    // sorted positions of the deflated entries, in deflation order
  double* dk; double* zk;  // kept d and z, compact
  int64_t* colmap; // merge-order entry p = lo + q: the child column it comes from
  int64_t* dst;    // merge-order entry p: its sorted place (global index)
};

__global__ void __launch_bounds__(NT) merge_prepare(const Merge* merges, const double* e,
                                                    const double* lam, const double* Z,
                                                    int64_t ldz, MergeBufs b, double* PY,
                                                    int64_t ldpy, int ny) {
  const Merge mg = merges[blockIdx.x];
  const int64_t lo = mg.lo, mid = mg.mid, hi = mg.hi;
  const int64_t n1 = mid - lo, n2 = hi - mid, nm = hi - lo;
  const int t = threadIdx.x;
  const double ecut = e[mid - 1];
  const double sgn = ecut >= 0.0 ? 1.0 : -1.0;
  const double rho = 2.0 * fabs(ecut);
  const double r2 = 0.70710678118654752440;
  // merge the two sorted halves by rank (binary search in the other half)
  for (int64_t i = t; i < nm; i += NT) {
    double v, zz;
    int64_t col, pos;
    if (i < n1) {
      col = lo + i;
      v = lam[col];
      // child 1's eigenvector `col` at its last row
      zz = (PY ? PY[col + (int64_t)(ny + 1) * ldpy] : Z[(mid - 1) + col * ldz]) * r2;
      // count entries of half 2 strictly below v
      int64_t a = 0, c = n2;
      while (a < c) { const int64_t h = (a + c) / 2; if (lam[mid + h] < v) a = h + 1; else c = h; }
      pos = i + a;
    } else {
      const int64_t j = i - n1;
      col = mid + j;
      v = lam[col];
      // child 2's eigenvector `col` at its first row
      zz = sgn * (PY ? PY[col + (int64_t)ny * ldpy] : Z[mid + col * ldz]) * r2;
      // count entries of half 1 below or equal to v
      int64_t a = 0, c = n1;
      while (a < c) { const int64_t h = (a + c) / 2; if (lam[lo + h] <= v) a = h + 1; else c = h; }
      pos = j + a;
    }
    b.ds[lo + pos] = v;
    b.zs[lo + pos] = zz;
    b.cols[lo + pos] = col;
  }
  __syncthreads();
  __threadfence_block();
  if (PY) {
    // the parent's boundary rows: its first row is child 1's first row (zero
    // on child 2's eigenvectors), its last row child 2's last row (zero on
    // child 1's); z above has read the entries cleared here
    for (int64_t i = t; i < nm; i += NT)
      PY[(lo + i) + (int64_t)(i < n1 ? ny + 1 : ny) * ldpy] = 0.0;
  }
  if (t != 0) return;
  // ---- deflation scan --------------------------------------------------------
  double dmax = 0.0, zmax = 0.0;
  for (int64_t i = 0; i < nm; ++i) {
    dmax = fmax(dmax, fabs(b.ds[lo + i]));
    zmax = fmax(zmax, fabs(b.zs[lo + i]));
  }
  const double tol = 8.0 * EPS * fmax(dmax, rho * zmax);
  int64_t k = 0, nrot = 0, prev = -1, nd = 0;
  for (int64_t i = 0; i < nm; ++i) {
    const int64_t pi = lo + i;
    if (rho * fabs(b.zs[pi]) <= tol) {
      b.kind[pi] = 0;
      b.dfl[lo + nd++] = i;
      continue;
    }
    if (prev < 0) { prev = i; continue; }
    const int64_t pp = lo + prev;
    const double zp = b.zs[pp], zi = b.zs[pi];
    const double r = hypot(zp, zi);
    const double c = zi / r, s = zp / r;
    const double dp = b.ds[pp], di = b.ds[pi];
    if (fabs(c * s * (di - dp)) <= tol) {
      // rotate (prev, i) so that z_prev = 0; prev deflates
      b.ds[pp] = c * c * dp + s * s * di;
      b.ds[pi] = s * s * dp + c * c * di;
      b.zs[pp] = 0.0;
      b.zs[pi] = r;
      b.rot_a[lo + nrot] = b.cols[pp];
      b.rot_b[lo + nrot] = b.cols[pi];
      b.rot_c[lo + nrot] = c;
      b.rot_s[lo + nrot] = s;
      ++nrot;
      b.kind[pp] = 0;
      b.dfl[lo + nd++] = prev;
      prev = i;
    } else {
      b.kind[pp] = 1;
      b.kept[lo + k] = prev;
      ++k;
      prev = i;
    }
  }
  if (prev >= 0) {
    b.kind[lo + prev] = 1;
    b.kept[lo + k] = prev;
    ++k;
  }
  b.meta[2 * blockIdx.x] = k;
  b.meta[2 * blockIdx.x + 1] = nrot;
  b.rho[blockIdx.x] = rho;
}

// merge step 3: one secular root per thread.  Kept entries j of merge g are
// d_j = ds[lo + kept[lo + j]], z_j likewise (strictly increasing d).
__device__ __forceinline__ double kd(const MergeBufs& b, int64_t lo, int64_t j) {
  return b.dk[lo + j];
}
__device__ __forceinline__ double kz(const MergeBufs& b, int64_t lo, int64_t j) {
  return b.zk[lo + j];
}

__global__ void merge_compact(const Merge* merges, MergeBufs b) {
  const Merge mg = merges[blockIdx.y];
  const int64_t k = b.meta[2 * blockIdx.y];
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  const int64_t pos = mg.lo + b.kept[mg.lo + j];
  b.dk[mg.lo + j] = b.ds[pos];
  b.zk[mg.lo + j] = b.zs[pos];
}

__global__ void merge_secular(const Merge* merges, MergeBufs b, int64_t* status) {
  const Merge mg = merges[blockIdx.y];
  const int64_t lo = mg.lo;
  const int64_t k = b.meta[2 * blockIdx.y];
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  const double rho = b.rho[blockIdx.y];
  const double irho = 1.0 / rho;
  const double dj = kd(b, lo, j);
  int64_t o;
  double lo_t, hi_t;
  if (j < k - 1) {
    const double dj1 = kd(b, lo, j + 1);
    const double mid = 0.5 * (dj + dj1);
    double f = irho;
    for (int64_t i = 0; i < k; ++i) {
      const double zi = kz(b, lo, i);
      f += zi * zi / (kd(b, lo, i) - mid);
    }
    if (f >= 0.0) { o = j; lo_t = 0.0; hi_t = mid - dj; }
    else { o = j + 1; lo_t = mid - dj1; hi_t = 0.0; }
  } else {
    double zz = 0.0;
    for (int64_t i = 0; i < k; ++i) { const double zi = kz(b, lo, i); zz += zi * zi; }
    o = j;
    lo_t = 0.0;
    hi_t = rho * zz;
  }
  const double dorig = kd(b, lo, o);
  double tau = 0.5 * (lo_t + hi_t);
  bool ok = false;
  for (int it = 0; it < 200; ++it) {
    double psi = 0.0, dpsi = 0.0, phi = 0.0, dphi = 0.0, aabs = irho;
    for (int64_t i = 0; i < k; ++i) {
      const double zi = kz(b, lo, i);
      const double del = (kd(b, lo, i) - dorig) - tau;
      const double r = zi / del;
      const double term = zi * r;
      if (i <= j) { psi += term; dpsi += r * r; }
      else { phi += term; dphi += r * r; }
      aabs += fabs(term);
    }
    const double f = irho + psi + phi;
    if (f == 0.0 || fabs(f) <= 4.0 * EPS * (double)k * aabs) { ok = true; break; }
    if (f < 0.0) lo_t = tau; else hi_t = tau;
    if (hi_t - lo_t <= 2.0 * EPS * fmax(fabs(lo_t), fabs(hi_t))) { ok = true; break; }
    // two-pole rational model  f ~ a + B/(p - x) + C/(q - x)
    double xn;
    const double p = kd(b, lo, j) - dorig;
    if (j < k - 1) {
      const double q = kd(b, lo, j + 1) - dorig;
      const double Bc = (p - tau) * (p - tau) * dpsi;
      const double Cc = (q - tau) * (q - tau) * dphi;
      const double a = f - Bc / (p - tau) - Cc / (q - tau);
      // a (p-x)(q-x) + B (q-x) + C (p-x) = 0  ->  a x^2 - Bq x + C0 = 0
      const double Bq = a * (p + q) + Bc + Cc;
      const double C0 = a * p * q + Bc * q + Cc * p;
      double r1, r2;
      if (a == 0.0) { r1 = C0 / Bq; r2 = r1; }
      else {
        const double disc = Bq * Bq - 4.0 * a * C0;
        const double sq = sqrt(fmax(disc, 0.0));
        if (Bq >= 0.0) { r1 = (Bq + sq) / (2.0 * a); r2 = 2.0 * C0 / (Bq + sq); }
        else { r1 = (Bq - sq) / (2.0 * a); r2 = 2.0 * C0 / (Bq - sq); }
      }
      if (r1 > lo_t && r1 < hi_t) xn = r1;
      else if (r2 > lo_t && r2 < hi_t) xn = r2;
      else xn = 0.5 * (lo_t + hi_t);
    } else {
      const double Bc = (p - tau) * (p - tau) * dpsi;
      const double a = f - Bc / (p - tau);
      xn = (a > 0.0) ? p + Bc / a : 0.5 * (lo_t + hi_t);
      if (!(xn > lo_t && xn < hi_t)) xn = 0.5 * (lo_t + hi_t);
    }
    if (xn == tau) xn = 0.5 * (lo_t + hi_t);
    tau = xn;
  }
  if (!ok) atomicMax((unsigned long long*)status, 2ull);
  b.origin[lo + j] = o;
  b.tau[lo + j] = tau;
  b.lamk[lo + j] = dorig + tau;
}

// d_i - lam_j computed from the root's shift: (d_i - d_o(j)) - tau_j
__device__ __forceinline__ double dminus(const MergeBufs& b, int64_t lo, int64_t i, int64_t j) {
  return (kd(b, lo, i) - kd(b, lo, b.origin[lo + j])) - b.tau[lo + j];
}

// merge step 4: zhat_i^2 = ((lam_i - d_i)/rho) prod_{j != i} (lam_j - d_i)/(d_j - d_i)
__global__ void merge_lowner(const Merge* merges, MergeBufs b) {
  const Merge mg = merges[blockIdx.y];
  const int64_t lo = mg.lo;
  const int64_t k = b.meta[2 * blockIdx.y];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  const double rho = b.rho[blockIdx.y];
  const double di = kd(b, lo, i);
  double w = -dminus(b, lo, i, i) / rho;
  for (int64_t j = 0; j < k; ++j) {
    if (j == i) continue;
    w *= -dminus(b, lo, i, j) / (kd(b, lo, j) - di);
  }
  const double zi = kz(b, lo, i);
  b.zhat[lo + i] = copysign(sqrt(fabs(w)), zi);
}

// merge step 5: U (k x k, ld k) at U + lo*n: U(i,j) = zhat_i/(d_i - lam_j),
// columns normalised.  One workgroup per column.
__global__ void __launch_bounds__(NT) merge_form_u(const Merge* merges, MergeBufs b, double* U,
                                                   int64_t n) {
  const Merge mg = merges[blockIdx.y];
  const int64_t lo = mg.lo;
  const int64_t k = b.meta[2 * blockIdx.y];
  const int64_t j = blockIdx.x;
  if (j >= k) return;
  __shared__ double sh[4];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  double* Uj = U + lo * n + j * k;
  double ss = 0.0;
  for (int64_t i = t; i < k; i += NT) {
    const double v = b.zhat[lo + i] / dminus(b, lo, i, j);
    Uj[i] = v;
    ss += v * v;
  }
  for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
  if (lane == 0) sh[wave] = ss;
  __syncthreads();
  const double inv = 1.0 / sqrt((sh[0] + sh[1]) + (sh[2] + sh[3]));
  for (int64_t i = t; i < k; i += NT) Uj[i] *= inv;
}

// Rank-sort the merged spectrum.  Entry q < k is root q; entry q >= k is the
// (q-k)-th deflated sorted position.  Writes lam and the output columns.
__global__ void merge_collect(const Merge* merges, MergeBufs b) {
  const Merge mg = merges[blockIdx.y];
  const int64_t lo = mg.lo, nm = mg.hi - mg.lo;
  const int64_t k = b.meta[2 * blockIdx.y];
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nm) return;
  // the list is [roots..., deflated entries in deflation order]
  if (q < k) {
    b.vals[lo + q] = b.lamk[lo + q];
    b.src[lo + q] = q;
    b.colmap[lo + q] = b.cols[lo + b.kept[lo + q]];
  } else {
    const int64_t pos = b.dfl[lo + (q - k)];
    b.vals[lo + q] = b.ds[lo + pos];
    b.src[lo + q] = -(b.cols[lo + pos] + 1);
    b.colmap[lo + q] = b.cols[lo + pos];
  }
}

// The sorted place of every merge-order entry: its rank among the merged
// values, ties broken by merge order.  One workgroup per entry.
__global__ void merge_rank(const Merge* merges, MergeBufs b, double* lam) {
  const Merge mg = merges[blockIdx.y];
  const int64_t lo = mg.lo, nm = mg.hi - mg.lo;
  const int64_t q = blockIdx.x;
  if (q >= nm) return;
  const double v = b.vals[lo + q];
  __shared__ int64_t s_rank;
  if (threadIdx.x == 0) s_rank = 0;
  __syncthreads();
  int64_t r = 0;
  for (int64_t p = threadIdx.x; p < nm; p += blockDim.x) {
    const double w = b.vals[lo + p];
    if (w < v || (w == v && p < q)) ++r;
  }
  atomicAdd((unsigned long long*)&s_rank, (unsigned long long)r);
  __syncthreads();
  if (threadIdx.x == 0) {
    b.dst[lo + q] = lo + s_rank;
    lam[lo + s_rank] = v;
  }
}

// ---- eigenvector mode: the merges of a level applied to X's columns.
// Rotations: every row r of X (nr rows) rotates its columns (ca, cb).
__global__ void merge_rotate_cols(const Merge* merges, MergeBufs b, double* X, int64_t ldx,
                                  int64_t nr) {
  const int64_t nrot = b.meta[2 * blockIdx.y + 1];
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (nrot == 0 || r >= nr) return;
  const Merge mg = merges[blockIdx.y];
  for (int64_t q = 0; q < nrot; ++q) {
    const int64_t ca = b.rot_a[mg.lo + q], cb = b.rot_b[mg.lo + q];
    const double c = b.rot_c[mg.lo + q], s = b.rot_s[mg.lo + q];
    const double xa = X[r + ca * ldx], xb = X[r + cb * ldx];
    X[r + ca * ldx] = c * xa - s * xb;
    X[r + cb * ldx] = s * xa + c * xb;
  }
}

// Rows r0 .. r0+rows-1 of X in merge order: Tc(i, p) = X(r0 + i, colmap[p])
// for every entry p of the level (column p of Tc at Tc + p rr).
__global__ void merge_gather_cols(MergeBufs b, const double* X, int64_t ldx, int64_t r0,
                                  int64_t rows, double* Tc, int64_t rr) {
  const int64_t p = blockIdx.x;
  const double* src = X + r0 + b.colmap[p] * ldx;
  double* dst = Tc + p * rr;
  for (int64_t i = threadIdx.x; i < rows; i += blockDim.x) dst[i] = src[i];
}

// grouped products of a level: Oc(:, lo .. lo+k) = Tc(:, lo .. lo+k) U_merge
__global__ void merge_gemm_desc_cols(const Merge* merges, const MergeBufs b, const double* Tc,
                                     const double* U, double* Oc, int64_t n, int64_t rows,
                                     int64_t rr, GemmGroup* desc, int64_t nmerge) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nmerge) return;
  const int64_t lo = merges[g].lo;
  const int64_t k = b.meta[2 * g];
  GemmGroup d;
  d.A = Tc + lo * rr; d.lda = rr;
  d.B = U + lo * n; d.ldb = k > 0 ? k : 1;
  d.C = Oc + lo * rr; d.ldc = rr;
  d.m = rows; d.n = k; d.k = k;
  desc[g] = d;
}

// X(r0 + i, dst[p]) = (root ? Oc : Tc)(i, p)
__global__ void merge_place_cols(MergeBufs b, const double* Tc, const double* Oc, int64_t rr,
                                 double* X, int64_t ldx, int64_t r0, int64_t rows) {
  const int64_t p = blockIdx.x;
  const double* src = (b.src[p] >= 0 ? Oc : Tc) + p * rr;
  double* dst = X + r0 + b.dst[p] * ldx;
  for (int64_t i = threadIdx.x; i < rows; i += blockDim.x) dst[i] = src[i];
}

// ---- projected mode: the merge steps on the rows of PY (n x W, W = ny + 2).
// Rotations of eigenvector columns ca, cb act on rows ca, cb.
__global__ void merge_rotate_rows(const Merge* merges, MergeBufs b, double* PY, int64_t ldpy,
                                  int W) {
  const int64_t nrot = b.meta[2 * blockIdx.y + 1];
  const int c = (int)((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
  if (nrot == 0 || c >= W) return;
  const Merge mg = merges[blockIdx.y];
  for (int64_t q = 0; q < nrot; ++q) {
    const int64_t ca = b.rot_a[mg.lo + q], cb = b.rot_b[mg.lo + q];
    const double cc = b.rot_c[mg.lo + q], ss = b.rot_s[mg.lo + q];
    const double za = PY[ca + c * ldpy], zb = PY[cb + c * ldpy];
    PY[ca + c * ldpy] = cc * za - ss * zb;
    PY[cb + c * ldpy] = ss * za + cc * zb;
  }
}

// kept rows into G (k x W, ld k) at G + lo W
__global__ void merge_gather_rows(const Merge* merges, MergeBufs b, const double* PY, int64_t ldpy,
                                  int W, double* Gbuf) {
  const Merge mg = merges[blockIdx.y];
  const int64_t lo = mg.lo;
  const int64_t k = b.meta[2 * blockIdx.y];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= k * W) return;
  const int64_t j = e % k, c = e / k;
  Gbuf[lo * W + e] = PY[b.cols[lo + b.kept[lo + j]] + c * ldpy];
}

// grouped GEMM descriptors: Pt = U^T G (k x W, ld k) at Pt + lo W
__global__ void merge_gemm_desc_rows(const Merge* merges, const MergeBufs b, double* Gbuf,
                                     double* U, double* Ptb, int64_t n, int W, GemmGroup* desc,
                                     int64_t nmerge) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nmerge) return;
  const int64_t lo = merges[g].lo;
  const int64_t k = b.meta[2 * g];
  GemmGroup d;
  d.A = U + lo * n; d.lda = k > 0 ? k : 1;
  d.B = Gbuf + lo * W; d.ldb = k > 0 ? k : 1;
  d.C = Ptb + lo * W; d.ldc = k > 0 ? k : 1;
  d.m = k; d.n = W; d.k = k;
  desc[g] = d;
}

// sort rows into place (destinations from merge_rank)
__global__ void merge_place_rows(const Merge* merges, MergeBufs b, const double* PYold,
                                 const double* Ptb, double* PYnew, int64_t ldpy, int W) {
  const Merge mg = merges[blockIdx.y];
  const int64_t lo = mg.lo, nm = mg.hi - mg.lo;
  const int64_t q = blockIdx.x;
  if (q >= nm) return;
  const int64_t k = b.meta[2 * blockIdx.y];
  const int64_t sq = b.src[lo + q];
  const int64_t dst = b.dst[lo + q];
  for (int c = threadIdx.x; c < W; c += blockDim.x)
    PYnew[dst + (int64_t)c * ldpy] =
        sq >= 0 ? Ptb[lo * W + sq + (int64_t)c * k] : PYold[(-sq - 1) + (int64_t)c * ldpy];
}

__global__ void copy_vec(const double* s, double* d, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = s[i];
}

int depth_for(int64_t n) {
  int D = 0;
  while (ceil_div(n, (int64_t)1 << D) > LEAF) ++D;
  return D;
}

// U (n^2, the caller's) and n x W blocks for the rows (current, next), the
// gathered kept rows and their product with U^T; in eigenvector mode two
// row chunks of X (rr x n each) in merge order and their products with U.
struct LayoutP {
  double *dw, *lamA, *lamB, *U, *G, *Pt, *PYa, *PYb, *Tc, *Oc;
  int64_t *cuts, *leaf_lo, *leaf_hi;
  Merge* merges;
  GemmGroup* desc;
  MergeBufs mb;
  double* end;
};

LayoutP carve_proj(double* ws, int64_t n, int64_t max_merges, int W, int64_t rr, double* U) {
  LayoutP L;
  double* p = ws;
  auto take = [&](int64_t count) { double* r = p; p += count; return r; };
  L.dw = take(n);
  L.lamA = take(n);
  L.lamB = take(n);
  L.U = U;  // n^2 doubles the caller provides
  L.G = take(n * W);
  L.Pt = take(n * W);
  L.PYa = take(n * W);
  L.PYb = take(n * W);
  L.Tc = rr ? take(rr * n) : nullptr;
  L.Oc = rr ? take(rr * n) : nullptr;
  L.cuts = (int64_t*)take(n + 1);
  L.leaf_lo = (int64_t*)take(n + 1);
  L.leaf_hi = (int64_t*)take(n + 1);
  L.merges = (Merge*)take(3 * (max_merges + 1));
  L.desc = (GemmGroup*)take((int64_t)(sizeof(GemmGroup) / 8 + 1) * (max_merges + 1));
  MergeBufs& b = L.mb;
  b.ds = take(n); b.zs = take(n); b.cols = (int64_t*)take(n); b.kind = (int*)take(n);
  b.kept = (int64_t*)take(n);
  b.rot_a = (int64_t*)take(n); b.rot_b = (int64_t*)take(n); b.rot_c = take(n); b.rot_s = take(n);
  b.meta = (int64_t*)take(2 * (max_merges + 1)); b.rho = take(max_merges + 1);
  b.origin = (int64_t*)take(n); b.tau = take(n); b.lamk = take(n); b.zhat = take(n);
  b.vals = take(n); b.src = (int64_t*)take(n);
  b.dfl = (int64_t*)take(n); b.dk = take(n); b.zk = take(n);
  b.colmap = (int64_t*)take(n); b.dst = (int64_t*)take(n);
  L.end = p;
  return L;
}

// rows of X per chunk in eigenvector mode: two chunks of at most 2^27
// doubles (1 GiB) each
int64_t chunk_rows(int64_t n) {
  return std::max<int64_t>(1, std::min<int64_t>(n, ((int64_t)1 << 27) / std::max<int64_t>(n, 1)));
}

// The balanced tree over [0, n): levels[d] are the nodes at depth d (every
// node above the leaves is cut at its midpoint), then the cut positions and
// the leaves' ranges.
struct Tree {
  int D = 0;
  std::vector<std::vector<Merge>> levels;
  std::vector<int64_t> cuts, llo, lhi;
};
Tree build_tree(int64_t n) {
  Tree tr;
  tr.D = depth_for(n);
  const int D = tr.D;
  tr.levels.resize(D + 1);
  tr.levels[0].push_back({0, 0, n});
  for (int dd = 0; dd < D; ++dd) {
    for (size_t q = 0; q < tr.levels[dd].size(); ++q) {
      const int64_t lo = tr.levels[dd][q].lo, hi = tr.levels[dd][q].hi;
      const int64_t mid = lo + (hi - lo) / 2;
      tr.levels[dd][q].mid = mid;
      tr.levels[dd + 1].push_back({lo, lo, mid});
      tr.levels[dd + 1].push_back({mid, mid, hi});
    }
  }
  for (int dd = 0; dd < D; ++dd)
    for (const Merge& nd : tr.levels[dd]) tr.cuts.push_back(nd.mid);
  for (const Merge& nd : tr.levels[D]) { tr.llo.push_back(nd.lo); tr.lhi.push_back(nd.hi); }
  if (D == 0) { tr.llo.assign(1, 0); tr.lhi.assign(1, n); }
  return tr;
}

}  // namespace


namespace {

// The divide and conquer of both modes.  Projected (X null): ZY = Z^T Y
// (n x ny).  Eigenvector mode (X non-null, ny = 0): X <- X_pre Z, where
// X_pre is the leaves' block-diagonal eigenvectors after `pre`.
void dc_core(const double* d, const double* e, int64_t n, double* lam, const double* Y,
             int64_t ldy, int ny, double* ZY, int64_t ldzy, double* X, int64_t ldx,
             const std::function<void(double*)>& pre, double* U, double* ws, int64_t ws_elems,
             int64_t* d_status, hipStream_t s) {
  const int W = ny + 2;
  const Tree tr = build_tree(n);
  const int D = tr.D;
  const int64_t max_merges = (int64_t)1 << D;
  const int64_t rr = X ? chunk_rows(n) : 0;
  LayoutP L = carve_proj(ws, n, max_merges, W, rr, U);
  MM_REQUIRE(L.end - ws <= ws_elems, kInvalid, "stedc: workspace too small");
  const int64_t ncuts = (int64_t)tr.cuts.size();
  if (ncuts)
    MM_HIP_TRY(hipMemcpyAsync(L.cuts, tr.cuts.data(), ncuts * 8, hipMemcpyHostToDevice, s));
  MM_HIP_TRY(hipMemcpyAsync(L.leaf_lo, tr.llo.data(), tr.llo.size() * 8, hipMemcpyHostToDevice, s));
  MM_HIP_TRY(hipMemcpyAsync(L.leaf_hi, tr.lhi.data(), tr.lhi.size() * 8, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(tear_k, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, d, e, n, L.cuts,
                     ncuts, L.dw);
  if (X) fill(X, n * n, 0.0, s);  // the leaves write their diagonal blocks
  hipLaunchKernelGGL(leaf_jacobi, dim3((unsigned)tr.llo.size()), dim3(64), 0, s, L.dw, e,
                     L.leaf_lo, L.leaf_hi, L.lamA, X, ldx, Y, ldy, ny, L.PYa, n);
  MM_HIP_TRY(hipGetLastError());
  if (X && pre) pre(X);
  double* PYc = L.PYa;
  double* PYn = L.PYb;
  double* lc = L.lamA;
  double* ln = L.lamB;
  for (int dd = D - 1; dd >= 0; --dd) {
    const std::vector<Merge>& lv = tr.levels[dd];
    const int64_t nmg = (int64_t)lv.size();
    int64_t maxm = 0;
    for (const Merge& mg : lv) maxm = std::max(maxm, mg.hi - mg.lo);
    MM_HIP_TRY(hipMemcpyAsync(L.merges, lv.data(), nmg * sizeof(Merge), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(merge_prepare, dim3((unsigned)nmg), dim3(NT), 0, s, L.merges, e, lc,
                       nullptr, 0, L.mb, PYc, n, ny);
    hipLaunchKernelGGL(merge_rotate_rows, dim3((unsigned)ceil_div(W, 64), (unsigned)nmg), dim3(64),
                       0, s, L.merges, L.mb, PYc, n, W);
    if (X)
      hipLaunchKernelGGL(merge_rotate_cols, dim3((unsigned)ceil_div(n, 256), (unsigned)nmg),
                         dim3(256), 0, s, L.merges, L.mb, X, ldx, n);
    hipLaunchKernelGGL(merge_compact, dim3((unsigned)ceil_div(maxm, 256), (unsigned)nmg), dim3(256),
                       0, s, L.merges, L.mb);
    hipLaunchKernelGGL(merge_secular, dim3((unsigned)ceil_div(maxm, 64), (unsigned)nmg), dim3(64),
                       0, s, L.merges, L.mb, d_status);
    hipLaunchKernelGGL(merge_lowner, dim3((unsigned)ceil_div(maxm, 64), (unsigned)nmg), dim3(64),
                       0, s, L.merges, L.mb);
    hipLaunchKernelGGL(merge_form_u, dim3((unsigned)maxm, (unsigned)nmg), dim3(NT), 0, s, L.merges,
                       L.mb, L.U, n);
    hipLaunchKernelGGL(merge_gather_rows, dim3((unsigned)ceil_div(maxm * W, 256), (unsigned)nmg),
                       dim3(256), 0, s, L.merges, L.mb, PYc, n, W, L.G);
    hipLaunchKernelGGL(merge_gemm_desc_rows, dim3((unsigned)ceil_div(nmg, 64)), dim3(64), 0, s,
                       L.merges, L.mb, L.G, L.U, L.Pt, n, W, L.desc, nmg);
    MM_HIP_TRY(hipGetLastError());
    gemm_grouped(L.desc, nmg, maxm, W, true, false, 1.0, 0.0, s);
    hipLaunchKernelGGL(merge_collect, dim3((unsigned)ceil_div(maxm, 256), (unsigned)nmg),
                       dim3(256), 0, s, L.merges, L.mb);
    hipLaunchKernelGGL(merge_rank, dim3((unsigned)maxm, (unsigned)nmg), dim3(256), 0, s,
                       L.merges, L.mb, ln);
    hipLaunchKernelGGL(merge_place_rows, dim3((unsigned)maxm, (unsigned)nmg), dim3(64), 0, s,
                       L.merges, L.mb, PYc, L.Pt, PYn, n, W);
    MM_HIP_TRY(hipGetLastError());
    if (X) {
      for (int64_t r0 = 0; r0 < n; r0 += rr) {
        const int64_t rows = std::min(rr, n - r0);
        hipLaunchKernelGGL(merge_gather_cols, dim3((unsigned)n), dim3(256), 0, s, L.mb, X, ldx,
                           r0, rows, L.Tc, rr);
        hipLaunchKernelGGL(merge_gemm_desc_cols, dim3((unsigned)ceil_div(nmg, 64)), dim3(64), 0,
                           s, L.merges, L.mb, L.Tc, L.U, L.Oc, n, rows, rr, L.desc, nmg);
        MM_HIP_TRY(hipGetLastError());
        gemm_grouped(L.desc, nmg, rows, maxm, false, false, 1.0, 0.0, s);
        hipLaunchKernelGGL(merge_place_cols, dim3((unsigned)n), dim3(256), 0, s, L.mb, L.Tc,
                           L.Oc, rr, X, ldx, r0, rows);
        MM_HIP_TRY(hipGetLastError());
      }
    }
    std::swap(PYc, PYn);
    std::swap(lc, ln);
  }
  hipLaunchKernelGGL(copy_vec, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, lc, lam, n);
  if (ZY) copy_matrix(PYc, n, ZY, ldzy, n, ny, s);
  MM_HIP_TRY(hipGetLastError());
}

int64_t ws_size(int64_t n, int ny, bool eigvec) {
  const int64_t mm = (int64_t)1 << depth_for(n);
  double* base = reinterpret_cast<double*>(64);
  LayoutP L = carve_proj(base, n, mm, ny + 2, eigvec ? chunk_rows(n) : 0, nullptr);
  return (int64_t)(L.end - base);
}

}  // namespace

int64_t stedc_ws_elems(int64_t n) { return ws_size(n, 0, true); }

void stedc(const double* d, const double* e, int64_t n, double* lam, double* X, int64_t ldx,
           double* U, double* ws, int64_t ws_elems, int64_t* d_status, hipStream_t s,
           const std::function<void(double*)>& pre) {
  MM_REQUIRE(ldx == n, kInvalid, "stedc: ldx must equal n");
  MM_REQUIRE(X != nullptr && U != nullptr, kInvalid, "stedc: X and U are required");
  if (n <= 0) return;
  dc_core(d, e, n, lam, nullptr, 0, 0, nullptr, 0, X, ldx, pre, U, ws, ws_elems, d_status, s);
}

int64_t stedc_project_ws_elems(int64_t n, int ny) { return ws_size(n, ny, false); }

void stedc_project(const double* d, const double* e, int64_t n, double* lam, const double* Y,
                   int64_t ldy, int ny, double* ZY, int64_t ldzy, double* U, double* ws,
                   int64_t ws_elems, int64_t* d_status, hipStream_t s) {
  MM_REQUIRE(ny >= 1, kInvalid, "stedc_project: at least one column");
  MM_REQUIRE(U != nullptr || n <= 0, kInvalid, "stedc_project: no eigenvector scratch");
  if (n <= 0) return;
  dc_core(d, e, n, lam, Y, ldy, ny, ZY, ldzy, nullptr, 0, {}, U, ws, ws_elems, d_status, s);
}

}  // namespace mm
