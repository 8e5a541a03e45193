// Selective solution of the decoupled modal equations (Sec. 3.2: once the
// modes are known, each scalar equation can be solved on its own, and so for
// a chosen subset only).  Mode n is kept when its coupling score
//   score_n = max_j |W(n, j)| * max_p |Pt(n, p)|
// exceeds tol times the largest score: a mode with no forcing weight is never
// excited from I(0) = 0, and one with no probe weight is never seen.
//
// Three launches: the scores (one thread per mode, column reads coalesced
// across the wave), the selection (one workgroup: the maximum, a count per
// thread over a contiguous slice of modes, an exclusive scan of the counts,
// then each slice's kept indices written in ascending order), and the gather
// of the kept modes into compact column-major arrays of leading dimension
// n_kept, which the modal steppers take as a smaller problem.
#include "kernels.h"

namespace mm {
namespace {

constexpr int NT = 256;
constexpr int SEL_T = 1024;

__global__ void __launch_bounds__(NT) mode_scores_k(const double* W, int nf, const double* Pt,
                                                    int np, int64_t n0, double* score) {
  const int64_t n = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (n >= n0) return;
  double a = 0.0, b = 0.0;
  for (int j = 0; j < nf; ++j) a = fmax(a, fabs(W[n + (int64_t)j * n0]));
  for (int p = 0; p < np; ++p) b = fmax(b, fabs(Pt[n + (int64_t)p * n0]));
  score[n] = a * b;
}

__global__ void __launch_bounds__(SEL_T) select_k(const double* score, int64_t n0, double tol,
                                                  int64_t* idx, int64_t* count) {
  __shared__ double mx[SEL_T];
  __shared__ int64_t off[SEL_T];
  const int t = threadIdx.x;
  double v = 0.0;
  for (int64_t n = t; n < n0; n += SEL_T) v = fmax(v, score[n]);
  mx[t] = v;
  __syncthreads();
  for (int h = SEL_T / 2; h > 0; h >>= 1) {
    if (t < h) mx[t] = fmax(mx[t], mx[t + h]);
    __syncthreads();
  }
  const double thr = tol * mx[0];
  const int64_t per = ceil_div(n0, SEL_T);
  const int64_t b = (int64_t)t * per;
  const int64_t e = b + per < n0 ? b + per : n0;
  int64_t c = 0;
  for (int64_t n = b; n < e; ++n) c += score[n] > thr;
  off[t] = c;
  __syncthreads();
  if (t == 0) {
    int64_t run = 0;
    for (int i = 0; i < SEL_T; ++i) {
      const int64_t ci = off[i];
      off[i] = run;
      run += ci;
    }
    count[0] = run;
  }
  __syncthreads();
  int64_t o = off[t];
  for (int64_t n = b; n < e; ++n)
    if (score[n] > thr) idx[o++] = n;
}

__global__ void __launch_bounds__(NT) gather_modes_k(const int64_t* idx, int64_t nk, int64_t n0,
                                                     const double* lam, const double* W, int nf,
                                                     const double* Pt, int np, const double* y,
                                                     double* lam_s, double* W_s, double* Pt_s,
                                                     double* y_s) {
  const int64_t k = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (k >= nk) return;
  const int64_t n = idx[k];
  lam_s[k] = lam[n];
  y_s[k] = y[n];
  for (int j = 0; j < nf; ++j) W_s[k + (int64_t)j * nk] = W[n + (int64_t)j * n0];
  for (int p = 0; p < np; ++p) Pt_s[k + (int64_t)p * nk] = Pt[n + (int64_t)p * n0];
}

}  // namespace

void select_modes(const double* W, int nf, const double* Pt, int np, int64_t n0, double tol,
                  double* score, int64_t* idx, int64_t* count, hipStream_t s) {
  MM_REQUIRE(n0 >= 1, kInvalid, "select_modes: no modes");
  hipLaunchKernelGGL(mode_scores_k, dim3((unsigned)ceil_div(n0, NT)), dim3(NT), 0, s, W, nf, Pt,
                     np, n0, score);
  hipLaunchKernelGGL(select_k, dim3(1), dim3(SEL_T), 0, s, score, n0, tol, idx, count);
  MM_HIP_TRY(hipGetLastError());
}

void gather_modes(const int64_t* idx, int64_t nk, int64_t n0, const double* lam, const double* W,
                  int nf, const double* Pt, int np, const double* y, double* lam_s, double* W_s,
                  double* Pt_s, double* y_s, hipStream_t s) {
  if (nk <= 0) return;
  MM_REQUIRE(nk <= n0, kInvalid, "gather_modes: more kept modes than modes");
  hipLaunchKernelGGL(gather_modes_k, dim3((unsigned)ceil_div(nk, NT)), dim3(NT), 0, s, idx, nk,
                     n0, lam, W, nf, Pt, np, y, lam_s, W_s, Pt_s, y_s);
  MM_HIP_TRY(hipGetLastError());
}

}  // namespace mm
