// C ABI of libmm (declared in include/mm.h).  Host-side orchestration only:
// every arithmetic step of the method runs in the HIP kernels of this
// directory.
#include "mm.h"

#include <algorithm>
#include <chrono>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "eig.h"
#include "kernels.h"

using namespace mm;

namespace {

thread_local std::string g_err;

struct Dev {
  void* p = nullptr;
  size_t bytes = 0;
  Dev() = default;
  Dev(const Dev&) = delete;
  Dev& operator=(const Dev&) = delete;
  ~Dev() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  void alloc(size_t b) {
    if (b <= bytes && p) return;
    release();
    if (b == 0) b = 8;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      throw Error{kNoMem, "device allocation of " + std::to_string(b) + " bytes failed"};
    }
    bytes = b;
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
  double* d() const { return static_cast<double*>(p); }
};

constexpr int kBand = 64;         // bandwidth of the first tridiagonalisation stage
constexpr int kMaxBandBlock = 8192;  // largest block of R's banded factor
constexpr int kMaxColumns = 4096;  // sources, probes
constexpr int kMaxRunColumns = 8;  // forcing columns and probes of one stepping call

// workspace of the eigensolver (both divide and conquer modes keep their n^2
// scratch in C's storage); ny: the projected columns (0: the full solver)
int64_t eig_ws_elems(int64_t n, int nb, int ny = 0) {
  return ny > 0 ? syevd_project_ws_elems(n, nb, ny) : syevd_ws_elems(n, nb);
}

// Probe partial sums of mm_step_modal_noalloc: a file-scope device array
// (one copy per GPU, held until the process ends).  Host code reaches it
// only through the address hipGetSymbolAddress returns on each device.
constexpr int64_t kScratchDoubles = (int64_t)1 << 23;  // 64 MiB
__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};

// The scratch array's address on the current device, looked up once per
// device (with that device current).
double* scratch_on_current_device() {
  int dev = 0;
  MM_HIP_TRY(hipGetDevice(&dev));
  MM_REQUIRE(dev >= 0 && dev < kMaxDevices, kDevice, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    MM_HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    MM_REQUIRE(ptr != nullptr, kDevice, "no address for the scratch array");
    g_scratch[dev] = static_cast<double*>(ptr);
  }
  return g_scratch[dev];
}

}  // namespace

struct mm_ctx {
  hipStream_t stream = nullptr;
  int64_t n = 0, m = 0, n0 = 0;
  int n_src = 0, n_probe = 0, nf = 0;
  double h = 0.0;
  const double* Lb = nullptr;  // borrowed inductance matrix (or null: generated from xyz)
  int64_t ldl = 0;
  int64_t r_nnz = 0, band = 0;
  Dev xyz, r_rowptr, r_col, r_val, M0, P;
  Dev status;  // [0] potrf pivot (INT64_MAX = fine), [1] eigensolver status,
               // [2] band of R, [3] electrode rank test, [4] non-finite input
  // reduced problem: forcing columns F = [R_D | L_D | K^T M0] (n0 x nf), probe
  // weights Pt = K^T P (n0 x n_probe), direct probe term PD = P A_D (n_probe x m)
  Dev F, Pt, PD;
  // electrode reduction (m > 0): H = I - Vh T Vh^T (small = [T | Re^{-T} | tau]),
  // two-sided factors YL, YR of L and R (n x m), the sparse low-rank part of R_i
  Dev e_rowptr, e_col, e_val, Vh, small, YL, YR, idxV, lr_idx, lr_V, lr_Y;
  int nsV = 0, ns_lr = 0;
  Dev iD_modal, iD_chol;  // injected currents at each method's current step
  // modal method
  bool decomposed = false;
  bool has_V = false;  // the eigenvectors are formed (mm_decompose, not _projected)
  // G: L_i's Cholesky factor, then its inverse (during the decomposition);
  // Q: the eigenvectors of C; V = G^{-T} Q the pencil's eigenvectors
  // (L_i-orthonormal), the only n0^2 buffer kept after mm_decompose
  Dev G, Q, V, lam, Wm, Pm, y;
  // selective modal stepping: the kept modes (ascending index), compact copies
  // of their lam, forcing and probe weights (ld sel_n) and their own state
  bool selected = false;
  int64_t sel_n = 0;
  Dev sel_score, sel_idx, sel_lam, sel_W, sel_P, sel_y;
  // Cholesky method
  bool factored = false;
  double f_theta = 0.0, f_dt = 0.0;
  Dev Z, Dinv, DinvT, panels, I, b, yv, kstep;
  bool use_graph = true;  // MM_NO_GRAPH=1 in the environment turns graphs off
  // MM_TRACE=1: the decomposition synchronises at the end of each phase and
  // prints the phase and its seconds to stderr (a progress trace; off by default)
  bool trace = false;
  std::chrono::steady_clock::time_point t_mark;
  // probe partial sums of one step call
  Dev pp;
  double* scratch = nullptr;  // this device's scratch array (mm_step_modal_noalloc)
  Dev scanws;  // chunk end values and start states of the time-parallel stepping
  Dev tmp;
  std::string err;

  // R as given (n x n) and its trailing block R[m:, m:] (the sparse part of R_i)
  Csr Rfull() const {
    Csr c;
    c.rows = n; c.cols = n; c.nnz = r_nnz;
    c.rowptr = r_rowptr.as<int64_t>();
    c.col = r_col.as<int32_t>();
    c.val = r_val.d();
    return c;
  }
  Csr R() const {
    Csr c = Rfull();
    c.rows = n0; c.cols = n0; c.off = m;
    return c;
  }
  // low-rank part of L_i (+ w R_i): rows m.. of Vh and YL (+ w YR)
  LowRank lr(double w) const {
    LowRank l;
    if (m == 0) return l;
    l.U = Vh.d() + m; l.Y1 = YL.d() + m;
    l.Y2 = w != 0.0 ? YR.d() + m : nullptr; l.w2 = w;
    l.ld = n; l.m = (int)m;
    return l;
  }
  RLowRank Rlr() const {
    RLowRank r;
    if (m == 0 || ns_lr == 0) return r;
    r.ns = ns_lr; r.m = (int)m;
    r.idx = lr_idx.as<int32_t>(); r.Vs = lr_V.d(); r.Ys = lr_Y.d();
    return r;
  }
  // the inductance matrix, from row and column `off` on
  LSrc lsrc(int64_t off) const {
    LSrc l;
    l.xyz = Lb ? nullptr : xyz.d();
    l.h = h;
    l.L = Lb;
    l.ld = ldl;
    l.off = off;
    return l;
  }
  const double* T() const { return small.d(); }
  const double* RinvT() const { return small.d() + m * m; }
};

namespace {

mm_status fail(mm_ctx* c, const Error& e) {
  if (c) c->err = e.msg;
  g_err = e.msg;
  return (mm_status)e.code;
}

template <class F>
mm_status guarded(mm_ctx* c, F&& f) {
  try {
    f();
    return MM_OK;
  } catch (const Error& e) {
    return fail(c, e);
  } catch (const std::bad_alloc&) {
    return fail(c, Error{kNoMem, "host allocation failed"});
  } catch (...) {
    return fail(c, Error{kDevice, "unexpected failure"});
  }
}

void copy_in(Dev& dst, const void* src, size_t bytes, hipStream_t s) {
  dst.alloc(bytes);
  if (bytes) MM_HIP_TRY(hipMemcpyAsync(dst.p, src, bytes, hipMemcpyDeviceToDevice, s));
}

void check_steps(double theta, double dt, int64_t n_steps) {
  MM_REQUIRE(theta >= 0.0 && theta <= 1.0, kInvalid, "theta must lie in [0, 1]");
  MM_REQUIRE(std::isfinite(dt) && dt > 0.0, kInvalid, "dt must be finite and positive");
  MM_REQUIRE(n_steps >= 0, kInvalid, "n_steps must be >= 0");
}

void check_run_columns(const mm_ctx* c, bool many_probes = false) {
  MM_REQUIRE(c->nf <= kMaxRunColumns, kInvalid,
             "a stepping call drives at most 8 forcing columns (2(Ne-1) + n_src); "
             "use mm_batch for many sources");
  MM_REQUIRE(many_probes || c->n_probe <= kMaxRunColumns, kInvalid,
             "this call observes at most 8 probes (mm_step_modal, mm_step_modal_exact and "
             "mm_step_modal_selective take more)");
}

// Steps per chunk of the many-probe modal stepping: the increments of a
// chunk (n0 x steps) take at most 2^28 doubles (2 GiB).
int64_t dy_chunk_steps(int64_t n0) {
  return std::max<int64_t>(8, ((int64_t)1 << 28) / std::max<int64_t>(n0, 1));
}

// Factor `A` (n x n) in place and report the first bad pivot.
void factor_checked(double* A, int64_t n, int64_t* d_status, Dev& ws, hipStream_t s,
                    const char* what) {
  ws.alloc(sizeof(double) * potrf_ws_elems(n));
  fill_i64(d_status, 1, INT64_MAX, s);
  potrf_lower(A, n, n, ws.d(), potrf_ws_elems(n), d_status, s);
  int64_t piv = INT64_MAX;
  MM_HIP_TRY(hipMemcpyAsync(&piv, d_status, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MM_HIP_TRY(hipStreamSynchronize(s));
  if (piv != INT64_MAX)
    throw Error{kNotSpd, std::string(what) + " is not positive definite (pivot " +
                             std::to_string(piv) + ")"};
}

// The reduced problem of the injected-current decomposition (Sec. 3.1):
// K = H[:, m:], L_i = (H^T L H)[m:, m:], R_i = (H^T R H)[m:, m:],
// R_D = K^T R A_D, L_D = K^T L A_D, K^T M0, K^T P, P A_D with A_D = H [Re^{-T}; 0].
// Without electrodes F = M0 and Pt = P.
void reduce_problem(mm_ctx* c, const mm_problem* pb) {
  hipStream_t s = c->stream;
  const int64_t n = c->n, n0 = c->n0;
  const int m = (int)c->m;
  c->F.alloc(sizeof(double) * n0 * std::max(1, c->nf));
  c->Pt.alloc(sizeof(double) * n0 * c->n_probe);
  if (m == 0) {
    if (c->n_src > 0)
      MM_HIP_TRY(hipMemcpyAsync(c->F.p, c->M0.p, sizeof(double) * n * c->n_src,
                                hipMemcpyDeviceToDevice, s));
    MM_HIP_TRY(hipMemcpyAsync(c->Pt.p, c->P.p, sizeof(double) * n * c->n_probe,
                              hipMemcpyDeviceToDevice, s));
    return;
  }
  // E (m x n CSR); the support of V is inside E's columns and rows 0..m-1
  MM_REQUIRE(pb->e_rowptr && pb->e_col && pb->e_val && pb->e_nnz >= 1, kInvalid,
             "electrodes need E (CSR)");
  copy_in(c->e_rowptr, pb->e_rowptr, sizeof(int64_t) * (m + 1), s);
  copy_in(c->e_col, pb->e_col, sizeof(int32_t) * pb->e_nnz, s);
  copy_in(c->e_val, pb->e_val, sizeof(double) * pb->e_nnz, s);
  std::vector<int64_t> rp(m + 1);
  std::vector<int32_t> ecol(pb->e_nnz);
  MM_HIP_TRY(hipMemcpyAsync(rp.data(), c->e_rowptr.p, sizeof(int64_t) * (m + 1),
                            hipMemcpyDeviceToHost, s));
  MM_HIP_TRY(hipMemcpyAsync(ecol.data(), c->e_col.p, sizeof(int32_t) * pb->e_nnz,
                            hipMemcpyDeviceToHost, s));
  MM_HIP_TRY(hipStreamSynchronize(s));
  MM_REQUIRE(rp[0] == 0 && rp[m] == pb->e_nnz, kInvalid, "E: bad row pointers");
  std::vector<unsigned char> inV(n, 0);
  for (int a = 0; a < m; ++a) inV[a] = 1;
  for (int32_t j : ecol) {
    MM_REQUIRE(j >= 0 && j < n, kInvalid, "E: column index out of range");
    inV[j] = 1;
  }
  std::vector<int32_t> idx;
  for (int64_t i = 0; i < n; ++i)
    if (inV[i]) idx.push_back((int32_t)i);
  c->nsV = (int)idx.size();
  c->idxV.alloc(sizeof(int32_t) * idx.size());
  MM_HIP_TRY(hipMemcpyAsync(c->idxV.p, idx.data(), sizeof(int32_t) * idx.size(),
                            hipMemcpyHostToDevice, s));
  Csr E;
  E.rows = m; E.cols = n; E.nnz = pb->e_nnz;
  E.rowptr = c->e_rowptr.as<int64_t>(); E.col = c->e_col.as<int32_t>(); E.val = c->e_val.d();
  // H = I - V T V^T from the QR of E^T
  c->Vh.alloc(sizeof(double) * n * m);
  c->small.alloc(sizeof(double) * (2 * m * m + m));
  const int kmax = std::max(std::max(m, c->n_src), c->n_probe);
  const int64_t wse = apply_h_ws_elems(m, kmax);
  Dev work, ws, X, U;
  work.alloc(sizeof(double) * n * kmax);
  ws.alloc(sizeof(double) * wse);
  X.alloc(sizeof(double) * n * kmax);
  U.alloc(sizeof(double) * n * m);
  int64_t* st = c->status.as<int64_t>() + 3;
  fill_i64(st, 1, 0, s);
  electrode_qr(E, n, m, c->Vh.d(), c->small.d(), work.d(), st, s);
  int64_t bad = 0;
  MM_HIP_TRY(hipMemcpyAsync(&bad, st, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MM_HIP_TRY(hipStreamSynchronize(s));
  MM_REQUIRE(bad == 0, kInvalid, "the electrode rows of E are linearly dependent");
  const double* V = c->Vh.d();
  const double* T = c->T();
  // two-sided factors: H^T L H = L - V YL^T - YL V^T (likewise R)
  c->YL.alloc(sizeof(double) * n * m);
  c->YR.alloc(sizeof(double) * n * m);
  l_times_rows(c->lsrc(0), n, c->idxV.as<int32_t>(), c->nsV, V, n, m, X.d(), n, s);
  two_sided_y(V, T, n, m, X.d(), c->YL.d(), ws.d(), wse, s);
  csr_times_dense(c->Rfull(), V, n, m, X.d(), n, s);
  two_sided_y(V, T, n, m, X.d(), c->YR.d(), ws.d(), wse, s);
  // U = H [I_m; 0] spans im E^T;  R_D = (H^T R U)[m:] Re^{-T},  L_D likewise
  fill(U.d(), n * m, 0.0, s);
  for (int a = 0; a < m; ++a) fill(U.d() + a * (n + 1), 1, 1.0, s);
  apply_h(V, T, n, m, U.d(), n, m, false, ws.d(), wse, s);
  auto project = [&](double* Y, int col0) {  // F(:, col0:col0+m) = (H^T Y)[m:] Re^{-T}
    apply_h(V, T, n, m, Y, n, m, true, ws.d(), wse, s);
    Gemm g;
    g.m = n0; g.n = m; g.k = m;
    g.A = Y + m; g.lda = n;
    g.B = c->RinvT(); g.ldb = m;
    g.C = c->F.d() + (int64_t)col0 * n0; g.ldc = n0;
    gemm(g, s);
  };
  csr_times_dense(c->Rfull(), U.d(), n, m, X.d(), n, s);
  project(X.d(), 0);
  l_times_rows(c->lsrc(0), n, c->idxV.as<int32_t>(), c->nsV, U.d(), n, m, X.d(), n, s);
  project(X.d(), m);
  if (c->n_src > 0) {  // K^T M0
    MM_HIP_TRY(hipMemcpyAsync(X.p, c->M0.p, sizeof(double) * n * c->n_src,
                              hipMemcpyDeviceToDevice, s));
    apply_h(V, T, n, m, X.d(), n, c->n_src, true, ws.d(), wse, s);
    copy_matrix(X.d() + m, n, c->F.d() + (int64_t)2 * m * n0, n0, n0, c->n_src, s);
  }
  // probes: Pt = (H^T P)[m:],  PD = P A_D = (H^T P)[:m]^T Re^{-T}
  MM_HIP_TRY(hipMemcpyAsync(X.p, c->P.p, sizeof(double) * n * c->n_probe,
                            hipMemcpyDeviceToDevice, s));
  apply_h(V, T, n, m, X.d(), n, c->n_probe, true, ws.d(), wse, s);
  copy_matrix(X.d() + m, n, c->Pt.d(), n0, n0, c->n_probe, s);
  c->PD.alloc(sizeof(double) * c->n_probe * m);
  {
    Gemm g;
    g.m = c->n_probe; g.n = m; g.k = m;
    g.A = X.d(); g.lda = n; g.ta = true;
    g.B = c->RinvT(); g.ldb = m;
    g.C = c->PD.d(); g.ldc = c->n_probe;
    gemm(g, s);
  }
  // the low-rank part of R_i lives on the rows where V or YR is non-zero
  Dev mark;
  mark.alloc(n0);
  mark_rows(V + m, c->YR.d() + m, n, n0, m, mark.as<unsigned char>(), s);
  std::vector<unsigned char> mk(n0);
  MM_HIP_TRY(hipMemcpyAsync(mk.data(), mark.p, n0, hipMemcpyDeviceToHost, s));
  MM_HIP_TRY(hipStreamSynchronize(s));
  std::vector<int32_t> li;
  for (int64_t i = 0; i < n0; ++i)
    if (mk[i]) li.push_back((int32_t)i);
  c->ns_lr = (int)li.size();
  if (c->ns_lr > 0) {
    c->lr_idx.alloc(sizeof(int32_t) * li.size());
    MM_HIP_TRY(hipMemcpyAsync(c->lr_idx.p, li.data(), sizeof(int32_t) * li.size(),
                              hipMemcpyHostToDevice, s));
    c->lr_V.alloc(sizeof(double) * li.size() * m);
    c->lr_Y.alloc(sizeof(double) * li.size() * m);
    gather_rows(V + m, n, c->lr_idx.as<int32_t>(), c->ns_lr, m, c->lr_V.d(), s);
    gather_rows(c->YR.d() + m, n, c->lr_idx.as<int32_t>(), c->ns_lr, m, c->lr_Y.d(), s);
  }
  c->iD_modal.alloc(sizeof(double) * m);
  c->iD_chol.alloc(sizeof(double) * m);
  fill(c->iD_modal.d(), m, 0.0, s);
  fill(c->iD_chol.d(), m, 0.0, s);
  MM_HIP_TRY(hipStreamSynchronize(s));  // the host vectors above must outlive the copies
}

}  // namespace

extern "C" {

mm_status mm_setup(const mm_problem* pb, void* stream, mm_ctx** out) {
  if (!out) { g_err = "mm_setup: out is NULL"; return MM_E_INVALID; }
  *out = nullptr;
  mm_ctx* c = nullptr;
  try {
    c = new mm_ctx();
  } catch (...) {
    g_err = "host allocation failed";
    return MM_E_NOMEM;
  }
  mm_status st = guarded(c, [&] {
    MM_REQUIRE(pb != nullptr, kInvalid, "problem is NULL");
    MM_REQUIRE(pb->n >= 1 && pb->n < ((int64_t)1 << 31), kInvalid, "n out of range");
    if (pb->L) {
      MM_REQUIRE(pb->ldl >= pb->n, kInvalid, "L: ldl must be >= n");
    } else {
      MM_REQUIRE(pb->xyz, kInvalid, "L or xyz is required");
      MM_REQUIRE(std::isfinite(pb->h) && pb->h > 0.0, kInvalid, "h must be finite and positive");
    }
    MM_REQUIRE(pb->r_rowptr && pb->r_col && pb->r_val && pb->r_nnz >= 1, kInvalid,
               "R is required");
    MM_REQUIRE(pb->n_probe >= 1 && pb->n_probe <= kMaxColumns && pb->P, kInvalid,
               "1..4096 probe rows are required");
    MM_REQUIRE(pb->n_src >= 0 && pb->n_src <= kMaxColumns && (pb->n_src == 0 || pb->M0),
               kInvalid, "0..4096 sources");
    MM_REQUIRE(pb->n_e == 0 || (pb->n_e >= 2 && pb->n_e - 1 < pb->n), kInvalid,
               "Ne must be 0 or 2..n");
    c->stream = (hipStream_t)stream;
    hipStream_t s = c->stream;
    c->scratch = scratch_on_current_device();
    const char* ng = std::getenv("MM_NO_GRAPH");
    c->use_graph = !(ng && ng[0] == '1');
    const char* tr = std::getenv("MM_TRACE");
    c->trace = tr && tr[0] == '1';
    c->n = pb->n;
    c->m = pb->n_e > 0 ? pb->n_e - 1 : 0;
    c->n0 = c->n - c->m;
    c->n_src = pb->n_src;
    c->n_probe = pb->n_probe;
    c->nf = 2 * (int)c->m + c->n_src;
    MM_REQUIRE(2 * c->m <= 8, kInvalid, "at most 5 electrodes");
    c->h = pb->h;
    c->Lb = pb->L;
    c->ldl = pb->ldl;
    c->r_nnz = pb->r_nnz;
    if (!c->Lb) copy_in(c->xyz, pb->xyz, sizeof(double) * 3 * c->n, s);
    copy_in(c->r_rowptr, pb->r_rowptr, sizeof(int64_t) * (c->n + 1), s);
    copy_in(c->r_col, pb->r_col, sizeof(int32_t) * std::max<int64_t>(1, c->r_nnz), s);
    copy_in(c->r_val, pb->r_val, sizeof(double) * std::max<int64_t>(1, c->r_nnz), s);
    copy_in(c->M0, pb->M0, sizeof(double) * c->n * c->n_src, s);
    copy_in(c->P, pb->P, sizeof(double) * c->n * c->n_probe, s);
    c->status.alloc(5 * sizeof(int64_t));
    {  // every floating-point input must be finite
      int64_t* flag = c->status.as<int64_t>() + 4;
      fill_i64(flag, 1, 0, s);
      if (c->Lb) flag_nonfinite_lower(c->Lb, c->ldl, c->n, flag, s);
      else flag_nonfinite(c->xyz.d(), 3 * c->n, flag, s);
      flag_nonfinite(c->r_val.d(), c->r_nnz, flag, s);
      flag_nonfinite(c->M0.d(), c->n * c->n_src, flag, s);
      flag_nonfinite(c->P.d(), c->n * c->n_probe, flag, s);
      if (c->m > 0 && pb->e_val && pb->e_nnz > 0) flag_nonfinite(pb->e_val, pb->e_nnz, flag, s);
      int64_t bad = 0;
      MM_HIP_TRY(hipMemcpyAsync(&bad, flag, sizeof(int64_t), hipMemcpyDeviceToHost, s));
      MM_HIP_TRY(hipStreamSynchronize(s));
      MM_REQUIRE(bad == 0, kInvalid, "an input (L or xyz, R, E, M0 or P) holds NaN or Inf");
    }
    csr_lower_band(c->Rfull(), c->status.as<int64_t>() + 2, s);
    MM_HIP_TRY(hipMemcpyAsync(&c->band, c->status.as<int64_t>() + 2, sizeof(int64_t),
                              hipMemcpyDeviceToHost, s));
    MM_HIP_TRY(hipStreamSynchronize(s));
    // a1: the reduced problem (electrodes), forcing columns and probe weights
    reduce_problem(c, pb);
  });
  if (st != MM_OK) {
    delete c;
    return st;
  }
  *out = c;
  return MM_OK;
}

namespace {

// The progress trace: with MM_TRACE=1, wait for the stream and print the
// phase just finished with its seconds.
void mark(mm_ctx* c, const char* what) {
  if (!c->trace) return;
  MM_HIP_TRY(hipStreamSynchronize(c->stream));
  const auto now = std::chrono::steady_clock::now();
  const double sec = std::chrono::duration<double>(now - c->t_mark).count();
  c->t_mark = now;
  std::fprintf(stderr, "libmm: n0 = %lld, %s done (%.2f s)\n", (long long)c->n0, what, sec);
  std::fflush(stderr);
}

// a0-a8 with the standard form taken on the resistance side, as the paper
// writes the eigenproblem (Sec. 3.2, eq. generalized_eigenvalues_discrete:
// Li v = tau Ri v).  Ri = R'' - V Y^T - Y V^T (R'' = R[m:, m:], sparse and
// banded; the electrode term of rank 2m) factors as F F^T with
// F = H A^{1/2}, R'' = H H^T (block bidiagonal, band.hip) and
// A = I + Z S Z^T, Z = H^{-1} [V, Y]; A^{-1/2} = I + Z Gamma Z^T.  Then
// C' = F^{-1} Li F^{-T} = A^{-1/2} (H^{-1} Li H^{-T}) A^{-1/2} has the time
// constants tau as eigenvalues, and with C' = Q' T Q'^T the pencil's
// Li-normalised eigenvectors are V = F^{-T} Q' T^{-1/2} (V^T Li V = I,
// V^T Ri V = T^{-1}), ordered by ascending lam = 1 / tau.  No dense
// factorisation of L is needed: the standard form costs 4 n0^2 Bb flops.
// project: eigenvalues and the projected weights V^T [F, P] only (Q' applied
// to the few columns F^{-1} [F, P] on the way through the eigensolver).
void decompose_impl(mm_ctx* c, bool project) {
    hipStream_t s = c->stream;
    const int64_t n0 = c->n0;
    const int m = (int)c->m;
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kBand, n0 - 1));
    const int ny = c->nf + c->n_probe;
    const int Bb = (int)band_block(c->band);
    MM_REQUIRE(Bb <= kMaxBandBlock, kInvalid,
               "R's bandwidth exceeds 8192: number the unknowns so that R is banded "
               "(a grid's natural order, or a bandwidth-reducing order)");
    const int64_t nblk = ceil_div(n0, (int64_t)Bb);
    c->decomposed = false;
    c->has_V = false;
    c->selected = false;
    c->t_mark = std::chrono::steady_clock::now();
    c->Q.release();
    c->V.release();
    c->G.release();
    // The small buffers first (an allocation that has to reuse memory just
    // freed by a large one of the same size can take seconds); at N = 98,304
    // one n0^2 buffer is 77 GB, and at most two and a half are live.
    const int64_t wse = eig_ws_elems(n0, nb, project ? ny : 0);
    Dev Cb, ws, Hinv, Hs, tmp, Zh, small, Yc, ZY, tau;
    ws.alloc(sizeof(double) * std::max(wse, band_factor_ws_elems(Bb)));
    Sb2stPlan plan = sb2st_plan(n0, nb);
    Dev tau1, T1, AB, V2, tau2, off, dv, ev;
    const int64_t np = std::max<int64_t>(1, sy2sb_npanels(n0, nb));
    tau1.alloc(sizeof(double) * np * nb);
    T1.alloc(sizeof(double) * np * nb * nb);
    AB.alloc(sizeof(double) * (2 * nb + 1) * n0);
    off.alloc(sizeof(int64_t) * (n0 + 1));
    dv.alloc(sizeof(double) * n0);
    ev.alloc(sizeof(double) * std::max<int64_t>(1, n0));
    tau.alloc(sizeof(double) * n0);
    Hinv.alloc(sizeof(double) * nblk * Bb * Bb);
    Hs.alloc(sizeof(double) * nblk * Bb * Bb);
    tmp.alloc(sizeof(double) * (int64_t)Bb * std::max<int64_t>(n0, ny));
    if (project) {
      Yc.alloc(sizeof(double) * n0 * ny);
      ZY.alloc(sizeof(double) * n0 * ny);
    }
    const int k2 = 2 * m;
    if (m > 0) {
      Zh.alloc(sizeof(double) * n0 * 5 * k2);   // [Z | U2 | Z] and P = X Z
      small.alloc(sizeof(double) * 4 * 64 + 8);  // Gz, Gamma, Qm, K, bad flag
    }
    c->lam.alloc(sizeof(double) * n0);
    c->Wm.alloc(sizeof(double) * n0 * std::max(1, c->nf));
    c->Pm.alloc(sizeof(double) * n0 * c->n_probe);
    c->y.alloc(sizeof(double) * n0);
    int64_t* st = c->status.as<int64_t>();
    // a2': R'' = H H^T
    band_factor(c->R(), n0, Bb, Hinv.d(), Hs.d(), ws.d(),
                std::max(wse, band_factor_ws_elems(Bb)), st, s);
    {
      int64_t piv = INT64_MAX;
      MM_HIP_TRY(hipMemcpyAsync(&piv, st, sizeof(int64_t), hipMemcpyDeviceToHost, s));
      MM_HIP_TRY(hipStreamSynchronize(s));
      if (piv != INT64_MAX)
        throw Error{kNotSpd, "R (its block of the unknowns without the excluded electrode "
                             "rows) is not positive definite"};
    }
    mark(c, "banded Cholesky factorisation of R''");
    // a0, a1: Li, both triangles, in C's storage.  C's columns start on
    // 128-byte boundaries (n0 is odd at the electrode plates): the band
    // reduction reads C's lower triangle also row-wise, in 128-byte pieces
    // of many columns, which would otherwise straddle lines
    const int64_t ldC = ceil_div(n0, 16) * 16;
    Cb.alloc(sizeof(double) * ldC * n0);
    double* C = Cb.d();
    assemble_L(c->lsrc(m), n0, C, ldC, true, s, c->lr(0.0));
    // a3': X = H^{-1} Li H^{-T}
    band_solve_left(Hinv.d(), Hs.d(), n0, Bb, C, ldC, n0, tmp.d(), s);
    band_solve_right_t(Hinv.d(), Hs.d(), n0, Bb, C, ldC, n0, tmp.d(), s);
    double* Z = nullptr;
    double* Gamma = nullptr;
    if (m > 0) {
      // Z = H^{-1} [V, Y] (rows m.. of the Householder vectors and of YR)
      Z = Zh.d();
      double* U2 = Z + n0 * k2;
      double* P = Z + 3 * n0 * k2;
      double* Gz = small.d();
      Gamma = Gz + 64;
      double* Qm = Gz + 128;
      double* K = Gz + 192;
      int64_t* bad = reinterpret_cast<int64_t*>(Gz + 256);
      copy_matrix(c->Vh.d() + m, c->n, Z, n0, n0, m, s);
      copy_matrix(c->YR.d() + m, c->n, Z + n0 * m, n0, n0, m, s);
      band_solve_left(Hinv.d(), Hs.d(), n0, Bb, Z, n0, k2, tmp.d(), s);
      {
        Gemm g;  // Gz = Z^T Z
        g.m = k2; g.n = k2; g.k = n0;
        g.A = Z; g.lda = n0; g.ta = true;
        g.B = Z; g.ldb = n0;
        g.C = Gz; g.ldc = k2;
        gemm(g, s);
      }
      fill_i64(bad, 1, 0, s);
      lowrank_gamma(Gz, m, Gamma, bad, s);
      {
        Gemm g;  // P = X Z (X symmetric, both triangles present)
        g.m = n0; g.n = k2; g.k = n0;
        g.A = C; g.lda = ldC;
        g.B = Z; g.ldb = n0;
        g.C = P; g.ldc = n0;
        gemm(g, s);
      }
      {
        Gemm g;  // Qm = Z^T P
        g.m = k2; g.n = k2; g.k = n0;
        g.A = Z; g.lda = n0; g.ta = true;
        g.B = P; g.ldb = n0;
        g.C = Qm; g.ldc = k2;
        gemm(g, s);
      }
      lowrank_gqg(Gamma, Qm, k2, K, s);
      {
        Gemm g;  // U2 = P Gamma
        g.m = n0; g.n = k2; g.k = k2;
        g.A = P; g.lda = n0;
        g.B = Gamma; g.ldb = k2;
        g.C = U2; g.ldc = n0;
        gemm(g, s);
      }
      {
        Gemm g;  // U2 += Z K
        g.m = n0; g.n = k2; g.k = k2;
        g.beta = 1.0;
        g.A = Z; g.lda = n0;
        g.B = K; g.ldb = k2;
        g.C = U2; g.ldc = n0;
        gemm(g, s);
      }
      // C' = X + Z U2^T + U2 Z^T (lower triangle): [Z | U2] [U2 | Z]^T
      copy_matrix(Z, n0, U2 + n0 * k2, n0, n0, k2, s);
      Gemm g;
      g.m = n0; g.n = n0; g.k = 2 * k2;
      g.beta = 1.0;
      g.A = Z; g.lda = n0;
      g.B = U2; g.ldb = n0; g.tb = true;
      g.C = C; g.ldc = ldC;
      g.lower = true;
      gemm(g, s);
      int64_t nbad = 0;
      MM_HIP_TRY(hipMemcpyAsync(&nbad, bad, sizeof(int64_t), hipMemcpyDeviceToHost, s));
      MM_HIP_TRY(hipStreamSynchronize(s));
      MM_REQUIRE(nbad == 0, kNotSpd, "the reduced resistance R_i is not positive definite");
    }
    mark(c, "standard form C' = F^{-1} L_i F^{-T}");
    // F^{-1} Y = A^{-1/2} H^{-1} Y for a few columns Y: H^{-1}, then
    // Y += Z (Gamma (Z^T Y)); the product buffer is the low-rank area's P
    auto apply_finv = [&](double* Y, int64_t ldy, int64_t cols) {
      band_solve_left(Hinv.d(), Hs.d(), n0, Bb, Y, ldy, cols, tmp.d(), s);
      if (m == 0 || cols == 0) return;
      double* t1 = tmp.d();             // k2 x cols
      double* t2 = tmp.d() + k2 * cols;  // k2 x cols
      Gemm g1;
      g1.m = k2; g1.n = cols; g1.k = n0;
      g1.A = Z; g1.lda = n0; g1.ta = true;
      g1.B = Y; g1.ldb = ldy;
      g1.C = t1; g1.ldc = k2;
      gemm(g1, s);
      Gemm g2;
      g2.m = k2; g2.n = cols; g2.k = k2;
      g2.A = Gamma; g2.lda = k2;
      g2.B = t1; g2.ldb = k2;
      g2.C = t2; g2.ldc = k2;
      gemm(g2, s);
      Gemm g3;
      g3.m = n0; g3.n = cols; g3.k = k2;
      g3.beta = 1.0;
      g3.A = Z; g3.lda = n0;
      g3.B = t2; g3.ldb = k2;
      g3.C = Y; g3.ldc = ldy;
      gemm(g3, s);
    };
    // the bulge-chase reflectors, kept for the back-transform, or for Q2^T of
    // more projected columns than the chase carries along
    const bool keep_q2 = !project || ny > sb2st_max_cols();
    if (keep_q2) {
      V2.alloc(sizeof(double) * std::max<int64_t>(1, plan.tasks) * nb);
      tau2.alloc(sizeof(double) * std::max<int64_t>(1, plan.tasks));
    }
    MM_HIP_TRY(hipMemcpyAsync(off.p, plan.offset.data(), sizeof(int64_t) * (n0 + 1),
                              hipMemcpyHostToDevice, s));
    EigWork w;
    w.nb = nb;
    w.tau1 = tau1.d(); w.T1 = T1.d(); w.AB = AB.d();
    w.V2 = keep_q2 ? V2.d() : nullptr;
    w.tau2 = keep_q2 ? tau2.d() : nullptr;
    w.d_offset = off.as<int64_t>(); w.d = dv.d(); w.e = ev.d();
    w.ws = ws.d(); w.ws_elems = wse;
    w.mark = [c](const char* what) { mark(c, what); };
    fill_i64(st + 1, 1, 0, s);
    if (project) {
      // a8 without Q': F^{-1} [F, P], then Q'^T on the way through
      if (c->nf > 0) copy_matrix(c->F.d(), n0, Yc.d(), n0, n0, c->nf, s);
      copy_matrix(c->Pt.d(), n0, Yc.d() + (int64_t)c->nf * n0, n0, n0, c->n_probe, s);
      apply_finv(Yc.d(), n0, ny);
      syevd_project(C, ldC, n0, tau.d(), Yc.d(), n0, ny, ZY.d(), n0, w, plan, st + 1, s);
      modes_from_tau(tau.d(), ZY.d(), n0, c->nf, c->n_probe, c->lam.d(), c->Wm.d(),
                     c->Pm.d(), s);
    } else {
      // a4-a7: Q' in Q's storage (C's storage is the merges' scratch)
      c->Q.alloc(sizeof(double) * n0 * n0);
      double* Q = c->Q.d();
      syevd(C, ldC, n0, tau.d(), Q, n0, w, plan, st + 1, s);
      MM_HIP_TRY(hipStreamSynchronize(s));
      V2.release();
      tau2.release();
      Cb.release();
      // V = F^{-T} Q' T^{-1/2} = H^{-T} (Q' + Z Gamma (Z^T Q')) T^{-1/2}, columns
      // in ascending lam
      if (m > 0) {
        double* t1 = tmp.d();
        double* t2 = tmp.d() + k2 * n0;
        Gemm g1;
        g1.m = k2; g1.n = n0; g1.k = n0;
        g1.A = Z; g1.lda = n0; g1.ta = true;
        g1.B = Q; g1.ldb = n0;
        g1.C = t1; g1.ldc = k2;
        gemm(g1, s);
        Gemm g2;
        g2.m = k2; g2.n = n0; g2.k = k2;
        g2.A = Gamma; g2.lda = k2;
        g2.B = t1; g2.ldb = k2;
        g2.C = t2; g2.ldc = k2;
        gemm(g2, s);
        Gemm g3;
        g3.m = n0; g3.n = n0; g3.k = k2;
        g3.beta = 1.0;
        g3.A = Z; g3.lda = n0;
        g3.B = t2; g3.ldb = k2;
        g3.C = Q; g3.ldc = n0;
        gemm(g3, s);
      }
      band_solve_left_t(Hinv.d(), Hs.d(), n0, Bb, Q, n0, n0, tmp.d(), s);
      reverse_scale_cols(Q, n0, n0, tau.d(), c->lam.d(), s);
      std::swap(c->V.p, c->Q.p);
      std::swap(c->V.bytes, c->Q.bytes);
      mark(c, "eigenvectors V = F^{-T} Q' T^{-1/2}");
      // a8: modal weights  W = V^T F,  Pt = V^T P
      if (c->nf > 0) {
        Gemm g;
        g.m = n0; g.n = c->nf; g.k = n0;
        g.A = c->V.d(); g.lda = n0; g.ta = true;
        g.B = c->F.d(); g.ldb = n0;
        g.C = c->Wm.d(); g.ldc = n0;
        gemm(g, s);
      }
      {
        Gemm g;
        g.m = n0; g.n = c->n_probe; g.k = n0;
        g.A = c->V.d(); g.lda = n0; g.ta = true;
        g.B = c->Pt.d(); g.ldb = n0;
        g.C = c->Pm.d(); g.ldc = n0;
        gemm(g, s);
      }
    }
    fill(c->y.d(), n0, 0.0, s);
    int64_t est = 0;
    double tau_min = 0.0;  // the eigenvalues of C' ascend
    MM_HIP_TRY(hipMemcpyAsync(&est, st + 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    MM_HIP_TRY(hipMemcpyAsync(&tau_min, tau.d(), sizeof(double), hipMemcpyDeviceToHost, s));
    MM_HIP_TRY(hipStreamSynchronize(s));
    MM_HIP_TRY(hipGetLastError());
    if (est != 0) throw Error{kNoConverge, "a secular equation did not converge"};
    // C' is congruent to Li, so a time constant <= 0 means Li is not
    // positive definite (a dense L handed over by the caller can be anything)
    if (!(tau_min > 0.0))
      throw Error{kNotSpd, "the reduced inductance L_i is not positive definite (smallest "
                           "time constant " + std::to_string(tau_min) + ")"};
    c->decomposed = true;
    c->has_V = !project;
}

}  // namespace

mm_status mm_decompose(mm_ctx* c) {
  if (!c) return MM_E_INVALID;
  return guarded(c, [&] { decompose_impl(c, false); });
}

mm_status mm_decompose_projected(mm_ctx* c) {
  if (!c) return MM_E_INVALID;
  return guarded(c, [&] { decompose_impl(c, true); });
}

namespace {

void step_modal_impl(mm_ctx* c, double theta, double dt, bool exact, int64_t n_steps,
                     const double* i_src, const double* i_D, double* signal,
                     bool scan = false, bool selective = false, bool no_alloc = false) {
    MM_REQUIRE(c->decomposed, kState, "modal stepping before mm_decompose");
    MM_REQUIRE(!selective || c->selected, kState,
               "mm_step_modal_selective before mm_select_modes");
    check_steps(theta, dt, n_steps);
    const bool many = c->n_probe > kMaxRunColumns;
    MM_REQUIRE(!(many && scan), kInvalid,
               "the time-parallel stepping observes at most 8 probes");
    check_run_columns(c, true);
    MM_REQUIRE(c->n_src == 0 || i_src, kInvalid, "i_src is required");
    MM_REQUIRE(c->m == 0 || i_D, kInvalid, "i_D is required");
    MM_REQUIRE(signal || n_steps == 0, kInvalid, "signal is required");
    if (n_steps == 0) return;
    hipStream_t s = c->stream;
    const int64_t nm = selective ? c->sel_n : c->n0;
    if (many) {
      // a10 for many probes: the steps of a chunk write their amplitude
      // increments dY (nm x L), and the chunk's signals are one product
      // P~^T dY (n_probe x L, i.e. L rows of the row-major signal)
      const int64_t L = std::min(n_steps, dy_chunk_steps(nm));
      c->pp.alloc(sizeof(double) * L * c->n_probe);
      c->tmp.alloc(sizeof(double) * std::max<int64_t>(1, nm) * L);
      const double* Pm = selective ? c->sel_P.d() : c->Pm.d();
      for (int64_t k0 = 0; k0 < n_steps; k0 += L) {
        const int64_t kl = std::min(L, n_steps - k0);
        ModalStep ms;
        ms.n0 = nm;
        ms.lam = selective ? c->sel_lam.d() : c->lam.d();
        ms.W = selective ? c->sel_W.d() : c->Wm.d();
        ms.f.nf = c->nf; ms.f.m = (int)c->m; ms.f.n_src = c->n_src;
        ms.f.i_src = i_src ? i_src + k0 * c->n_src : nullptr;
        ms.f.i_D = i_D ? i_D + k0 * c->m : nullptr;
        ms.n_probe = 0;
        ms.theta = theta; ms.dt = dt;
        ms.exact = exact;
        ms.y = selective ? c->sel_y.d() : c->y.d();
        ms.dy_out = c->tmp.d();
        if (nm > 0) {
          modal_steps(ms, 0, kl, s);
          Gemm g;
          g.m = c->n_probe; g.n = kl; g.k = nm;
          g.A = Pm; g.lda = nm; g.ta = true;
          g.B = c->tmp.d(); g.ldb = nm;
          g.C = c->pp.d(); g.ldc = c->n_probe;
          gemm(g, s);
        } else {
          fill(c->pp.d(), kl * c->n_probe, 0.0, s);
        }
        probe_finish(c->pp.d(), kl, 1, c->n_probe, c->m ? c->PD.d() : nullptr, (int)c->m,
                     i_D ? i_D + k0 * c->m : nullptr, 0, dt, signal + k0 * c->n_probe, s);
      }
      MM_HIP_TRY(hipStreamSynchronize(s));  // the chunk buffers are released here
      c->tmp.release();
      if (c->m && !selective)
        MM_HIP_TRY(hipMemcpyAsync(c->iD_modal.p, i_D + n_steps * c->m, sizeof(double) * c->m,
                                  hipMemcpyDeviceToDevice, s));
      return;
    }
    const int G = modal_groups(nm);
    double* partial = nullptr;
    if (no_alloc) {
      MM_REQUIRE(n_steps * G * c->n_probe <= kScratchDoubles, kInvalid,
                 "mm_step_modal_noalloc: n_steps x ceil(n0 / 256) x n_probe must not exceed "
                 "2^23 (call it on fewer steps at a time)");
      partial = c->scratch;
    } else {
      c->pp.alloc(sizeof(double) * n_steps * G * c->n_probe);
      partial = c->pp.d();
    }
    ModalStep ms;
    ms.n0 = nm;
    ms.lam = selective ? c->sel_lam.d() : c->lam.d();
    ms.W = selective ? c->sel_W.d() : c->Wm.d();
    ms.f.nf = c->nf; ms.f.m = (int)c->m; ms.f.n_src = c->n_src;
    ms.f.i_src = i_src; ms.f.i_D = i_D;
    ms.Pt = selective ? c->sel_P.d() : c->Pm.d();
    ms.n_probe = c->n_probe;
    ms.theta = theta; ms.dt = dt;
    ms.exact = exact;
    ms.y = selective ? c->sel_y.d() : c->y.d();
    ms.probe_partial = partial;
    if (scan && nm > 0) {
      const int64_t L = scan_chunk(nm, n_steps);
      c->scanws.alloc(sizeof(double) * 2 * ceil_div(n_steps, L) * nm);
      modal_steps_scan(ms, n_steps, L, c->scanws.d(), s);
    } else {
      modal_steps(ms, 0, n_steps, s);
    }
    probe_finish(partial, n_steps, G, c->n_probe, c->m ? c->PD.d() : nullptr, (int)c->m,
                 i_D, 0, dt, signal, s);
    // the injected currents belong to the full modal state (current reconstruction)
    if (c->m && !selective)
      MM_HIP_TRY(hipMemcpyAsync(c->iD_modal.p, i_D + n_steps * c->m, sizeof(double) * c->m,
                                hipMemcpyDeviceToDevice, s));
}

}  // namespace

mm_status mm_step_modal(mm_ctx* c, double theta, double dt, int64_t n_steps,
                        const double* i_src, const double* i_D, double* signal) {
  if (!c) return MM_E_INVALID;
  return guarded(c, [&] { step_modal_impl(c, theta, dt, false, n_steps, i_src, i_D, signal); });
}

mm_status mm_step_modal_noalloc(mm_ctx* c, double theta, double dt, int64_t n_steps,
                                const double* i_src, const double* i_D, double* signal) {
  if (!c) return MM_E_INVALID;
  return guarded(c, [&] {
    MM_REQUIRE(c->n_probe <= kMaxRunColumns, kInvalid,
               "mm_step_modal_noalloc: at most 8 probes");
    MM_REQUIRE(c->scratch != nullptr, kState, "mm_step_modal_noalloc: no scratch array");
    step_modal_impl(c, theta, dt, false, n_steps, i_src, i_D, signal, false, false, true);
  });
}

mm_status mm_step_modal_exact(mm_ctx* c, double dt, int64_t n_steps, const double* i_src,
                              const double* i_D, double* signal) {
  if (!c) return MM_E_INVALID;
  return guarded(c, [&] { step_modal_impl(c, 0.5, dt, true, n_steps, i_src, i_D, signal); });
}

mm_status mm_step_modal_scan(mm_ctx* c, double theta, int32_t exact, double dt, int64_t n_steps,
                             const double* i_src, const double* i_D, double* signal) {
  if (!c) return MM_E_INVALID;
  return guarded(c, [&] {
    step_modal_impl(c, exact ? 0.5 : theta, dt, exact != 0, n_steps, i_src, i_D, signal, true);
  });
}

mm_status mm_select_modes(mm_ctx* c, double tol, int64_t* n_kept, int64_t* kept) {
  if (!c) return MM_E_INVALID;
  return guarded(c, [&] {
    MM_REQUIRE(c->decomposed, kState, "mm_select_modes before mm_decompose");
    MM_REQUIRE(std::isfinite(tol) && tol >= 0.0, kInvalid, "tol must be finite and >= 0");
    MM_REQUIRE(n_kept, kInvalid, "n_kept is required");
    hipStream_t s = c->stream;
    const int64_t n0 = c->n0;
    c->selected = false;
    c->sel_score.alloc(sizeof(double) * n0);
    c->sel_idx.alloc(sizeof(int64_t) * (n0 + 1));
    int64_t* idx = c->sel_idx.as<int64_t>();
    select_modes(c->Wm.d(), c->nf, c->Pm.d(), c->n_probe, n0, tol, c->sel_score.d(), idx,
                 idx + n0, s);
    int64_t nk = 0;
    MM_HIP_TRY(hipMemcpyAsync(&nk, idx + n0, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    MM_HIP_TRY(hipStreamSynchronize(s));
    MM_REQUIRE(nk >= 0 && nk <= n0, kDevice, "mm_select_modes: kept count out of range");
    const int64_t cap = std::max<int64_t>(nk, 1);
    c->sel_lam.alloc(sizeof(double) * cap);
    c->sel_W.alloc(sizeof(double) * cap * std::max(1, c->nf));
    c->sel_P.alloc(sizeof(double) * cap * std::max(1, c->n_probe));
    c->sel_y.alloc(sizeof(double) * cap);
    gather_modes(idx, nk, n0, c->lam.d(), c->Wm.d(), c->nf, c->Pm.d(), c->n_probe, c->y.d(),
                 c->sel_lam.d(), c->sel_W.d(), c->sel_P.d(), c->sel_y.d(), s);
    if (kept && nk > 0)
      MM_HIP_TRY(hipMemcpyAsync(kept, idx, sizeof(int64_t) * nk, hipMemcpyDeviceToDevice, s));
    c->sel_n = nk;
    c->selected = true;
    *n_kept = nk;
  });
}

mm_status mm_step_modal_selective(mm_ctx* c, double theta, uint32_t flags, double dt,
                                  int64_t n_steps, const double* i_src, const double* i_D,
                                  double* signal) {
  if (!c) return MM_E_INVALID;
  return guarded(c, [&] {
    MM_REQUIRE((flags & ~(MM_STEP_EXACT | MM_STEP_SCAN)) == 0, kInvalid, "unknown flags");
    const bool exact = (flags & MM_STEP_EXACT) != 0;
    step_modal_impl(c, exact ? 0.5 : theta, dt, exact, n_steps, i_src, i_D, signal,
                    (flags & MM_STEP_SCAN) != 0, true);
  });
}

mm_status mm_modal_phasors(mm_ctx* c, int64_t n_w, const double* omega, const double* amp_src,
                           const double* amp_D, double* out) {
  if (!c) return MM_E_INVALID;
  return guarded(c, [&] {
    MM_REQUIRE(c->decomposed, kState, "mm_modal_phasors before mm_decompose");
    MM_REQUIRE(n_w >= 0, kInvalid, "n_w must be >= 0");
    check_run_columns(c);
    if (n_w == 0) return;
    MM_REQUIRE(omega && out, kInvalid, "omega and out are required");
    MM_REQUIRE(c->n_src == 0 || amp_src, kInvalid, "amp_src is required");
    MM_REQUIRE(c->m == 0 || amp_D, kInvalid, "amp_D is required");
    hipStream_t s = c->stream;
    c->pp.alloc(sizeof(double) * n_w * phasor_groups(c->n0) * c->n_probe * 2);
    ModalPhasor mp;
    mp.n0 = c->n0;
    mp.lam = c->lam.d();
    mp.W = c->Wm.d();
    mp.Pt = c->Pm.d();
    mp.PD = c->m ? c->PD.d() : nullptr;
    mp.m = (int)c->m; mp.n_src = c->n_src; mp.n_probe = c->n_probe;
    mp.n_w = n_w;
    mp.omega = omega; mp.amp_src = amp_src; mp.amp_D = amp_D;
    mp.partial = c->pp.d();
    mp.out = out;
    modal_phasors(mp, s);
  });
}

mm_status mm_step_cholesky(mm_ctx* c, double theta, double dt, int64_t n_steps,
                           const double* i_src, const double* i_D, double* signal) {
  if (!c) return MM_E_INVALID;
  return guarded(c, [&] {
    check_steps(theta, dt, n_steps);
    check_run_columns(c, true);
    MM_REQUIRE(c->n_src == 0 || i_src, kInvalid, "i_src is required");
    MM_REQUIRE(c->m == 0 || i_D, kInvalid, "i_D is required");
    MM_REQUIRE(signal || n_steps == 0, kInvalid, "signal is required");
    hipStream_t s = c->stream;
    const int64_t n0 = c->n0;
    const int B = trsv_block(n0);
    const int64_t NB = ceil_div(n0, B);
    if (!c->I.p) {
      c->I.alloc(sizeof(double) * n0);
      fill(c->I.d(), n0, 0.0, s);
    }
    if (!c->factored || c->f_theta != theta || c->f_dt != dt) {
      c->factored = false;
      c->Z.alloc(sizeof(double) * n0 * n0);
      c->Dinv.alloc(sizeof(double) * NB * B * B);
      c->DinvT.alloc(sizeof(double) * NB * B * B);
      c->b.alloc(sizeof(double) * n0);
      c->yv.alloc(sizeof(double) * n0);
      c->kstep.alloc(2 * sizeof(int64_t));
      // b0: Z = Li + theta dt Ri = C C^T   (Ne = 0: Li = L, Ri = R)
      double* Z = c->Z.d();
      const int m = (int)c->m;
      assemble_L(c->lsrc(m), n0, Z, n0, false, s, c->lr(theta * dt));
      add_csr_lower(Z, n0, theta * dt, c->R(), s);
      factor_checked(Z, n0, c->status.as<int64_t>(), c->tmp, s, "Li + theta dt Ri");
      c->tmp.alloc(sizeof(double) * trtri_ws_elems(B));
      diag_block_inverses(Z, n0, n0, B, c->Dinv.d(), c->tmp.d(), trtri_ws_elems(B), s);
      transpose_blocks(c->Dinv.d(), NB, B, c->DinvT.d(), s);
      const int64_t pe = trsv_panel_elems(n0, B);
      c->panels.alloc(sizeof(double) * std::max<int64_t>(pe, 1));
      const int64_t nfwd = pe - (int64_t)B * B * (NB * (NB - 1) / 2);
      trsv_prescale(Z, n0, B, c->Dinv.d(), c->panels.d(), c->panels.d() + nfwd, s);
      MM_HIP_TRY(hipStreamSynchronize(s));
      c->tmp.release();
      c->Z.release();  // the steps read only the panels and the block inverses
      c->factored = true;
      c->f_theta = theta;
      c->f_dt = dt;
    }
    if (n_steps == 0) return;
    const int64_t parts = trsv_parts(n0);
    if (c->n_probe <= kMaxRunColumns) c->pp.alloc(sizeof(double) * n_steps * parts * c->n_probe);
    CholStep cs;
    cs.n0 = n0;
    {
      const int64_t nfwd = trsv_panel_elems(n0, B) - (int64_t)B * B * (NB * (NB - 1) / 2);
      cs.pf = c->panels.d();
      cs.pb = c->panels.d() + nfwd;
    }
    cs.B = B;
    cs.Dinv = c->Dinv.d();
    cs.DinvT = c->DinvT.d();
    cs.kstep = c->kstep.as<int64_t>();
    cs.use_graph = c->use_graph;
    cs.Ri = c->R();
    cs.Rlr = c->Rlr();
    cs.f.F = c->F.d(); cs.f.nf = c->nf; cs.f.m = (int)c->m; cs.f.n_src = c->n_src;
    cs.f.i_src = i_src; cs.f.i_D = i_D;
    cs.theta = theta; cs.dt = dt;
    cs.I = c->I.d(); cs.b = c->b.d(); cs.y = c->yv.d();
    cs.Pt = c->Pt.d(); cs.n_probe = c->n_probe;
    cs.probe_partial = c->pp.d();
    if (c->n_probe > kMaxRunColumns) {
      // many probes (b4): the steps of a chunk write their increments dI
      // (n0 x L), and the chunk's signals are one product P^T dI
      const int64_t L = std::min(n_steps, dy_chunk_steps(n0));
      c->pp.alloc(sizeof(double) * L * c->n_probe);
      c->tmp.alloc(sizeof(double) * n0 * L);
      cs.n_probe = 0;
      cs.probe_partial = nullptr;
      cs.dI_out = c->tmp.d();
      for (int64_t k0 = 0; k0 < n_steps; k0 += L) {
        const int64_t kl = std::min(L, n_steps - k0);
        cs.f.i_src = i_src ? i_src + k0 * c->n_src : nullptr;
        cs.f.i_D = i_D ? i_D + k0 * c->m : nullptr;
        chol_steps(cs, 0, kl, s);
        Gemm g;
        g.m = c->n_probe; g.n = kl; g.k = n0;
        g.A = c->Pt.d(); g.lda = n0; g.ta = true;
        g.B = c->tmp.d(); g.ldb = n0;
        g.C = c->pp.d(); g.ldc = c->n_probe;
        gemm(g, s);
        probe_finish(c->pp.d(), kl, 1, c->n_probe, c->m ? c->PD.d() : nullptr, (int)c->m,
                     i_D ? i_D + k0 * c->m : nullptr, 0, dt, signal + k0 * c->n_probe, s);
      }
      MM_HIP_TRY(hipStreamSynchronize(s));  // the chunk buffer is released here
      c->tmp.release();
    } else {
      chol_steps(cs, 0, n_steps, s);
      probe_finish(c->pp.d(), n_steps, parts, c->n_probe, c->m ? c->PD.d() : nullptr,
                   (int)c->m, i_D, 0, dt, signal, s);
    }
    if (c->m)
      MM_HIP_TRY(hipMemcpyAsync(c->iD_chol.p, i_D + n_steps * c->m, sizeof(double) * c->m,
                                hipMemcpyDeviceToDevice, s));
  });
}

mm_status mm_probe(mm_ctx* c, int32_t which, int32_t n_rows, const double* rows, double* out) {
  if (!c) return MM_E_INVALID;
  return guarded(c, [&] {
    MM_REQUIRE(out != nullptr, kInvalid, "out is NULL");
    MM_REQUIRE(which == MM_MODAL || which == MM_CHOLESKY, kInvalid, "which");
    MM_REQUIRE(rows == nullptr || n_rows >= 1, kInvalid, "n_rows");
    hipStream_t s = c->stream;
    const int64_t n = c->n, n0 = c->n0;
    const int m = (int)c->m;
    Dev buf;
    buf.alloc(sizeof(double) * (n0 + n));
    double* Ii = buf.d();           // reduced current (n0)
    double* Ifull = buf.d() + n0;   // full current (n)
    if (which == MM_MODAL) {
      MM_REQUIRE(c->decomposed, kState, "mm_probe(MM_MODAL) before mm_decompose");
      MM_REQUIRE(c->has_V, kState,
                 "mm_probe(MM_MODAL) needs the eigenvectors: use mm_decompose, not "
                 "mm_decompose_projected");
      // a11: Ii = V y  (V = G^{-T} Q)
      Gemm g;
      g.m = n0; g.n = 1; g.k = n0;
      g.A = c->V.d(); g.lda = n0;
      g.B = c->y.d(); g.ldb = n0;
      g.C = Ii; g.ldc = n0;
      gemm(g, s);
    } else {
      MM_REQUIRE(c->I.p != nullptr, kState, "mm_probe(MM_CHOLESKY) before any Cholesky step");
      MM_HIP_TRY(hipMemcpyAsync(Ii, c->I.p, sizeof(double) * n0, hipMemcpyDeviceToDevice, s));
    }
    if (m == 0) {
      MM_HIP_TRY(hipMemcpyAsync(Ifull, Ii, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    } else {
      // I = K Ii + A_D iD = H [Re^{-T} iD ; Ii]
      const double* iD = (which == MM_MODAL ? c->iD_modal : c->iD_chol).d();
      electrode_lift(c->RinvT(), iD, m, Ii, n0, Ifull, s);
      const int64_t wse = apply_h_ws_elems(m, 1);
      Dev ws;
      ws.alloc(sizeof(double) * wse);
      apply_h(c->Vh.d(), c->T(), n, m, Ifull, n, 1, false, ws.d(), wse, s);
      MM_HIP_TRY(hipStreamSynchronize(s));  // ws is released here
    }
    if (!rows) {
      MM_HIP_TRY(hipMemcpyAsync(out, Ifull, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    } else {
      Gemm g;
      g.m = n_rows; g.n = 1; g.k = n;
      g.A = rows; g.lda = n; g.ta = true;
      g.B = Ifull; g.ldb = n;
      g.C = out; g.ldc = n_rows;
      gemm(g, s);
    }
    MM_HIP_TRY(hipStreamSynchronize(s));
  });
}

mm_status mm_reset_state(mm_ctx* c) {
  if (!c) return MM_E_INVALID;
  return guarded(c, [&] {
    if (c->y.p) fill(c->y.d(), c->n0, 0.0, c->stream);
    if (c->selected && c->sel_n > 0) fill(c->sel_y.d(), c->sel_n, 0.0, c->stream);
    if (c->I.p) fill(c->I.d(), c->n0, 0.0, c->stream);
    if (c->m) {
      fill(c->iD_modal.d(), c->m, 0.0, c->stream);
      fill(c->iD_chol.d(), c->m, 0.0, c->stream);
    }
  });
}

namespace {

// The state vector of one method: its reduced unknowns (n0) and the injected
// currents of its last step (m).
double* state_of(mm_ctx* c, int32_t which, bool create) {
  MM_REQUIRE(which == MM_MODAL || which == MM_CHOLESKY, kInvalid, "which");
  if (which == MM_MODAL) {
    MM_REQUIRE(c->decomposed, kState, "the modal state exists after mm_decompose");
    return c->y.d();
  }
  if (!c->I.p) {
    MM_REQUIRE(create, kState, "no Cholesky step has run");
    c->I.alloc(sizeof(double) * c->n0);
    fill(c->I.d(), c->n0, 0.0, c->stream);
  }
  return c->I.d();
}

}  // namespace

mm_status mm_get_state(mm_ctx* c, int32_t which, double* out) {
  if (!c) return MM_E_INVALID;
  return guarded(c, [&] {
    MM_REQUIRE(out != nullptr, kInvalid, "out is NULL");
    const double* st = state_of(c, which, false);
    hipStream_t s = c->stream;
    MM_HIP_TRY(hipMemcpyAsync(out, st, sizeof(double) * c->n0, hipMemcpyDeviceToDevice, s));
    if (c->m)
      MM_HIP_TRY(hipMemcpyAsync(out + c->n0, (which == MM_MODAL ? c->iD_modal : c->iD_chol).p,
                                sizeof(double) * c->m, hipMemcpyDeviceToDevice, s));
  });
}

mm_status mm_set_state(mm_ctx* c, int32_t which, const double* in) {
  if (!c) return MM_E_INVALID;
  return guarded(c, [&] {
    MM_REQUIRE(in != nullptr, kInvalid, "in is NULL");
    double* st = state_of(c, which, true);
    hipStream_t s = c->stream;
    MM_HIP_TRY(hipMemcpyAsync(st, in, sizeof(double) * c->n0, hipMemcpyDeviceToDevice, s));
    if (c->m)
      MM_HIP_TRY(hipMemcpyAsync((which == MM_MODAL ? c->iD_modal : c->iD_chol).p, in + c->n0,
                                sizeof(double) * c->m, hipMemcpyDeviceToDevice, s));
  });
}

mm_status mm_eigenvalues(mm_ctx* c, double* out) {
  if (!c) return MM_E_INVALID;
  return guarded(c, [&] {
    MM_REQUIRE(c->decomposed, kState, "mm_eigenvalues before mm_decompose");
    MM_REQUIRE(out != nullptr, kInvalid, "out is NULL");
    MM_HIP_TRY(hipMemcpyAsync(out, c->lam.p, sizeof(double) * c->n0, hipMemcpyDeviceToDevice,
                              c->stream));
  });
}

}  // extern "C"

struct mm_batch {
  mm_ctx* ctx = nullptr;
  int n_runs = 0;
  int64_t total_steps = 0;
  int tile = 0;
  BatchStep bs;
  Dev order, lens, woff, soff, wcol, pcol, partial;
  double* signals = nullptr;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~mm_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

namespace {

template <class T>
void upload(Dev& d, const std::vector<T>& v, hipStream_t s) {
  d.alloc(sizeof(T) * std::max<size_t>(1, v.size()));
  if (!v.empty())
    MM_HIP_TRY(hipMemcpyAsync(d.p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s));
}

// Time one launch of tile `tile` on the batch truncated to `tcap` steps per
// run (the autotuner's sample).
float time_tile(mm_batch* b, int tile, int64_t tcap, hipStream_t s) {
  const int n = b->n_runs;
  std::vector<int64_t> lens(n), soff(n);
  std::vector<int64_t> hl(n);
  MM_HIP_TRY(hipMemcpyAsync(hl.data(), b->lens.p, sizeof(int64_t) * n, hipMemcpyDeviceToHost, s));
  MM_HIP_TRY(hipStreamSynchronize(s));
  int64_t acc = 0;
  for (int r = 0; r < n; ++r) {
    lens[r] = std::min(hl[r], tcap);
    soff[r] = acc;
    acc += lens[r];
  }
  Dev dl, ds, part;
  upload(dl, lens, s);
  upload(ds, soff, s);
  BatchStep t = b->bs;
  t.lens = dl.as<int64_t>();
  t.soff = ds.as<int64_t>();
  t.G = batch_groups(t.n0, tile);
  part.alloc(sizeof(double) * std::max<int64_t>(1, acc) * t.G);
  t.partial = part.d();
  hipEvent_t e0, e1;
  MM_HIP_TRY(hipEventCreate(&e0));
  MM_HIP_TRY(hipEventCreate(&e1));
  batch_steps(t, tile, 0, nullptr, s);  // warm-up
  MM_HIP_TRY(hipEventRecord(e0, s));
  batch_steps(t, tile, 0, nullptr, s);
  batch_steps(t, tile, 0, nullptr, s);
  MM_HIP_TRY(hipEventRecord(e1, s));
  MM_HIP_TRY(hipEventSynchronize(e1));
  float ms = 0.f;
  MM_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms;
}

}  // namespace

extern "C" {

mm_status mm_batch_create(mm_ctx* c, double theta, double dt, int32_t n_runs,
                          const int64_t* lens, const int32_t* src, const int32_t* probe,
                          const double* waves, double* signals, int32_t tile, mm_batch** out) {
  if (!c || !out) return MM_E_INVALID;
  *out = nullptr;
  mm_batch* b = nullptr;
  mm_status st = guarded(c, [&] {
    MM_REQUIRE(c->decomposed, kState, "mm_batch_create before mm_decompose");
    check_steps(theta, dt, 0);
    MM_REQUIRE(n_runs >= 1 && lens && src && probe, kInvalid, "n_runs >= 1, lens, src, probe");
    MM_REQUIRE(tile >= -1 && tile < kNumBatchTiles, kInvalid, "tile must be -1 or a tile index");
    b = new mm_batch();
    b->ctx = c;
    b->n_runs = n_runs;
    hipStream_t s = c->stream;
    std::vector<int64_t> hl(n_runs), woff(n_runs), soff(n_runs);
    std::vector<int32_t> wcol(n_runs), pcol(n_runs), order(n_runs);
    int64_t ws = 0, ss = 0;
    for (int r = 0; r < n_runs; ++r) {
      MM_REQUIRE(lens[r] >= 0, kInvalid, "run lengths must be >= 0");
      MM_REQUIRE(src[r] >= 0 && src[r] < c->n_src, kInvalid, "source index out of range");
      MM_REQUIRE(probe[r] >= 0 && probe[r] < c->n_probe, kInvalid, "probe index out of range");
      hl[r] = lens[r];
      woff[r] = ws;
      soff[r] = ss;
      ws += lens[r] + 1;
      ss += lens[r];
      wcol[r] = 2 * (int32_t)c->m + src[r];  // forcing column of source src[r]
      pcol[r] = probe[r];
      order[r] = r;
    }
    MM_REQUIRE(ss == 0 || (waves && signals), kInvalid, "waves and signals are required");
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int q) { return hl[a] > hl[q]; });  // longest first
    b->total_steps = ss;
    b->signals = signals;
    upload(b->order, order, s);
    upload(b->lens, hl, s);
    upload(b->woff, woff, s);
    upload(b->soff, soff, s);
    upload(b->wcol, wcol, s);
    upload(b->pcol, pcol, s);
    BatchStep& t = b->bs;
    t.n0 = c->n0;
    t.lam = c->lam.d();
    t.W = c->Wm.d();
    t.ldw = c->n0;
    t.Pm = c->Pm.d();
    t.theta = theta;
    t.dt = dt;
    t.n_runs = n_runs;
    t.order = b->order.as<int32_t>();
    t.lens = b->lens.as<int64_t>();
    t.woff = b->woff.as<int64_t>();
    t.soff = b->soff.as<int64_t>();
    t.wcol = b->wcol.as<int32_t>();
    t.pcol = b->pcol.as<int32_t>();
    t.waves = waves;
    // autotuner: time every tile on the batch cut to 256 steps per run
    if (tile < 0) {
      float best = 0.f;
      for (int q = 0; q < kNumBatchTiles; ++q) {
        const float ms = time_tile(b, q, 256, s);
        if (q == 0 || ms < best) {
          best = ms;
          tile = q;
        }
      }
    }
    b->tile = tile;
    t.G = batch_groups(c->n0, tile);
    b->partial.alloc(sizeof(double) * std::max<int64_t>(1, ss) * t.G);
    t.partial = b->partial.d();
    // one graph: the stepping launch and the signal pass
    MM_HIP_TRY(hipStreamSynchronize(s));
    MM_HIP_TRY(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    MM_HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    batch_steps(t, tile, ss, signals, b->cap);
    MM_HIP_TRY(hipStreamEndCapture(b->cap, &b->graph));
    MM_HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  });
  if (st != MM_OK) {
    delete b;
    return st;
  }
  *out = b;
  return MM_OK;
}

mm_status mm_batch_run(mm_batch* b) {
  if (!b) return MM_E_INVALID;
  return guarded(b->ctx, [&] {
    MM_HIP_TRY(hipGraphLaunch(b->exec, b->ctx->stream));
  });
}

mm_status mm_batch_info(const mm_batch* b, int64_t* out) {
  if (!b || !out) return MM_E_INVALID;
  out[0] = kBatchTiles[b->tile].threads;
  out[1] = kBatchTiles[b->tile].modes;
  out[2] = b->bs.G;
  out[3] = b->total_steps;
  return MM_OK;
}

void mm_batch_destroy(mm_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->ctx->stream);
  delete b;
}

mm_status mm_adjoint_modal(mm_ctx* c, double theta, double dt, int64_t n_steps,
                           int32_t n_runs, const int32_t* src, const int32_t* probe,
                           const double* i_src, const double* s_obs, int64_t ckpt_every,
                           double* J, double* dJ_dR, double* dJ_di) {
  if (!c) return MM_E_INVALID;
  return guarded(c, [&] {
    MM_REQUIRE(c->decomposed, kState, "mm_adjoint_modal before mm_decompose");
    MM_REQUIRE(c->has_V, kState,
               "mm_adjoint_modal needs the eigenvectors: use mm_decompose, not "
               "mm_decompose_projected");
    check_steps(theta, dt, n_steps);
    MM_REQUIRE(c->m == 0, kInvalid, "mm_adjoint_modal: problems without electrodes only");
    MM_REQUIRE(n_steps >= 1 && n_runs >= 1 && src && probe, kInvalid,
               "n_steps >= 1, n_runs >= 1, src and probe are required");
    MM_REQUIRE(ckpt_every >= 1, kInvalid, "ckpt_every >= 1");
    MM_REQUIRE(i_src && s_obs && J && dJ_dR && dJ_di, kInvalid, "missing array argument");
    hipStream_t s = c->stream;
    const int64_t n0 = c->n0, T = n_steps;
    std::vector<int32_t> wcol(n_runs), pcol(n_runs);
    for (int r = 0; r < n_runs; ++r) {
      MM_REQUIRE(src[r] >= 0 && src[r] < c->n_src, kInvalid, "source index out of range");
      MM_REQUIRE(probe[r] >= 0 && probe[r] < c->n_probe, kInvalid, "probe index out of range");
      wcol[r] = src[r];
      pcol[r] = probe[r];
    }
    Dev dw, dp, ckpt, psig, resid, sq, nu, pu, du;
    upload(dw, wcol, s);
    upload(dp, pcol, s);
    AdjointStep a;
    a.n0 = n0; a.T = T; a.K = std::min(ckpt_every, T); a.n_ckpt = ceil_div(T, a.K);
    a.G = adjoint_groups(n0); a.n_runs = n_runs;
    a.lam = c->lam.d(); a.W = c->Wm.d(); a.ldw = n0; a.Pm = c->Pm.d();
    a.wcol = dw.as<int32_t>(); a.pcol = dp.as<int32_t>();
    a.theta = theta; a.dt = dt;
    a.wave = i_src; a.obs = s_obs;
    ckpt.alloc(sizeof(double) * n_runs * a.n_ckpt * n0);
    psig.alloc(sizeof(double) * n_runs * T * a.G);
    resid.alloc(sizeof(double) * n_runs * T);
    sq.alloc(sizeof(double) * n_runs * T);
    nu.alloc(sizeof(double) * n_runs * n0);
    pu.alloc(sizeof(double) * n_runs * T * a.G);
    du.alloc(sizeof(double) * T);
    a.ckpt = ckpt.d(); a.part_sig = psig.d(); a.resid = resid.d(); a.nu = nu.d();
    a.part_u = pu.d();
    fill(nu.d(), n_runs * n0, 0.0, s);
    adjoint_forward(a, J, sq.d(), s);
    // backward over the segments, last first; S += L Z^T per segment
    Dev S, Zb, Lb;
    S.alloc(sizeof(double) * n0 * n0);
    const int64_t cols = (int64_t)n_runs * a.K;
    Zb.alloc(sizeof(double) * n0 * cols);
    Lb.alloc(sizeof(double) * n0 * cols);
    for (int64_t j = a.n_ckpt - 1; j >= 0; --j) {
      const int64_t k0 = j * a.K, k1 = std::min(T, k0 + a.K);
      if (k1 - k0 < a.K) {  // short last segment: its unused columns must be zero
        fill(Zb.d(), n0 * cols, 0.0, s);
        fill(Lb.d(), n0 * cols, 0.0, s);
      }
      adjoint_segment(a, k0, k1, Zb.d(), Lb.d(), s);
      Gemm g;
      g.m = n0; g.n = n0; g.k = cols;
      g.beta = (j == a.n_ckpt - 1) ? 0.0 : 1.0;
      g.A = Lb.d(); g.lda = n0;
      g.B = Zb.d(); g.ldb = n0; g.tb = true;
      g.C = S.d(); g.ldc = n0;
      gemm(g, s);
    }
    adjoint_waveform_grad(a, du.d(), dJ_di, s);
    MM_HIP_TRY(hipStreamSynchronize(s));  // Zb, Lb released below
    Zb.release();
    Lb.release();
    // dJ/dR = -V S V^T at the stored entries (V = G^{-T} Q, the pencil's
    // eigenvectors)
    Dev T1;
    T1.alloc(sizeof(double) * n0 * n0);
    const double* V = c->V.d();
    {
      Gemm g;
      g.m = n0; g.n = n0; g.k = n0;
      g.A = V; g.lda = n0;
      g.B = S.d(); g.ldb = n0;
      g.C = T1.d(); g.ldc = n0;
      gemm(g, s);
    }
    {
      Gemm g;  // Phi = T1 V^T, into S's storage
      g.m = n0; g.n = n0; g.k = n0;
      g.A = T1.d(); g.lda = n0;
      g.B = V; g.ldb = n0; g.tb = true;
      g.C = S.d(); g.ldc = n0;
      gemm(g, s);
    }
    adjoint_gather(c->Rfull(), S.d(), n0, dJ_dR, s);
    MM_HIP_TRY(hipStreamSynchronize(s));
  });
}

mm_status mm_info(const mm_ctx* c, int64_t* out) {
  if (!c || !out) return MM_E_INVALID;
  out[0] = c->n;
  out[1] = c->n0;
  out[2] = c->decomposed ? 1 : 0;
  return MM_OK;
}

void mm_destroy(mm_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  delete c;
}

const char* mm_last_error(const mm_ctx* c) { return c ? c->err.c_str() : g_err.c_str(); }

// ---------------------------------------------------------------------------
// building blocks
// ---------------------------------------------------------------------------
mm_status mmk_dgemm(int32_t ta, int32_t tb, int64_t m, int64_t n, int64_t k, double alpha,
                    const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                    double* C, int64_t ldc, void* stream) {
  return guarded(nullptr, [&] {
    MM_REQUIRE(m >= 0 && n >= 0 && k >= 0, kInvalid, "negative size");
    MM_REQUIRE(ldc >= std::max<int64_t>(1, m), kInvalid, "ldc");
    Gemm g;
    g.m = m; g.n = n; g.k = k; g.alpha = alpha; g.beta = beta;
    g.A = A; g.lda = lda; g.ta = ta != 0;
    g.B = B; g.ldb = ldb; g.tb = tb != 0;
    g.C = C; g.ldc = ldc;
    Dev ws;
    const int64_t wse = 8 * std::max<int64_t>(1, m * n);
    if (k >= 2048 && m * n <= ((int64_t)1 << 24)) ws.alloc(sizeof(double) * wse);
    gemm(g, (hipStream_t)stream, ws.p ? ws.d() : nullptr, ws.p ? wse : 0);
    MM_HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  });
}

mm_status mmk_dgemm_tri(int32_t ta, int32_t tb, int64_t m, int64_t n, int64_t k, double alpha,
                        const double* A, int64_t lda, const double* B, int64_t ldb,
                        double beta, double* C, int64_t ldc, int32_t flags, int64_t b_band,
                        void* stream) {
  return guarded(nullptr, [&] {
    MM_REQUIRE(m >= 0 && n >= 0 && k >= 0, kInvalid, "negative size");
    MM_REQUIRE(ldc >= std::max<int64_t>(1, m), kInvalid, "ldc");
    MM_REQUIRE((flags & ~15) == 0 && b_band >= -1, kInvalid, "flags or b_band");
    Gemm g;
    g.m = m; g.n = n; g.k = k; g.alpha = alpha; g.beta = beta;
    g.A = A; g.lda = lda; g.ta = ta != 0;
    g.B = B; g.ldb = ldb; g.tb = tb != 0;
    g.C = C; g.ldc = ldc;
    g.lower = (flags & MMK_LOWER) != 0;
    g.a_lower = (flags & MMK_A_LOWER) != 0;
    g.a_upper = (flags & MMK_A_UPPER) != 0;
    g.b_lower = (flags & MMK_B_LOWER) != 0;
    g.b_band = b_band;
    gemm(g, (hipStream_t)stream);
    MM_HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  });
}

mm_status mmk_dsymm_lower(int64_t m, int64_t n, double alpha, const double* A, int64_t lda,
                          const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                          void* stream) {
  return guarded(nullptr, [&] {
    MM_REQUIRE(m >= 0 && n >= 0, kInvalid, "negative size");
    MM_REQUIRE(lda >= std::max<int64_t>(1, m) && ldb >= std::max<int64_t>(1, m) &&
                   ldc >= std::max<int64_t>(1, m), kInvalid, "lda, ldb or ldc");
    Gemm g;
    g.m = m; g.n = n; g.k = m; g.alpha = alpha; g.beta = beta;
    g.A = A; g.lda = lda; g.a_sym = true;
    g.B = B; g.ldb = ldb;
    g.C = C; g.ldc = ldc;
    Dev ws;  // split-K partials for tall, narrow products
    const int64_t wse = 8 * std::max<int64_t>(1, m * n);
    if (m >= 4096 && m * n <= ((int64_t)1 << 24)) ws.alloc(sizeof(double) * wse);
    gemm(g, (hipStream_t)stream, ws.p ? ws.d() : nullptr, ws.p ? wse : 0);
    MM_HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  });
}

mm_status mmk_dpotrf(int64_t n, double* A, int64_t lda, int64_t* info, void* stream) {
  return guarded(nullptr, [&] {
    MM_REQUIRE(n >= 0 && lda >= std::max<int64_t>(1, n), kInvalid, "n or lda");
    hipStream_t s = (hipStream_t)stream;
    Dev ws, st;
    ws.alloc(sizeof(double) * potrf_ws_elems(n));
    st.alloc(sizeof(int64_t));
    fill_i64(st.as<int64_t>(), 1, INT64_MAX, s);
    potrf_lower(A, lda, n, ws.d(), potrf_ws_elems(n), st.as<int64_t>(), s);
    int64_t piv = INT64_MAX;
    MM_HIP_TRY(hipMemcpyAsync(&piv, st.p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    MM_HIP_TRY(hipStreamSynchronize(s));
    if (info) *info = (piv == INT64_MAX) ? -1 : piv;
  });
}

mm_status mmk_dtrtri(int64_t n, double* A, int64_t lda, void* stream) {
  return guarded(nullptr, [&] {
    MM_REQUIRE(n >= 0 && lda >= std::max<int64_t>(1, n), kInvalid, "n or lda");
    hipStream_t s = (hipStream_t)stream;
    Dev ws;
    ws.alloc(sizeof(double) * trtri_ws_elems(n));
    trtri_lower(A, lda, n, ws.d(), trtri_ws_elems(n), s);
    MM_HIP_TRY(hipStreamSynchronize(s));
  });
}

mm_status mmk_dsy2sb(int64_t n, double* A, int64_t lda, int32_t nb, double* AB, int64_t ldab,
                     void* stream) {
  return guarded(nullptr, [&] {
    MM_REQUIRE(n >= 1 && nb >= 1 && nb <= 64 && ldab >= 2 * nb + 1, kInvalid, "sizes");
    hipStream_t s = (hipStream_t)stream;
    Dev ws, tau, T;
    const int64_t np = std::max<int64_t>(1, sy2sb_npanels(n, nb));
    ws.alloc(sizeof(double) * sy2sb_ws_elems(n, nb));
    tau.alloc(sizeof(double) * np * nb);
    T.alloc(sizeof(double) * np * nb * nb);
    sy2sb(A, lda, n, nb, tau.d(), T.d(), ws.d(), sy2sb_ws_elems(n, nb), s);
    extract_band(A, lda, n, nb, AB, ldab, s);
    MM_HIP_TRY(hipStreamSynchronize(s));
  });
}

mm_status mmk_dsb2st(int64_t n, int32_t nb, double* AB, int64_t ldab, double* d, double* e,
                     void* stream) {
  return guarded(nullptr, [&] {
    MM_REQUIRE(n >= 1 && nb >= 1 && nb <= 64 && ldab >= 2 * nb + 1, kInvalid, "sizes");
    hipStream_t s = (hipStream_t)stream;
    Sb2stPlan plan = sb2st_plan(n, nb);
    Dev off, V2, tau2;
    off.alloc(sizeof(int64_t) * (n + 1));
    V2.alloc(sizeof(double) * std::max<int64_t>(1, plan.tasks) * nb);
    tau2.alloc(sizeof(double) * std::max<int64_t>(1, plan.tasks));
    MM_HIP_TRY(hipMemcpyAsync(off.p, plan.offset.data(), sizeof(int64_t) * (n + 1),
                              hipMemcpyHostToDevice, s));
    sb2st(AB, ldab, plan, off.as<int64_t>(), V2.d(), tau2.d(), d, e, s);
    MM_HIP_TRY(hipStreamSynchronize(s));
  });
}

mm_status mmk_dstedc(int64_t n, const double* d, const double* e, double* w, double* Z,
                     void* stream) {
  return guarded(nullptr, [&] {
    MM_REQUIRE(n >= 1, kInvalid, "n");
    hipStream_t s = (hipStream_t)stream;
    Dev ws, U, st;
    ws.alloc(sizeof(double) * stedc_ws_elems(n));
    U.alloc(sizeof(double) * n * n);
    st.alloc(sizeof(int64_t));
    fill_i64(st.as<int64_t>(), 1, 0, s);
    stedc(d, e, n, w, Z, n, U.d(), ws.d(), stedc_ws_elems(n), st.as<int64_t>(), s);
    int64_t est = 0;
    MM_HIP_TRY(hipMemcpyAsync(&est, st.p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    MM_HIP_TRY(hipStreamSynchronize(s));
    if (est != 0) throw Error{kNoConverge, "a secular equation did not converge"};
  });
}

mm_status mmk_dsyevd(int64_t n, double* A, int64_t lda, int32_t nb, double* w, double* Z,
                     void* stream) {
  return guarded(nullptr, [&] {
    MM_REQUIRE(n >= 1 && nb >= 1 && nb <= 64 && lda >= n, kInvalid, "sizes");
    hipStream_t s = (hipStream_t)stream;
    Sb2stPlan plan = sb2st_plan(n, nb);
    const int64_t wse = eig_ws_elems(n, nb);
    Dev ws, tau1, T1, AB, V2, tau2, off, dv, ev, st;
    const int64_t np = std::max<int64_t>(1, sy2sb_npanels(n, nb));
    ws.alloc(sizeof(double) * wse);
    tau1.alloc(sizeof(double) * np * nb);
    T1.alloc(sizeof(double) * np * nb * nb);
    AB.alloc(sizeof(double) * (2 * nb + 1) * n);
    V2.alloc(sizeof(double) * std::max<int64_t>(1, plan.tasks) * nb);
    tau2.alloc(sizeof(double) * std::max<int64_t>(1, plan.tasks));
    off.alloc(sizeof(int64_t) * (n + 1));
    dv.alloc(sizeof(double) * n);
    ev.alloc(sizeof(double) * n);
    st.alloc(sizeof(int64_t));
    MM_HIP_TRY(hipMemcpyAsync(off.p, plan.offset.data(), sizeof(int64_t) * (n + 1),
                              hipMemcpyHostToDevice, s));
    fill_i64(st.as<int64_t>(), 1, 0, s);
    EigWork wk;
    wk.nb = nb;
    wk.tau1 = tau1.d(); wk.T1 = T1.d(); wk.AB = AB.d(); wk.V2 = V2.d(); wk.tau2 = tau2.d();
    wk.d_offset = off.as<int64_t>(); wk.d = dv.d(); wk.e = ev.d();
    wk.ws = ws.d(); wk.ws_elems = wse;
    syevd(A, lda, n, w, Z, n, wk, plan, st.as<int64_t>(), s);
    int64_t est = 0;
    MM_HIP_TRY(hipMemcpyAsync(&est, st.p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    MM_HIP_TRY(hipStreamSynchronize(s));
    if (est != 0) throw Error{kNoConverge, "a secular equation did not converge"};
  });
}

}  // extern "C"
