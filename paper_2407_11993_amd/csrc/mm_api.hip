// C ABI of libmm (declared in include/mm.h).  Host-side orchestration only:
// every arithmetic step of the method runs in the HIP kernels of this
// directory.
#include "mm.h"

#include <climits>
#include <cstdlib>
#include <cstring>
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

constexpr int kBand = 64;  // bandwidth of the first tridiagonalisation stage

int64_t eig_ws_elems(int64_t n, int nb) {
  int64_t w = std::max(sy2sb_ws_elems(n, nb), stedc_ws_elems(n));
  w = std::max(w, apply_q1_ws_elems(n, nb, n));
  w = std::max(w, potrf_ws_elems(n));
  w = std::max(w, trtri_ws_elems(n));
  return w;
}

}  // namespace

struct mm_ctx {
  hipStream_t stream = nullptr;
  int64_t n = 0, m = 0, n0 = 0;
  int n_src = 0, n_probe = 0, nf = 0;
  double h = 0.0;
  int64_t r_nnz = 0, band = 0;
  Dev xyz, r_rowptr, r_col, r_val, M0, P;
  Dev status;  // [0] potrf pivot (INT64_MAX = fine), [1] eigensolver status
  // modal method
  bool decomposed = false;
  Dev G, Q, lam, Wm, Pm, y;
  // Cholesky method
  bool factored = false;
  double f_theta = 0.0, f_dt = 0.0;
  Dev Z, Dinv, DinvT, I, b, yv, kstep;
  bool use_graph = true;  // MM_NO_GRAPH=1 in the environment turns graphs off
  // probe partial sums of one step call
  Dev pp;
  Dev tmp;
  std::string err;

  Csr R() const {
    Csr c;
    c.rows = n; c.cols = n; c.nnz = r_nnz;
    c.rowptr = r_rowptr.as<int64_t>();
    c.col = r_col.as<int32_t>();
    c.val = r_val.d();
    return c;
  }
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
  MM_REQUIRE(dt > 0.0, kInvalid, "dt must be positive");
  MM_REQUIRE(n_steps >= 0, kInvalid, "n_steps must be >= 0");
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
    MM_REQUIRE(pb->h > 0.0, kInvalid, "h must be positive");
    MM_REQUIRE(pb->xyz && pb->r_rowptr && pb->r_col && pb->r_val, kInvalid,
               "xyz and R are required");
    MM_REQUIRE(pb->n_probe >= 1 && pb->n_probe <= 8 && pb->P, kInvalid,
               "1..8 probe rows are required");
    MM_REQUIRE(pb->n_src >= 0 && pb->n_src <= 8 && (pb->n_src == 0 || pb->M0), kInvalid,
               "0..8 sources");
    MM_REQUIRE(pb->n_e == 0 || pb->n_e >= 2, kInvalid, "Ne must be 0 or >= 2");
    MM_REQUIRE(pb->n_e == 0, kInvalid, "electrodes are not supported by this build yet");
    c->stream = (hipStream_t)stream;
    hipStream_t s = c->stream;
    const char* ng = std::getenv("MM_NO_GRAPH");
    c->use_graph = !(ng && ng[0] == '1');
    c->n = pb->n;
    c->m = pb->n_e > 0 ? pb->n_e - 1 : 0;
    c->n0 = c->n - c->m;
    c->n_src = pb->n_src;
    c->n_probe = pb->n_probe;
    c->nf = 2 * (int)c->m + c->n_src;
    MM_REQUIRE(c->nf <= 8, kInvalid, "too many forcing terms (2(Ne-1) + n_src <= 8)");
    c->h = pb->h;
    c->r_nnz = pb->r_nnz;
    copy_in(c->xyz, pb->xyz, sizeof(double) * 3 * c->n, s);
    copy_in(c->r_rowptr, pb->r_rowptr, sizeof(int64_t) * (c->n + 1), s);
    copy_in(c->r_col, pb->r_col, sizeof(int32_t) * std::max<int64_t>(1, c->r_nnz), s);
    copy_in(c->r_val, pb->r_val, sizeof(double) * std::max<int64_t>(1, c->r_nnz), s);
    copy_in(c->M0, pb->M0, sizeof(double) * c->n * c->n_src, s);
    copy_in(c->P, pb->P, sizeof(double) * c->n * c->n_probe, s);
    c->status.alloc(4 * sizeof(int64_t));
    csr_lower_band(c->R(), c->status.as<int64_t>() + 2, s);
    MM_HIP_TRY(hipMemcpyAsync(&c->band, c->status.as<int64_t>() + 2, sizeof(int64_t),
                              hipMemcpyDeviceToHost, s));
    MM_HIP_TRY(hipStreamSynchronize(s));
  });
  if (st != MM_OK) {
    delete c;
    return st;
  }
  *out = c;
  return MM_OK;
}

mm_status mm_decompose(mm_ctx* c) {
  if (!c) return MM_E_INVALID;
  return guarded(c, [&] {
    hipStream_t s = c->stream;
    const int64_t n0 = c->n0;
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kBand, n0 - 1));
    c->decomposed = false;
    c->G.alloc(sizeof(double) * n0 * n0);
    c->Q.alloc(sizeof(double) * n0 * n0);
    c->lam.alloc(sizeof(double) * n0);
    c->Wm.alloc(sizeof(double) * n0 * std::max(1, c->nf));
    c->Pm.alloc(sizeof(double) * n0 * c->n_probe);
    c->y.alloc(sizeof(double) * n0);
    Dev Cb, ws, GF, GP;
    Cb.alloc(sizeof(double) * n0 * n0);
    double* G = c->G.d();
    double* Q = c->Q.d();
    double* C = Cb.d();
    int64_t* st = c->status.as<int64_t>();
    // a0: L (lower triangle);  a2: Li = G G^T  (Ne = 0: Li = L)
    assemble_L(c->xyz.d(), c->h, c->n, G, n0, false, s);
    factor_checked(G, n0, st, ws, s, "L");
    // a3: C = G^{-1} R G^{-T}:  G <- G^{-1};  W = G^{-1} R (in Q);  C = G^{-1} W^T
    const int64_t wse = eig_ws_elems(n0, nb);
    ws.alloc(sizeof(double) * wse);
    trtri_lower(G, n0, n0, ws.d(), wse, s);
    dense_times_csr(G, n0, c->R(), Q, n0, s);
    {
      Gemm g;
      g.m = n0; g.n = n0; g.k = n0;
      g.A = G; g.lda = n0; g.a_lower = true;
      g.B = Q; g.ldb = n0; g.tb = true; g.b_band = c->band;
      g.C = C; g.ldc = n0;
      g.lower = true;
      gemm(g, s);
    }
    symmetrize_from_lower(C, n0, n0, s);
    // G^{-1} applied to the forcing vectors and the probe rows (Ne = 0: F = M0)
    GF.alloc(sizeof(double) * n0 * std::max(1, c->nf));
    GP.alloc(sizeof(double) * n0 * c->n_probe);
    if (c->nf > 0) {
      Gemm g;
      g.m = n0; g.n = c->nf; g.k = n0;
      g.A = G; g.lda = n0; g.a_lower = true;
      g.B = c->M0.d(); g.ldb = n0;
      g.C = GF.d(); g.ldc = n0;
      gemm(g, s);
    }
    {
      Gemm g;
      g.m = n0; g.n = c->n_probe; g.k = n0;
      g.A = G; g.lda = n0; g.a_lower = true;
      g.B = c->P.d(); g.ldb = n0;
      g.C = GP.d(); g.ldc = n0;
      gemm(g, s);
    }
    // a4-a7: C = Q Lam Q^T
    Sb2stPlan plan = sb2st_plan(n0, nb);
    Dev tau1, T1, AB, V2, tau2, off, dv, ev;
    const int64_t np = std::max<int64_t>(1, sy2sb_npanels(n0, nb));
    tau1.alloc(sizeof(double) * np * nb);
    T1.alloc(sizeof(double) * np * nb * nb);
    AB.alloc(sizeof(double) * (2 * nb + 1) * n0);
    V2.alloc(sizeof(double) * std::max<int64_t>(1, plan.tasks) * nb);
    tau2.alloc(sizeof(double) * std::max<int64_t>(1, plan.tasks));
    off.alloc(sizeof(int64_t) * (n0 + 1));
    dv.alloc(sizeof(double) * n0);
    ev.alloc(sizeof(double) * std::max<int64_t>(1, n0));
    MM_HIP_TRY(hipMemcpyAsync(off.p, plan.offset.data(), sizeof(int64_t) * (n0 + 1),
                              hipMemcpyHostToDevice, s));
    EigWork w;
    w.nb = nb;
    w.tau1 = tau1.d(); w.T1 = T1.d(); w.AB = AB.d(); w.V2 = V2.d(); w.tau2 = tau2.d();
    w.d_offset = off.as<int64_t>(); w.d = dv.d(); w.e = ev.d();
    w.ws = ws.d(); w.ws_elems = wse;
    fill_i64(st + 1, 1, 0, s);
    syevd(C, n0, n0, c->lam.d(), Q, n0, w, plan, st + 1, s);
    // a8: modal weights  W = Q^T G^{-1} F,  Pt = Q^T G^{-1} P
    if (c->nf > 0) {
      Gemm g;
      g.m = n0; g.n = c->nf; g.k = n0;
      g.A = Q; g.lda = n0; g.ta = true;
      g.B = GF.d(); g.ldb = n0;
      g.C = c->Wm.d(); g.ldc = n0;
      gemm(g, s);
    }
    {
      Gemm g;
      g.m = n0; g.n = c->n_probe; g.k = n0;
      g.A = Q; g.lda = n0; g.ta = true;
      g.B = GP.d(); g.ldb = n0;
      g.C = c->Pm.d(); g.ldc = n0;
      gemm(g, s);
    }
    fill(c->y.d(), n0, 0.0, s);
    int64_t est = 0;
    MM_HIP_TRY(hipMemcpyAsync(&est, st + 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    MM_HIP_TRY(hipStreamSynchronize(s));
    MM_HIP_TRY(hipGetLastError());
    if (est != 0) throw Error{kNoConverge, "a secular equation did not converge"};
    c->decomposed = true;
  });
}

mm_status mm_step_modal(mm_ctx* c, double theta, double dt, int64_t n_steps,
                        const double* i_src, const double* i_D, double* signal) {
  if (!c) return MM_E_INVALID;
  return guarded(c, [&] {
    MM_REQUIRE(c->decomposed, kState, "mm_step_modal before mm_decompose");
    check_steps(theta, dt, n_steps);
    MM_REQUIRE(c->n_src == 0 || i_src, kInvalid, "i_src is required");
    MM_REQUIRE(c->m == 0 || i_D, kInvalid, "i_D is required");
    MM_REQUIRE(signal || n_steps == 0, kInvalid, "signal is required");
    if (n_steps == 0) return;
    hipStream_t s = c->stream;
    const int G = modal_groups(c->n0);
    c->pp.alloc(sizeof(double) * n_steps * G * c->n_probe);
    ModalStep ms;
    ms.n0 = c->n0;
    ms.lam = c->lam.d();
    ms.W = c->Wm.d();
    ms.f.nf = c->nf; ms.f.m = (int)c->m; ms.f.n_src = c->n_src;
    ms.f.i_src = i_src; ms.f.i_D = i_D;
    ms.Pt = c->Pm.d();
    ms.n_probe = c->n_probe;
    ms.theta = theta; ms.dt = dt;
    ms.y = c->y.d();
    ms.probe_partial = c->pp.d();
    modal_steps(ms, 0, n_steps, s);
    probe_finish(c->pp.d(), n_steps, G, c->n_probe, nullptr, 0, i_D, 0, dt, signal, s);
  });
}

mm_status mm_step_cholesky(mm_ctx* c, double theta, double dt, int64_t n_steps,
                           const double* i_src, const double* i_D, double* signal) {
  if (!c) return MM_E_INVALID;
  return guarded(c, [&] {
    check_steps(theta, dt, n_steps);
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
      c->kstep.alloc(sizeof(int64_t));
      // b0: Z = Li + theta dt Ri = C C^T   (Ne = 0: Li = L, Ri = R)
      double* Z = c->Z.d();
      assemble_L(c->xyz.d(), c->h, c->n, Z, n0, false, s);
      add_csr_lower(Z, n0, theta * dt, c->R(), s);
      factor_checked(Z, n0, c->status.as<int64_t>(), c->tmp, s, "Li + theta dt Ri");
      c->tmp.alloc(sizeof(double) * trtri_ws_elems(B));
      diag_block_inverses(Z, n0, n0, B, c->Dinv.d(), c->tmp.d(), trtri_ws_elems(B), s);
      transpose_blocks(c->Dinv.d(), NB, B, c->DinvT.d(), s);
      MM_HIP_TRY(hipStreamSynchronize(s));
      c->tmp.release();
      c->factored = true;
      c->f_theta = theta;
      c->f_dt = dt;
    }
    if (n_steps == 0) return;
    const int64_t parts = trsv_parts(n0);
    c->pp.alloc(sizeof(double) * n_steps * parts * c->n_probe);
    CholStep cs;
    cs.n0 = n0;
    cs.Cf = c->Z.d(); cs.ld = n0;
    cs.B = B;
    cs.Dinv = c->Dinv.d();
    cs.DinvT = c->DinvT.d();
    cs.kstep = c->kstep.as<int64_t>();
    cs.use_graph = c->use_graph;
    cs.Ri = c->R();
    cs.f.F = c->M0.d(); cs.f.nf = c->nf; cs.f.m = (int)c->m; cs.f.n_src = c->n_src;
    cs.f.i_src = i_src; cs.f.i_D = i_D;
    cs.theta = theta; cs.dt = dt;
    cs.I = c->I.d(); cs.b = c->b.d(); cs.y = c->yv.d();
    cs.Pt = c->P.d(); cs.n_probe = c->n_probe;
    cs.probe_partial = c->pp.d();
    chol_steps(cs, 0, n_steps, s);
    probe_finish(c->pp.d(), n_steps, parts, c->n_probe, nullptr, 0, i_D, 0, dt, signal, s);
  });
}

mm_status mm_probe(mm_ctx* c, int32_t which, int32_t n_rows, const double* rows, double* out) {
  if (!c) return MM_E_INVALID;
  return guarded(c, [&] {
    MM_REQUIRE(out != nullptr, kInvalid, "out is NULL");
    MM_REQUIRE(which == MM_MODAL || which == MM_CHOLESKY, kInvalid, "which");
    MM_REQUIRE(rows == nullptr || n_rows >= 1, kInvalid, "n_rows");
    hipStream_t s = c->stream;
    const int64_t n0 = c->n0;
    Dev buf;
    buf.alloc(sizeof(double) * 2 * n0);
    double* Ifull = buf.d();
    if (which == MM_MODAL) {
      MM_REQUIRE(c->decomposed, kState, "mm_probe(MM_MODAL) before mm_decompose");
      double* t = buf.d() + n0;
      // a11: Ii = G^{-T} (Q y)
      Gemm g1;
      g1.m = n0; g1.n = 1; g1.k = n0;
      g1.A = c->Q.d(); g1.lda = n0;
      g1.B = c->y.d(); g1.ldb = n0;
      g1.C = t; g1.ldc = n0;
      gemm(g1, s);
      Gemm g2;
      g2.m = n0; g2.n = 1; g2.k = n0;
      g2.A = c->G.d(); g2.lda = n0; g2.ta = true; g2.a_upper = true;
      g2.B = t; g2.ldb = n0;
      g2.C = Ifull; g2.ldc = n0;
      gemm(g2, s);
    } else {
      MM_REQUIRE(c->I.p != nullptr, kState, "mm_probe(MM_CHOLESKY) before any Cholesky step");
      MM_HIP_TRY(hipMemcpyAsync(Ifull, c->I.p, sizeof(double) * n0, hipMemcpyDeviceToDevice, s));
    }
    if (!rows) {
      MM_HIP_TRY(hipMemcpyAsync(out, Ifull, sizeof(double) * c->n, hipMemcpyDeviceToDevice, s));
    } else {
      Gemm g;
      g.m = n_rows; g.n = 1; g.k = c->n;
      g.A = rows; g.lda = c->n; g.ta = true;
      g.B = Ifull; g.ldb = c->n;
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
    if (c->I.p) fill(c->I.d(), c->n0, 0.0, c->stream);
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
    Dev ws, st;
    ws.alloc(sizeof(double) * stedc_ws_elems(n));
    st.alloc(sizeof(int64_t));
    fill_i64(st.as<int64_t>(), 1, 0, s);
    stedc(d, e, n, w, Z, n, ws.d(), stedc_ws_elems(n), st.as<int64_t>(), s);
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
