// Internal definitions shared by the HIP sources of libmm (gfx950, FP64).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

namespace mm {

typedef double v4d __attribute__((ext_vector_type(4)));

// Status codes mirror include/mm.h.
enum : int {
  kOk = 0,
  kInvalid = 1,
  kNoMem = 2,
  kNotSpd = 3,
  kNoConverge = 4,
  kState = 5,
  kDevice = 6,
};

struct Error {
  int code;
  std::string msg;
};

#define MM_HIP_TRY(expr)                                                     \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess)                                                    \
      throw ::mm::Error{::mm::kDevice, std::string(#expr) + ": " +           \
                                           hipGetErrorString(e_)};           \
  } while (0)

#define MM_REQUIRE(cond, code, text)                                         \
  do {                                                                       \
    if (!(cond)) throw ::mm::Error{(code), (text)};                          \
  } while (0)

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// A store written through to the device's point of coherence (relaxed, agent
// scope: a plain vector store with the device-scope cache policy).  For data
// that the next launch of a long chain of small kernels reads, possibly on
// another XCD: the write-back of dirty L2 lines that ends each launch then
// has little left to do.
__device__ __forceinline__ void store_dev(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// GEMM: C = alpha op(A) op(B) + beta C, column-major, FP64 MFMA.
// Options that restrict the work to the non-zero structure:
//   lower    : only C(i,j) with i >= j is computed and written;
//   a_lower  : op(A)(i,k) = 0 for k > i     (k loop ends at the tile's last row)
//   b_band   : op(B)(k,j) = 0 for k > j + b_band   (if b_band >= 0)
//   a_upper  : op(A)(i,k) = 0 for k < i     (k loop starts at the tile's first row)
//   b_lower  : op(B)(k,j) = 0 for k < j     (k loop starts at the tile's first col)
// The zero parts named by these options must hold zeros in memory.
// ---------------------------------------------------------------------------
struct Gemm {
  int64_t m = 0, n = 0, k = 0;
  double alpha = 1.0, beta = 0.0;
  const double* A = nullptr;
  int64_t lda = 1;
  bool ta = false;
  const double* B = nullptr;
  int64_t ldb = 1;
  bool tb = false;
  double* C = nullptr;
  int64_t ldc = 1;
  bool lower = false;
  bool a_lower = false;
  bool a_upper = false;
  bool b_lower = false;
  int64_t b_band = -1;
  // op(A) symmetric with only its lower triangle stored: element (i, k) is
  // read from A(max(i, k), min(i, k)).  Not with ta or the other A flags.
  bool a_sym = false;
  int64_t batch = 1;
  int64_t sA = 0, sB = 0, sC = 0;  // batch strides (elements)
};

// One problem of a grouped GEMM whose sizes live in device memory.
struct GemmGroup {
  const double* A;
  const double* B;
  double* C;
  int64_t m, n, k;
  int64_t lda, ldb, ldc;
};

// Launch one GEMM on `stream`.  `ws` (ws_elems doubles) enables split-K for
// tall, narrow outputs with a long k; pass nullptr to disable it.
void gemm(const Gemm& g, hipStream_t stream, double* ws = nullptr,
          int64_t ws_elems = 0);

// Grouped GEMM: C_g = alpha op(A_g) op(B_g) + beta C_g for g < n_groups with
// the descriptors in device memory; max_m, max_n bound every group's m, n.
void gemm_grouped(const GemmGroup* d_groups, int64_t n_groups, int64_t max_m,
                  int64_t max_n, bool ta, bool tb, double alpha, double beta,
                  hipStream_t stream);

}  // namespace mm
