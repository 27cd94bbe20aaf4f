// Kernel-level entry points (include/tt_kernels.h).
#include <string.h>

#include <mutex>
#include <string>

#include "../../include/tt_kernels.h"
#include "tt_internal.h"

using namespace tt;

namespace {
thread_local std::string k_err;
tt_status kfail(tt_status s, const std::string& m) {
  k_err = m;
  return s;
}
#define KCHK(call)                                                                   \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess) return kfail(TT_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// ---- device scratch of tt_kernel_gram_noalloc --------------------------------
// One array per GPU, owned by the library for the life of the process.  In
// host code `noalloc_scratch` names a host-side stand-in; its device address
// is taken once per device with hipGetSymbolAddress and used from then on.
constexpr size_t NOALLOC_BYTES = (size_t)32 << 20;
static __device__ __align__(256) char noalloc_scratch[NOALLOC_BYTES];
constexpr int NOALLOC_MAX_DEV = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[NOALLOC_MAX_DEV] = {};

// The device address of the scratch array on the current device (taken on
// the first call on that device).
hipError_t noalloc_scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= NOALLOC_MAX_DEV) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
    if (e != hipSuccess) return e;
    g_noalloc_ptr[dev] = p;
  }
  *out = g_noalloc_ptr[dev];
  return hipSuccess;
}

// dims table of a kernel-level call: all zero but dims[0] = n (a kernel, so
// the call issues no memset or host copy into the scratch).
__global__ void k_noalloc_dims(int* __restrict__ dims, int n) {
  if (threadIdx.x < 64) dims[threadIdx.x] = threadIdx.x == 0 ? n : 0;
}
}  // namespace

namespace tt {
void kernel_error(const std::string& m) { k_err = m; }
}  // namespace tt

extern "C" {

const char* tt_kernel_last_error(void) { return k_err.c_str(); }

tt_status tt_kernel_lds_check(int32_t n, int32_t ncap2, int32_t pcap, size_t* max_bytes) {
  if (n < 0 || ncap2 < 0 || pcap < 0) return kfail(TT_ERR_INVALID_ARG, "negative size");
  const char *w1 = "", *w2 = "";
  const size_t a = n > 0 ? eig_lds_bytes(n, false, &w1) : 0;
  const size_t b = ncap2 > 0 ? svd_lds_bytes(ncap2, pcap, false, &w2) : 0;
  if (max_bytes) *max_bytes = a > b ? a : b;
  if (!lds_fits(a) || !lds_fits(b))
    return kfail(TT_ERR_INVALID_ARG, std::string("LDS above 160 KiB in ") + (lds_fits(a) ? w2 : w1));
  return TT_OK;
}

size_t tt_kernel_eigh_workspace(int32_t n) {
  if (n < 1 || n > 1024) return 0;
  return align256(64 * sizeof(int)) + align256((size_t)n * n * 8) + align256((size_t)n * 8) * 2 +
         align256(eig_work_doubles(n) * 8);
}

tt_status tt_kernel_eigh(const double* A, int32_t n, int32_t lda, double clip, double* lam,
                         double* V, int32_t ldv, int32_t* kept, void* ws, size_t ws_bytes,
                         void* stream) {
  if (!A || !lam || !V || !ws || n < 1 || n > 1024 || lda < n || ldv < n)
    return kfail(TT_ERR_INVALID_ARG, "bad eigh arguments");
  if (ws_bytes < tt_kernel_eigh_workspace(n)) return kfail(TT_ERR_OOM, "workspace too small");
  {
    const char* which = "";
    const size_t lds = eig_lds_bytes(n, true, &which);
    if (!lds_fits(lds))
      return kfail(TT_ERR_INVALID_ARG, std::string("LDS above 160 KiB in ") + which);
  }
  hipStream_t s = (hipStream_t)stream;
  char* p = (char*)ws;
  int* dims = (int*)p;
  p += align256(64 * sizeof(int));
  double* Acopy = (double*)p;
  p += align256((size_t)n * n * 8);
  double* sq = (double*)p;
  p += align256((size_t)n * 8);
  double* isq = (double*)p;
  p += align256((size_t)n * 8);
  double* work = (double*)p;
  int hd[64];
  memset(hd, 0, sizeof(hd));
  hd[0] = n;
  KCHK(hipMemcpyAsync(dims, hd, sizeof(hd), hipMemcpyHostToDevice, s));
  KCHK(hipMemcpy2DAsync(Acopy, n * 8, A, lda * 8, n * 8, n, hipMemcpyDeviceToDevice, s));
  KCHK(hipMemsetAsync(work, 0, eig_work_doubles(n) * 8, s));
  EigJob j{Acopy, n, 0, lam, V, ldv, sq, isq, 1, clip, work};
  eig_batched(&j, 1, n, dims, s);
  KCHK(hipGetLastError());
  KCHK(hipMemcpyAsync(hd, dims, sizeof(hd), hipMemcpyDeviceToHost, s));
  KCHK(hipStreamSynchronize(s));
  if (kept) *kept = hd[1];
  if (hd[D_FLAG]) return kfail(TT_ERR_NUMERIC, "eigensolver flagged a failure");
  return TT_OK;
}

size_t tt_kernel_svd_workspace(int32_t a, int32_t b) {
  const int q = a < b ? a : b, p = a < b ? b : a;
  if (a < 1 || b < 1 || q > 1024 || p > 1024) return 0;
  const int N = 2 * q;
  return align256(64 * sizeof(int)) + align256((size_t)p * q * 8) + align256((size_t)q * 8) * 2 +
         align256(eig_work_doubles(N) * 8);
}

tt_status tt_kernel_svd(const double* M, int32_t a, int32_t b, int32_t ldm, double* sig, double* V,
                        int32_t ldv, int32_t* kept, void* ws, size_t ws_bytes, void* stream) {
  const int q = a < b ? a : b, p = a < b ? b : a;
  if (!M || !sig || !V || !ws || a < 1 || b < 1 || q > 1024 || p > 1024 || ldm < b || ldv < q)
    return kfail(TT_ERR_INVALID_ARG, "bad svd arguments");
  if (ws_bytes < tt_kernel_svd_workspace(a, b)) return kfail(TT_ERR_OOM, "workspace too small");
  {
    const char* which = "";
    const size_t lds = svd_lds_bytes(2 * q, p, true, &which);
    if (!lds_fits(lds))
      return kfail(TT_ERR_INVALID_ARG, std::string("LDS above 160 KiB in ") + which);
  }
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  int* dims = (int*)w;
  w += align256(64 * sizeof(int));
  double* Awork = (double*)w;
  w += align256((size_t)p * q * 8);
  double* sq = (double*)w;
  w += align256((size_t)q * 8);
  double* isq = (double*)w;
  w += align256((size_t)q * 8);
  double* work = (double*)w;
  const int N = 2 * q;
  int hd[64];
  memset(hd, 0, sizeof(hd));
  hd[0] = a;
  hd[1] = b;
  hd[2] = a <= b ? 0 : 1;
  KCHK(hipMemcpyAsync(dims, hd, sizeof(hd), hipMemcpyHostToDevice, s));
  KCHK(hipMemsetAsync(work, 0, eig_work_doubles(N) * 8, s));
  EigJob j{Awork, q, 3, sig, V, ldv, sq, isq, 4, 1.0, work};
  svd_short_side(M, ldm, 0, 1, 2, j, N, p, dims, s);
  KCHK(hipGetLastError());
  KCHK(hipMemcpyAsync(hd, dims, sizeof(hd), hipMemcpyDeviceToHost, s));
  KCHK(hipStreamSynchronize(s));
  if (kept) *kept = hd[4];
  if (hd[D_FLAG]) return kfail(TT_ERR_NUMERIC, "singular value solver flagged a failure");
  return TT_OK;
}

size_t tt_kernel_gram_workspace(int32_t K, int32_t n, int32_t lda) {
  if (K < 1 || n < 1 || lda < n) return 0;
  return align256(64 * sizeof(int)) + align256(gram_partial_doubles(gram_plan(K, n, lda)) * 8);
}

tt_status tt_kernel_gram(const double* A, int32_t K, int32_t n, int32_t lda, double* G,
                         int32_t ldg, void* ws, size_t ws_bytes, void* stream) {
  if (!A || !G || !ws || K < 1 || n < 1 || lda < n || ldg < n)
    return kfail(TT_ERR_INVALID_ARG, "bad gram arguments");
  if (ws_bytes < tt_kernel_gram_workspace(K, n, lda)) return kfail(TT_ERR_OOM, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  int* dims = (int*)ws;
  double* part = (double*)((char*)ws + align256(64 * sizeof(int)));
  int hd[64];
  memset(hd, 0, sizeof(hd));
  hd[0] = n;
  KCHK(hipMemcpyAsync(dims, hd, sizeof(hd), hipMemcpyHostToDevice, s));
  gram_tall(gram_plan(K, n, lda), A, dimv(0), part, G, ldg, dims, s);
  KCHK(hipGetLastError());
  KCHK(hipStreamSynchronize(s));
  return TT_OK;
}

tt_status tt_kernel_gram_noalloc(const double* A, int32_t K, int32_t n, int32_t lda, double* G,
                                 int32_t ldg, void* stream) {
  if (!A || !G || K < 1 || n < 1 || lda < n || ldg < n)
    return kfail(TT_ERR_INVALID_ARG, "bad gram arguments");
  const GramPlan plan = gram_plan(K, n, lda);
  const size_t need = align256(64 * sizeof(int)) + align256(gram_partial_doubles(plan) * 8);
  if (need > NOALLOC_BYTES)
    return kfail(TT_ERR_INVALID_ARG, "gram_noalloc: the partial tiles need " + std::to_string(need) +
                                         " bytes, above the " + std::to_string(NOALLOC_BYTES) +
                                         "-byte device scratch (use tt_kernel_gram)");
  void* base = nullptr;
  KCHK(noalloc_scratch_ptr(&base));
  hipStream_t s = (hipStream_t)stream;
  int* dims = (int*)base;
  double* part = (double*)((char*)base + align256(64 * sizeof(int)));
  k_noalloc_dims<<<1, 64, 0, s>>>(dims, n);
  gram_tall(plan, A, dimv(0), part, G, ldg, dims, s);
  KCHK(hipGetLastError());
  KCHK(hipStreamSynchronize(s));
  return TT_OK;
}

size_t tt_kernel_gram_f32_workspace(int32_t K, int32_t n, int32_t lda) {
  if (K < 1 || n < 1 || n > 1024 || lda < n) return 0;
  return align256(64 * sizeof(int)) + align256(gram_partial_doubles(gram_plan(K, n, lda)) * 8) +
         align256(((size_t)n + 64) * sizeof(unsigned));
}

tt_status tt_kernel_gram_f32(const float* A, int32_t K, int32_t n, int32_t lda, double* G,
                             int32_t ldg, void* ws, size_t ws_bytes, void* stream) {
  if (!A || !G || !ws || K < 1 || n < 1 || n > 1024 || lda < n || ldg < n)
    return kfail(TT_ERR_INVALID_ARG, "bad gram_f32 arguments");
  if (ws_bytes < tt_kernel_gram_f32_workspace(K, n, lda)) return kfail(TT_ERR_OOM, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  const GramPlan plan = gram_plan(K, n, lda);
  char* p = (char*)ws;
  int* dims = (int*)p;
  p += align256(64 * sizeof(int));
  double* part = (double*)p;
  p += align256(gram_partial_doubles(plan) * 8);
  unsigned* colmax = (unsigned*)p;
  int hd[64];
  memset(hd, 0, sizeof(hd));
  hd[0] = n;
  KCHK(hipMemcpyAsync(dims, hd, sizeof(hd), hipMemcpyHostToDevice, s));
  gram_split_partial(plan, A, dimv(0), colmax, part, dims, s);
  gram_split_reduce(plan, dimv(0), part, G, ldg, dims, s);
  KCHK(hipGetLastError());
  KCHK(hipStreamSynchronize(s));
  return TT_OK;
}

size_t tt_kernel_gemm_tall_workspace(void) { return align256(64 * sizeof(int)); }

tt_status tt_kernel_gemm_tall(const double* A, int32_t K, int32_t k, int32_t lda, const double* B,
                              int32_t n, int32_t ldb, double* C, int32_t ldc, void* ws,
                              size_t ws_bytes, void* stream) {
  if (!A || !B || !C || !ws || K < 1 || k < 0 || n < 1 || lda < k || ldb < n || ldc < n)
    return kfail(TT_ERR_INVALID_ARG, "bad gemm_tall arguments");
  if (ws_bytes < tt_kernel_gemm_tall_workspace()) return kfail(TT_ERR_OOM, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  int* dims = (int*)ws;
  int hd[64];
  memset(hd, 0, sizeof(hd));
  hd[0] = k;
  hd[1] = n;
  KCHK(hipMemcpyAsync(dims, hd, sizeof(hd), hipMemcpyHostToDevice, s));
  gemm_tall(K, A, lda, B, ldb, C, ldc, dimv(0), dimv(1), k, n, dims, s);
  KCHK(hipGetLastError());
  KCHK(hipStreamSynchronize(s));
  return TT_OK;
}

tt_status tt_kernel_gemm(const double* A, int32_t lda, int32_t ta, const double* B, int32_t ldb,
                         int32_t tb, double* C, int32_t ldc, int32_t m, int32_t n, int32_t k,
                         void* ws, size_t ws_bytes, void* stream) {
  if (!A || !B || !C || !ws || m < 1 || n < 1 || k < 0) return kfail(TT_ERR_INVALID_ARG, "bad gemm arguments");
  if (ws_bytes < tt_kernel_gemm_tall_workspace()) return kfail(TT_ERR_OOM, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  int* dims = (int*)ws;
  int hd[64];
  memset(hd, 0, sizeof(hd));
  hd[0] = m;
  hd[1] = n;
  hd[2] = k;
  KCHK(hipMemcpyAsync(dims, hd, sizeof(hd), hipMemcpyHostToDevice, s));
  GemmDesc g;
  memset(&g, 0, sizeof(g));
  g.A = A; g.B = B; g.C = C; g.lda = lda; g.ldb = ldb; g.ldc = ldc;
  g.transA = ta; g.transB = tb;
  g.m = dimv(0); g.n = dimv(1); g.k = dimv(2);
  g.alpha = 1.0;
  g.cond_idx = -1;
  g.bclip_idx = -1;
  gemm(g, m, n, 1, dims, s);
  KCHK(hipGetLastError());
  KCHK(hipStreamSynchronize(s));
  return TT_OK;
}

}  // extern "C"
